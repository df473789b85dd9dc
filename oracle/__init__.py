"""CPU FP64 oracle for random-circuit amplitudes (test infrastructure only).

Plain, slow, obviously correct reference implementations, written from the
paper, used ONLY by the test-suite, the package smoke check and the benchmark's
CPU-baseline leg.  The GPU contraction library never imports, links or calls
anything here, and nothing here imports the library.

What it computes, per the paper:

* gate matrices (Supplement, "Random quantum circuits": sqrt(X), sqrt(Y),
  sqrt(W) and the fSim gate);
* amplitudes <x|U|0^n> by the Schroedinger state-vector method (main text,
  section on the customized TNC algorithm, first paragraph);
* a brute-force 2^n x 2^n circuit unitary for tiny n (a second, independent
  path that pins the state vector);
* the amplitude as the contraction of the circuit's tensor network with index
  slicing (main text TNC section; Supplement "Tensor network contraction
  algorithm"), pairwise contractions as in the Supplement's Eq. (matmul);
* XEB fidelity and the Porter-Thomas density of the Eq. (fxeb) family, and the
  per-amplitude relative error of Table II.

Inputs (circuits, orders, sliced wires) come from the seeded generators in
``rqcgen``; the oracle reads only gate names, qubits and parameters, and builds
its own matrices.
"""
from .gates import gate_matrix, sqrt_x, sqrt_y, sqrt_w, fsim
from .statevector import statevector, amplitudes_sv, apply_gate
from .unitary import circuit_unitary
from .tn import build_network, contract_network, contract_sliced, pairwise_contract
from .stats import (xeb_fidelity, porter_thomas_pdf, relative_error_each,
                    relative_error_norm, collision_moment)
