"""Schroedinger state-vector simulation in FP64 (main text, TNC section,
first paragraph: an n-qubit state is a rank-n tensor; applying a gate contracts
the gate tensor with the state's indices; time O(m 2^n), memory O(2^n)).

The state is a numpy array of shape (2,)*n, axis j = qubit j, so the flat
C-order index is sum_j x_j 2^(n-1-j).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .gates import gate_matrix


def apply_gate(psi: np.ndarray, mat: np.ndarray, qubits: Sequence[int]) -> np.ndarray:
    """Contract a k-qubit gate (2^k x 2^k, rows = outputs) into the state."""
    k = len(qubits)
    g = np.asarray(mat, dtype=np.complex128).reshape((2,) * (2 * k))
    # g axes: outputs 0..k-1, inputs k..2k-1; contract inputs with the state axes
    out = np.tensordot(g, psi, axes=(list(range(k, 2 * k)), list(qubits)))
    # out axes: gate outputs, then the remaining state axes in order
    rest = [q for q in range(psi.ndim) if q not in qubits]
    src = list(qubits) + rest
    return np.moveaxis(out, list(range(psi.ndim)), src)


def statevector(circuit) -> np.ndarray:
    """U|0^n> for the circuit's gate list (names/params/qubits only)."""
    n = circuit.n_qubits
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    for g in circuit.gates:
        psi = apply_gate(psi, gate_matrix(g.name, g.params), g.qubits)
    return psi


def amplitudes_sv(circuit, open_qubits: Sequence[int], closed_bits: Sequence[int],
                  psi: np.ndarray = None) -> np.ndarray:
    """Bunch a[y] = <x_C, y_O| U |0^n>, y indexed by sum_j y_j 2^(|O|-1-j)
    over the open qubits in increasing order; closed_bits[q] is read for the
    closed qubits only."""
    if psi is None:
        psi = statevector(circuit)
    n = circuit.n_qubits
    open_set = sorted(set(open_qubits))
    idx = []
    for q in range(n):
        idx.append(slice(None) if q in open_set else int(closed_bits[q]))
    return np.asarray(psi[tuple(idx)]).reshape(-1).copy()
