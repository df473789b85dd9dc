"""Pins for the oracle's state-vector simulator: the brute-force unitary
(independent code), a hand-derived two-qubit example, product states, the
empty circuit and norm preservation."""
import math

import numpy as np
import pytest

import oracle
from rqcgen import Circuit, Gate, make_rqc


@pytest.mark.parametrize("rows,cols,d,seed", [(2, 3, 6, 0), (2, 4, 8, 1), (3, 3, 5, 2), (1, 4, 9, 3)])
def test_statevector_matches_bruteforce_unitary(rows, cols, d, seed):
    c = make_rqc(rows, cols, d, seed)
    psi = oracle.statevector(c).reshape(-1)
    u = oracle.circuit_unitary(c)
    np.testing.assert_allclose(psi, u[:, 0], atol=1e-12)
    np.testing.assert_allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-12)


def test_reversed_and_distant_qubit_pairs():
    rng = np.random.default_rng(0)
    gates = [Gate("sqrt_x", (0,)), Gate("sqrt_w", (2,)), Gate("sqrt_y", (4,)),
             Gate("fsim", (4, 1), (0.7, 0.3)), Gate("fsim", (3, 0), (1.2, -0.5)),
             Gate("fsim", (0, 4), (0.4, 2.0)), Gate("sqrt_y", (1,))]
    c = Circuit(5, gates)
    psi = oracle.statevector(c).reshape(-1)
    u = oracle.circuit_unitary(c)
    np.testing.assert_allclose(psi, u[:, 0], atol=1e-13)
    del rng


def test_hand_derived_two_qubit_example():
    # sqrt(X) on qubit 0: (|00> - i|10>)/sqrt2; fSim(pi/2, 0) sends |10> to
    # -i|01>: result (|00> - |01>)/sqrt2 with qubit 0 most significant.
    c = Circuit(2, [Gate("sqrt_x", (0,)), Gate("fsim", (0, 1), (math.pi / 2, 0.0))])
    psi = oracle.statevector(c).reshape(-1)
    np.testing.assert_allclose(psi, np.array([1, -1, 0, 0]) / math.sqrt(2), atol=1e-15)


def test_product_state_closed_form():
    c = make_rqc(2, 3, 7, seed=9, two_qubit=False)
    psi = oracle.statevector(c).reshape(-1)
    vec = np.array([1.0 + 0j])
    for q in range(c.n_qubits):
        v = np.array([1, 0], dtype=complex)
        for g in c.gates:
            if g.qubits == (q,):
                v = oracle.gate_matrix(g.name) @ v
        vec = np.kron(vec, v)
    np.testing.assert_allclose(psi, vec, atol=1e-14)


def test_empty_circuit_is_delta():
    c = Circuit(6, [])
    psi = oracle.statevector(c).reshape(-1)
    e = np.zeros(64, dtype=complex)
    e[0] = 1
    np.testing.assert_array_equal(psi, e)


def test_norm_preserved_20_qubits():
    c = make_rqc(4, 5, 8, seed=0)
    psi = oracle.statevector(c)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


def test_bunch_indexing():
    c = make_rqc(2, 3, 6, seed=4)
    psi = oracle.statevector(c).reshape(-1)
    bits = [1, 0, 1, 1, 0, 1]
    open_q = [1, 4]
    a = oracle.amplitudes_sv(c, open_q, bits)
    for y in range(4):
        x = list(bits)
        x[1], x[4] = (y >> 1) & 1, y & 1
        idx = int("".join(map(str, x)), 2)
        assert a[y] == psi[idx]
