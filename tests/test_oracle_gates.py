"""Pins for the oracle's gate matrices: closed forms fixed by the Supplement's
definitions (section "Random quantum circuits")."""
import math

import numpy as np
import pytest

import oracle
from rqcgen import make_rqc, one_qubit_matrix, fsim_matrix

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
W = (X + Y) / math.sqrt(2)


@pytest.mark.parametrize("root,P", [(oracle.sqrt_x, X), (oracle.sqrt_y, Y), (oracle.sqrt_w, W)])
def test_square_roots_square_to_minus_i_pauli(root, P):
    g = root()
    np.testing.assert_allclose(g @ g, -1j * P, atol=1e-15)


@pytest.mark.parametrize("name", ["sqrt_x", "sqrt_y", "sqrt_w"])
def test_one_qubit_unitary(name):
    g = oracle.gate_matrix(name)
    np.testing.assert_allclose(g.conj().T @ g, np.eye(2), atol=1e-15)


@pytest.mark.parametrize("theta,phi", [(math.pi / 2, math.pi / 6), (0.3, 1.1), (1.0, -0.4)])
def test_fsim_unitary(theta, phi):
    f = oracle.fsim(theta, phi)
    np.testing.assert_allclose(f.conj().T @ f, np.eye(4), atol=1e-15)
    f5 = oracle.fsim(theta, phi, 0.2, -0.7, 0.4)
    np.testing.assert_allclose(f5.conj().T @ f5, np.eye(4), atol=1e-14)


def test_fsim_half_pi_action():
    phi = math.pi / 6
    f = oracle.fsim(math.pi / 2, phi)
    e = np.eye(4)
    np.testing.assert_allclose(f @ e[0], e[0], atol=1e-15)             # |00> -> |00>
    np.testing.assert_allclose(f @ e[1], -1j * e[2], atol=1e-15)       # |01> -> -i|10>
    np.testing.assert_allclose(f @ e[2], -1j * e[1], atol=1e-15)       # |10> -> -i|01>
    np.testing.assert_allclose(f @ e[3], np.exp(-1j * phi) * e[3], atol=1e-15)


def test_fsim_symmetric_under_qubit_exchange():
    swap = np.eye(4)[[0, 2, 1, 3]]
    f = oracle.fsim(math.pi / 2, math.pi / 6)
    np.testing.assert_allclose(swap @ f @ swap, f, atol=1e-15)


def test_fsim_zero_angle_is_controlled_phase():
    f = oracle.fsim(0.0, 0.9)
    np.testing.assert_allclose(f, np.diag([1, 1, 1, np.exp(-0.9j)]), atol=1e-15)


def test_generator_matrices_match_oracle():
    """The input generator's matrices (handed to the GPU library) agree with
    the oracle's independent construction."""
    for name in ("sqrt_x", "sqrt_y", "sqrt_w"):
        np.testing.assert_allclose(one_qubit_matrix(name), oracle.gate_matrix(name), atol=0)
    np.testing.assert_allclose(fsim_matrix(math.pi / 2, math.pi / 6),
                               oracle.fsim(math.pi / 2, math.pi / 6), atol=1e-16)
    c = make_rqc(3, 3, 6, seed=5)
    for g in c.gates:
        np.testing.assert_allclose(g.matrix, oracle.gate_matrix(g.name, g.params), atol=1e-16)
