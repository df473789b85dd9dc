"""Brute-force circuit unitary for tiny circuits (independent pin of the
state-vector code).

Each gate is embedded into a full 2^n x 2^n matrix by explicit loops over
basis states (entry <x'|G|x> = g[(x'_q), (x_q)] when every other qubit agrees),
and the unitary is the ordinary matrix product of the embedded gates.
"""
from __future__ import annotations

import numpy as np

from .gates import gate_matrix


def _bit(x: int, q: int, n: int) -> int:
    return (x >> (n - 1 - q)) & 1


def embed(mat: np.ndarray, qubits, n: int) -> np.ndarray:
    dim = 1 << n
    k = len(qubits)
    full = np.zeros((dim, dim), dtype=np.complex128)
    for x in range(dim):
        col = 0
        for q in qubits:
            col = (col << 1) | _bit(x, q, n)
        for row in range(1 << k):
            y = x
            for j, q in enumerate(qubits):
                b = (row >> (k - 1 - j)) & 1
                pos = n - 1 - q
                y = (y & ~(1 << pos)) | (b << pos)
            full[y, x] += mat[row, col]
    return full


def circuit_unitary(circuit) -> np.ndarray:
    n = circuit.n_qubits
    if n > 10:
        raise ValueError("brute-force unitary limited to 10 qubits")
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circuit.gates:
        u = embed(gate_matrix(g.name, g.params), g.qubits, n) @ u
    return u
