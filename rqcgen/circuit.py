"""Seeded random-quantum-circuit generator (input side only).

Builds the random circuits of the paper's Supplement, section "Random quantum
circuits": interlaced layers of random single-qubit gates drawn from
{sqrt(X), sqrt(Y), sqrt(W)} and fSim two-qubit gates laid out in the four
grid-edge patterns A, B, C, D.

This module holds no part of the contraction arithmetic.  It emits gate names,
qubit lists, parameters and the complex128 gate matrices that a caller hands to
the contraction library.  The CPU oracle rebuilds its own matrices from the
names and parameters and never uses the ones produced here.

Conventions fixed here (the paper leaves them open):

* Sites are (r, c) on a rows x cols grid; qubits are the present sites numbered
  in row-major order, missing sites skipped.
* Edge patterns: A = horizontal (r,c)-(r,c+1) with r+c even, B = horizontal
  with r+c odd, C = vertical (r,c)-(r+1,c) with r+c even, D = vertical with
  r+c odd.  Each pattern is a matching and every grid edge appears exactly once
  per A, B, C, D group.  Edges touching a missing site are dropped.
* The cycle sequence is the periodic string ABCDCDAB truncated to d cycles
  (d = 8 and d = 12 give the two sequences the paper prints).
* One cycle = a single-qubit layer on every qubit, then the two-qubit layer of
  that cycle's pattern; one final single-qubit layer precedes measurement.
  The initial state is |0...0>.
* Single-qubit gates: the first layer draws uniformly from the 3 gates, later
  layers draw uniformly from the 2 gates that differ from the previous one on
  the same qubit (no immediate repeat).
* fSim(theta, phi) with all Delta parameters zero.
* Two-qubit gate matrices act on |q[0] q[1]> with q[0] the more significant
  bit; fSim is symmetric under exchanging its qubits.
* Bit strings: character j is qubit j; basis index = sum_j x_j 2^(n-1-j).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PATTERN_SEQUENCE = "ABCDCDAB"
ONE_QUBIT_NAMES = ("sqrt_x", "sqrt_y", "sqrt_w")


@dataclass
class Gate:
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    matrix: Optional[np.ndarray] = None  # complex128, (2,2) or (4,4), row-major


@dataclass
class Circuit:
    n_qubits: int
    gates: List[Gate]
    rows: int = 0
    cols: int = 0
    sites: List[Tuple[int, int]] = field(default_factory=list)  # qubit -> (r, c)
    cycles: int = 0
    seed: int = 0

    @property
    def n_two_qubit(self) -> int:
        return sum(1 for g in self.gates if len(g.qubits) == 2)


def one_qubit_matrix(name: str) -> np.ndarray:
    """The three single-qubit gates of the Supplement's circuit section."""
    h = math.sqrt(2.0) / 2.0
    if name == "sqrt_x":
        m = [[1.0, -1j], [-1j, 1.0]]
    elif name == "sqrt_y":
        m = [[1.0, -1.0], [1.0, 1.0]]
    elif name == "sqrt_w":
        m = [[1.0, -h * (1 + 1j)], [h * (1 - 1j), 1.0]]
    else:
        raise ValueError(f"unknown single-qubit gate {name!r}")
    return h * np.array(m, dtype=np.complex128)


def fsim_matrix(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi) with the three Delta phases set to zero."""
    c, s = math.cos(theta), math.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = complex(math.cos(phi), -math.sin(phi))
    return m


def pattern_edges(rows: int, cols: int, pattern: str,
                  present: Sequence[Sequence[bool]]) -> List[Tuple[Tuple[int, int], Tuple[int, int]]]:
    """Grid edges of one two-qubit pattern, missing sites removed."""
    out = []
    for r in range(rows):
        for c in range(cols):
            even = (r + c) % 2 == 0
            if pattern in "AB":
                if c + 1 >= cols or even != (pattern == "A"):
                    continue
                a, b = (r, c), (r, c + 1)
            else:
                if r + 1 >= rows or even != (pattern == "C"):
                    continue
                a, b = (r, c), (r + 1, c)
            if present[a[0]][a[1]] and present[b[0]][b[1]]:
                out.append((a, b))
    return out


def cycle_patterns(cycles: int) -> str:
    reps = PATTERN_SEQUENCE * (cycles // len(PATTERN_SEQUENCE) + 1)
    return reps[:cycles]


def make_rqc(rows: int, cols: int, cycles: int, seed: int, n_missing: int = 0,
             theta: float = math.pi / 2, phi: float = math.pi / 6,
             missing: Optional[Sequence[Tuple[int, int]]] = None,
             two_qubit: bool = True) -> Circuit:
    """Seeded random circuit on a rows x cols grid.

    ``n_missing`` sites are drawn uniformly (without replacement) from the grid
    by the same generator that later draws the single-qubit gates; ``missing``
    names them explicitly instead.  ``two_qubit=False`` drops every two-qubit
    layer (a product-state circuit, used as a closed-form check).
    """
    rng = np.random.default_rng(seed)
    if missing is None:
        missing = []
        if n_missing:
            flat = rng.choice(rows * cols, size=n_missing, replace=False)
            missing = [(int(i) // cols, int(i) % cols) for i in sorted(flat)]
    missing_set = set(tuple(m) for m in missing)
    present = [[(r, c) not in missing_set for c in range(cols)] for r in range(rows)]
    sites = [(r, c) for r in range(rows) for c in range(cols) if present[r][c]]
    qubit_of = {s: i for i, s in enumerate(sites)}
    n = len(sites)

    gates: List[Gate] = []
    prev = [-1] * n

    def one_qubit_layer():
        for q in range(n):
            if prev[q] < 0:
                k = int(rng.integers(3))
            else:
                k = int(rng.integers(2))
                if k >= prev[q]:
                    k += 1
            prev[q] = k
            name = ONE_QUBIT_NAMES[k]
            gates.append(Gate(name, (q,), (), one_qubit_matrix(name)))

    fs = fsim_matrix(theta, phi)
    for pat in cycle_patterns(cycles):
        one_qubit_layer()
        if two_qubit:
            edges = pattern_edges(rows, cols, pat, present)
            for a, b in edges:
                qa, qb = qubit_of[a], qubit_of[b]
                gates.append(Gate("fsim", (qa, qb), (theta, phi), fs.copy()))
    if cycles > 0:
        one_qubit_layer()
    return Circuit(n, gates, rows, cols, sites, cycles, seed)


def near_square_grid(n: int) -> Tuple[int, int]:
    """rows = floor(sqrt(n)), cols = ceil(n / rows)."""
    rows = int(math.isqrt(n))
    cols = -(-n // rows)
    return rows, cols


def uneven_circuit(i: int, seed0: int = 1000, n_range=(24, 40), d_range=(10, 20)) -> Circuit:
    """Circuit i of the uneven batch: n and d drawn from seed0 + i, a
    near-square grid with the surplus sites dropped by the same seed."""
    rng = np.random.default_rng(seed0 + i)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    d = int(rng.integers(d_range[0], d_range[1] + 1))
    rows, cols = near_square_grid(n)
    return make_rqc(rows, cols, d, seed0 + i, n_missing=rows * cols - n)


def make_uneven_batch(count: int, seed0: int = 1000, n_range=(24, 40),
                      d_range=(10, 20)) -> List[Circuit]:
    """Circuits of uneven size: n and d drawn per circuit from seed0 + i."""
    return [uneven_circuit(i, seed0, n_range, d_range) for i in range(count)]


def random_bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    """Uniform bit strings, uint8[count, n], qubit j in column j."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(count, n), dtype=np.uint8)


def bits_to_index(bits: Sequence[int]) -> int:
    idx = 0
    for b in bits:
        idx = (idx << 1) | int(b)
    return idx
