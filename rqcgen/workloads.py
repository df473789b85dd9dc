"""The synthetic workloads (inputs only): circuits, open qubits, closed bits
and contraction orders for the benchmark configurations.

* config 1: 20 qubits on a 4x5 grid, 8 cycles, seed 0; greedy order by seed 0,
  no slicing; 64 uniformly random bit strings (seed 1).
* config 2: pairwise-contraction microbench, rank-27 x rank-25 complex
  tensors sharing 12 indices at seeded positions, output permuted (seed 2).
* config 3: 53 qubits on a 6x9 grid with one seeded-missing site, 14 cycles,
  seed 3; the 6 highest-numbered qubits open (a bunch of 64), the other 47
  closed at uniformly random bits (seed 3); sliced so every per-slice tensor
  has at most 2^32 entries.  Its order is frozen in data/config3_order.json
  (written by make_orders.py) so every machine contracts the same network.
* config 5: the batched uneven workload, 512 circuits from make_uneven_batch
  (24..40 qubits, 10..20 cycles, seeds 1000 + i), the 6 highest-numbered
  qubits of each open, the others closed at uniformly random bits (seed
  1000 + i); orders and sliced wires frozen in data/config5_orders.npz
  (written by make_batch_orders.py; at most 8 sliced wires each).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from .circuit import Circuit, make_rqc, random_bitstrings, uneven_circuit
from .network import network_structure
from .order import greedy_order

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


@dataclass
class Workload:
    name: str
    circuit: Circuit
    open_qubits: List[int]
    out_bits: np.ndarray
    pairs: List[Tuple[int, int]]
    sliced: List[int]


def config1(all_open: bool = True) -> Workload:
    c = make_rqc(4, 5, 8, seed=0)
    open_q = list(range(20)) if all_open else []
    ns = network_structure(c, open_q)
    pairs = greedy_order(ns, seed=0)
    bits = np.zeros(20, dtype=np.uint8)
    return Workload("rqc-20q-4x5-d8", c, open_q, bits, pairs, [])


def config1_bitstrings() -> np.ndarray:
    return random_bitstrings(20, 64, seed=1)


def config3_circuit() -> Tuple[Circuit, List[int], np.ndarray]:
    c = make_rqc(6, 9, 14, seed=3, n_missing=1)
    open_q = list(range(c.n_qubits - 6, c.n_qubits))
    bits = random_bitstrings(c.n_qubits, 1, seed=3)[0]
    bits[open_q] = 0
    return c, open_q, bits


def load_order(name: str):
    with open(os.path.join(DATA, name)) as f:
        d = json.load(f)
    return [tuple(p) for p in d["pairs"]], list(d["sliced"]), d


def config3() -> Workload:
    c, open_q, bits = config3_circuit()
    pairs, sliced, _ = load_order("config3_order.json")
    return Workload("rqc-53q-6x9m1-d14-S32", c, open_q, bits, pairs, sliced)


def config2_pair(seed: int = 2):
    """Index structure of one rank-27 x rank-25 pair: 12 shared indices at
    seeded positions; output = a seeded permutation of the 28 free indices.
    Returns (labels_a, labels_b, labels_out) with labels 0..39."""
    rng = np.random.default_rng(seed)
    labels = rng.permutation(40)
    shared = list(labels[:12])
    free_a = list(labels[12:27])
    free_b = list(labels[27:40])
    la = list(rng.permutation(shared + free_a))
    lb = list(rng.permutation(shared + free_b))
    lo = list(rng.permutation(free_a + free_b))
    return [int(x) for x in la], [int(x) for x in lb], [int(x) for x in lo]


def config4() -> Workload:
    """The 30-qubit cross-check network of the precision study: a 5x6 grid,
    14 cycles, seed 4, every qubit open (2^30 amplitudes), contracted in the
    gate-by-gate order."""
    from .order import schroedinger_order
    c = make_rqc(5, 6, 14, seed=4)
    open_q = list(range(30))
    return Workload("rqc-30q-5x6-d14-all-open", c, open_q, np.zeros(30, dtype=np.uint8),
                    schroedinger_order(c, open_q), [])


def config4_uniform_indices(n_samples: int = 100_000) -> np.ndarray:
    """The uniformly drawn basis indices of the 30-qubit cross-check
    (numpy default_rng(6))."""
    return np.random.default_rng(6).integers(0, 2 ** 30, size=n_samples, dtype=np.int64)


def config5_table() -> dict:
    """The frozen per-circuit order table of config 5 (numpy arrays)."""
    with np.load(os.path.join(DATA, "config5_orders.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def config5(indices=None, max_total_flops: float = None, table: dict = None) -> List[Workload]:
    """Config-5 circuits (all 512, the given indices, or those whose frozen
    order costs at most max_total_flops over all slices), in index order."""
    t = table if table is not None else config5_table()
    count = len(t["S"])
    idx = range(count) if indices is None else indices
    out = []
    for i in idx:
        if max_total_flops is not None and t["total_flops"][i] > max_total_flops:
            continue
        c = uneven_circuit(i)
        open_q = list(range(c.n_qubits - 6, c.n_qubits))
        bits = random_bitstrings(c.n_qubits, 1, seed=1000 + i)[0]
        bits[open_q] = 0
        p0, p1 = t["pair_off"][i], t["pair_off"][i + 1]
        s0, s1 = t["sliced_off"][i], t["sliced_off"][i + 1]
        pairs = [(int(a), int(b)) for a, b in t["pairs"][p0:p1]]
        sliced = [int(x) for x in t["sliced"][s0:s1]]
        out.append(Workload(f"uneven-{i}-{c.n_qubits}q-d{c.cycles}", c, open_q, bits, pairs, sliced))
    return out
