"""Tensor-network contraction of a circuit amplitude in FP64.

Follows the paper's description (main text, TNC section; Supplement, "Tensor
network contraction algorithm", Fig. S2): the initial state and the target
basis are rank-1 tensors, single-qubit gates rank-2 and two-qubit gates rank-4
tensors, every bond of dimension 2; contracting the network gives the
amplitude.  A contraction order is a list of pairwise contractions (SSA form:
step t contracts ids pairs[t] and creates id n_leaves + t).  Index slicing
fixes a set of bonds to given values; the network equals the sum of the sliced
networks over all 2^k assignments.  Leaving qubits open gives a bunch of
amplitudes (main text, "Establishing quantum supremacy baseline").

Each pairwise step is the plain definition of the Supplement's Eq. (matmul):
sum over the shared indices of A times B, kept free indices of A then of B,
evaluated with numpy.tensordot.

Canonical numbering (a written convention, not shared code): leaves 0..n-1
are the |0> vectors (index [out]); then the gates in circuit order (indices
[outs..., ins...]); then the closed qubits' output vectors in qubit order
(index [in]).  Wire q < n leaves the |0> vector of qubit q, and each gate
appends one new wire per qubit of its qubit list.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .gates import gate_matrix


def build_network(circuit, open_qubits: Sequence[int] = (), closed_bits: Sequence[int] = None):
    """Leaves as (tensor, wires) and the open wires in increasing qubit order."""
    n = circuit.n_qubits
    open_set = sorted(set(int(q) for q in open_qubits))
    leaves: List[Tuple[np.ndarray, List[int]]] = []
    for q in range(n):
        leaves.append((np.array([1.0, 0.0], dtype=np.complex128), [q]))
    cur = list(range(n))
    nw = n
    for g in circuit.gates:
        k = len(g.qubits)
        ins = [cur[q] for q in g.qubits]
        outs = []
        for q in g.qubits:
            cur[q] = nw
            outs.append(nw)
            nw += 1
        t = gate_matrix(g.name, g.params).reshape((2,) * (2 * k))
        leaves.append((t, outs + ins))
    for q in range(n):
        if q in open_set:
            continue
        v = np.zeros(2, dtype=np.complex128)
        v[int(closed_bits[q]) if closed_bits is not None else 0] = 1.0
        leaves.append((v, [cur[q]]))
    return leaves, [cur[q] for q in open_set]


def pairwise_contract(a: np.ndarray, wa: Sequence[int], b: np.ndarray, wb: Sequence[int]):
    """Supplement Eq. (matmul): C[free A, free B] = sum_shared A * B."""
    shared = [w for w in wa if w in wb]
    ax_a = [list(wa).index(w) for w in shared]
    ax_b = [list(wb).index(w) for w in shared]
    c = np.tensordot(a, b, axes=(ax_a, ax_b))
    wc = [w for w in wa if w not in shared] + [w for w in wb if w not in shared]
    return c, wc


def _fix(t: np.ndarray, wires: List[int], fixed: Dict[int, int]):
    for w, v in fixed.items():
        if w in wires:
            ax = wires.index(w)
            t = np.take(t, int(v), axis=ax)
            wires = wires[:ax] + wires[ax + 1:]
    return t, wires


def contract_network(leaves, pairs: Sequence[Tuple[int, int]], open_wires: Sequence[int],
                     fixed: Optional[Dict[int, int]] = None) -> np.ndarray:
    """Contract one (sliced) network in the given order.  ``fixed`` maps wire
    -> value for sliced wires.  Returns the flattened bunch over open wires."""
    fixed = fixed or {}
    live: Dict[int, Tuple[np.ndarray, List[int]]] = {}
    for i, (t, w) in enumerate(leaves):
        live[i] = _fix(t, list(w), fixed)
    nxt = len(leaves)
    if len(pairs) != len(leaves) - 1:
        raise ValueError("order is not a full contraction tree")
    for a, b in pairs:
        ta, wa = live.pop(a)
        tb, wb = live.pop(b)
        live[nxt] = pairwise_contract(ta, wa, tb, wb)
        nxt += 1
    (t, w), = live.values()
    ow = [x for x in open_wires if x not in fixed]
    if sorted(w) != sorted(ow):
        raise ValueError("final tensor wires do not match the open wires")
    t = np.transpose(t, [w.index(x) for x in ow]) if ow else t
    return np.asarray(t).reshape(-1)


def slice_assignment(sliced: Sequence[int], s: int) -> Dict[int, int]:
    """Slice id s fixes sliced[j] to bit j of s."""
    return {int(w): (int(s) >> j) & 1 for j, w in enumerate(sliced)}


def contract_slice(leaves, pairs, open_wires, sliced, s, sub_sliced: Sequence[int] = ()):
    """One slice; optionally as the sum of its 2^j sub-slices (identical value)."""
    base = slice_assignment(sliced, s)
    total = None
    for u in range(1 << len(sub_sliced)):
        fx = dict(base)
        fx.update(slice_assignment(sub_sliced, u))
        v = contract_network(leaves, pairs, open_wires, fx)
        total = v if total is None else total + v
    return total


def contract_sliced(leaves, pairs, open_wires, sliced: Sequence[int] = (),
                    slices: Optional[Sequence[int]] = None) -> np.ndarray:
    """Sum over slices (all 2^k by default) of the sliced networks."""
    if slices is None:
        slices = range(1 << len(sliced))
    total = None
    for s in slices:
        v = contract_slice(leaves, pairs, open_wires, sliced, s)
        total = v if total is None else total + v
    return total


def contract_entry(sub_a: np.ndarray, shared_a, sub_b: np.ndarray, shared_b) -> complex:
    """One output entry of Eq. (matmul): with every free index of A and B
    fixed, the sum over the shared indices of A * B.  sub_a / sub_b hold the
    remaining (shared) axes, labelled by shared_a / shared_b (the same labels,
    possibly in different orders)."""
    sb = np.transpose(sub_b, [list(shared_b).index(l) for l in shared_a]) if len(shared_a) else sub_b
    return complex(np.sum(sub_a * sb))


def contract_entries(a: np.ndarray, la, b: np.ndarray, lb, lc, coords) -> np.ndarray:
    """Entries C[coords[i]] of C = sum over shared labels of A * B, entry by
    entry (coords: output index values, one column per label of lc)."""
    shared_a = [l for l in la if l in lb]
    shared_b = [l for l in lb if l in la]
    out = np.empty(len(coords), dtype=np.complex128)
    for i, c in enumerate(coords):
        fix = dict(zip(lc, (int(x) for x in c)))
        sa = a[tuple(fix[l] if l in fix else slice(None) for l in la)]
        sb = b[tuple(fix[l] if l in fix else slice(None) for l in lb)]
        out[i] = contract_entry(sa, shared_a, sb, shared_b)
    return out
