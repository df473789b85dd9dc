"""Index structure of the canonical tensor network of a circuit (graph only).

The network for an amplitude <x_C, y_O| U |0^n> (paper, main text section on
the customized TNC algorithm, and Supplement Fig. S2): rank-1 input vectors,
rank-2 single-qubit gates, rank-4 two-qubit gates and rank-1 output vectors on
the closed qubits; every bond has dimension 2.

Canonical numbering, shared with the contraction library as a written
convention (not as code):

* leaves 0..n-1 are the |0> vectors, index list [out];
* then one leaf per gate in circuit order, index list [outs..., ins...];
* then one output vector per closed qubit, in qubit order, index list [in];
* wire q (0 <= q < n) is the output of the |0> vector on qubit q; every gate
  appends one new wire per qubit of its qubit list, in that order;
* the final wires of the open qubits are the open indices of the network, in
  increasing qubit order.

Only wire identities are produced here; no tensor values.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

from .circuit import Circuit


@dataclass
class NetworkStructure:
    n_qubits: int
    n_wires: int
    leaf_wires: List[List[int]]   # per leaf, its wires in index order
    open_wires: List[int]         # final wires of the open qubits, qubit order
    open_qubits: List[int]
    leaf_kind: List[str]          # "in", gate name, or "out"
    final_wire: List[int]         # per qubit, the wire leaving the circuit

    @property
    def n_leaves(self) -> int:
        return len(self.leaf_wires)


def network_structure(circuit: Circuit, open_qubits: Sequence[int] = ()) -> NetworkStructure:
    n = circuit.n_qubits
    open_set = sorted(set(int(q) for q in open_qubits))
    for q in open_set:
        if not 0 <= q < n:
            raise ValueError(f"open qubit {q} out of range")
    leaf_wires: List[List[int]] = [[q] for q in range(n)]
    kinds = ["in"] * n
    cur = list(range(n))
    n_wires = n
    for g in circuit.gates:
        ins = [cur[q] for q in g.qubits]
        outs = []
        for q in g.qubits:
            cur[q] = n_wires
            outs.append(n_wires)
            n_wires += 1
        leaf_wires.append(outs + ins)
        kinds.append(g.name)
    closed = [q for q in range(n) if q not in open_set]
    for q in closed:
        leaf_wires.append([cur[q]])
        kinds.append("out")
    return NetworkStructure(n, n_wires, leaf_wires, [cur[q] for q in open_set],
                            open_set, kinds, list(cur))
