"""Writes the frozen contraction orders of the batched uneven workload
(rqcgen/data/config5_orders.npz): 512 circuits drawn by make_uneven_batch
(n uniform on 24..40 qubits, d uniform on 10..20 cycles, seeds 1000 + i),
each with its 6 highest-numbered qubits open.

Per circuit: recursive-bisection trees (seeds 0..2) are reconfigured,
sliced to the per-tensor bound 2^S with reconfiguration between slicing
steps (rqcgen.optimize; S = 28, raised one at a time while more than 8
wires would be sliced), and the one with the lowest total cost in the
kernel time model (scaled FP16 storage: alpha = 100) is kept.

  python -m rqcgen.make_batch_orders [--count 512] [--jobs 6]
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

from .circuit import uneven_circuit
from .network import network_structure
from .optimize import CostModel, _Net, optimize_tree
from .workloads import DATA

S_BASE = 28
K_MAX = 8
ALPHA = 100.0


def _best_order(i: int):
    c = uneven_circuit(i)
    open_q = list(range(c.n_qubits - 6, c.n_qubits))
    ns = network_structure(c, open_q)
    net = _Net(ns)
    best = None
    for sd in range(3):
        S = S_BASE
        while True:
            t = net.bisection_tree(sd, 0.35, 0.65, 8, True)
            r = optimize_tree(net, t, CostModel(ALPHA, S), m=8, source=f"bisect:{sd}")
            if len(r.sliced) <= K_MAX:
                break
            S += 1
        key = (r.total_cost, r.total_flops)
        if best is None or key < best[0]:
            best = (key, r, S)
    _, r, S = best
    return dict(i=i, n=c.n_qubits, d=c.cycles, pairs=np.asarray(r.pairs, dtype=np.int32).reshape(-1, 2),
                sliced=np.asarray(r.sliced, dtype=np.int32), S=S, total=r.total_flops,
                per_slice=r.flops_per_slice, log2_max=r.log2_max, method=r.source)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    t0 = time.time()
    with Pool(a.jobs) as pool:
        res = []
        for r in pool.imap(_best_order, range(a.count)):
            res.append(r)
            print(f"{r['i']:4d} n={r['n']} d={r['d']} {r['method']:9s} S={r['S']} k={len(r['sliced'])} "
                  f"total={r['total']:.3e} ({time.time() - t0:.0f} s)", flush=True)
    pair_off = np.cumsum([0] + [len(r["pairs"]) for r in res]).astype(np.int64)
    sl_off = np.cumsum([0] + [len(r["sliced"]) for r in res]).astype(np.int64)
    out = os.path.join(DATA, "config5_orders.npz")
    np.savez_compressed(
        out, pairs=np.concatenate([r["pairs"] for r in res]), pair_off=pair_off,
        sliced=np.concatenate([r["sliced"] for r in res]), sliced_off=sl_off,
        S=np.array([r["S"] for r in res], dtype=np.int32), n=np.array([r["n"] for r in res], dtype=np.int32),
        d=np.array([r["d"] for r in res], dtype=np.int32),
        total_flops=np.array([r["total"] for r in res]), flops_per_slice=np.array([r["per_slice"] for r in res]),
        log2_max=np.array([r["log2_max"] for r in res], dtype=np.int32),
        method=np.array([r["method"] for r in res]))
    print(f"wrote {out}", file=sys.stderr)


if __name__ == "__main__":
    main()
