"""Writes the frozen contraction orders of the batched uneven workload
(rqcgen/data/config5_orders.npz): 512 circuits drawn by make_uneven_batch
(n uniform on 24..40 qubits, d uniform on 10..20 cycles, seeds 1000 + i),
each with its 6 highest-numbered qubits open.

Per circuit the candidates are greedy orders (seeds 0..3) and recursive
bisection orders (seeds 0..2); each is sliced to the per-tensor bound
2^S with S = 28, raised one at a time while more than 8 wires would be
sliced; the candidate with the lowest total flop count (per-slice flops x
slice count) is kept.

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
from .order import bisection_order, greedy_order, order_stats, slice_to_fit
from .workloads import DATA

S_BASE = 28
K_MAX = 8


def _best_order(i: int):
    c = uneven_circuit(i)
    open_q = list(range(c.n_qubits - 6, c.n_qubits))
    ns = network_structure(c, open_q)
    cands = [("greedy", sd, greedy_order(ns, seed=sd)) for sd in range(4)]
    cands += [("bisect", sd, bisection_order(ns, seed=sd)) for sd in range(3)]
    best = None
    for kind, sd, pairs in cands:
        S = S_BASE
        while True:
            sliced = slice_to_fit(ns, pairs, S)
            if len(sliced) <= K_MAX:
                break
            S += 1
        st = order_stats(ns, pairs, sliced)
        key = (st.total_flops, st.flops_per_slice)
        if best is None or key < best[0]:
            best = (key, kind, sd, pairs, sliced, S, st)
    _, kind, sd, pairs, sliced, S, st = best
    return dict(i=i, n=c.n_qubits, d=c.cycles, pairs=np.asarray(pairs, dtype=np.int32).reshape(-1, 2),
                sliced=np.asarray(sliced, dtype=np.int32), S=S, total=st.total_flops,
                per_slice=st.flops_per_slice, log2_max=st.log2_max, method=f"{kind}:{sd}")


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
