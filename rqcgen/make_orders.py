"""Writes the frozen contraction orders of the benchmark networks
(rqcgen/data/*.json).  Deterministic search: recursive-bisection orders over
a fixed grid of seeds and balance windows, each sliced to the size bound,
the lowest total flop count kept."""
from __future__ import annotations

import json
import os
import sys

from .network import network_structure
from .order import bisection_order, order_stats, slice_to_fit
from .workloads import DATA, config3_circuit


def search(ns, max_log2, seeds=range(6), windows=((0.3, 0.7), (0.25, 0.75), (0.35, 0.65)),
           leaf_sizes=(4, 8), live_cap=None):
    best = None
    for lo, hi in windows:
        for leaf in leaf_sizes:
            for kl in (True, False):
                for sd in seeds:
                    pairs = bisection_order(ns, seed=sd, lo=lo, hi=hi, leaf_size=leaf, use_kl=kl)
                    sliced = slice_to_fit(ns, pairs, max_log2, max_live_elems=live_cap)
                    st = order_stats(ns, pairs, sliced)
                    key = (st.total_flops, st.flops_per_slice)
                    if best is None or key < best[0]:
                        best = (key, pairs, sliced, st, dict(lo=lo, hi=hi, leaf=leaf, kl=kl, seed=sd))
                        print(f"  lo={lo} hi={hi} leaf={leaf} kl={kl} seed={sd}: k={len(sliced)} "
                              f"flops/slice={st.flops_per_slice:.3e} total={st.total_flops:.3e} "
                              f"peak={st.peak_elems:.3e}", flush=True)
    return best


def main():
    os.makedirs(DATA, exist_ok=True)
    c, open_q, _ = config3_circuit()
    ns = network_structure(c, open_q)
    # 2^32-entry bound per tensor (complex64: 32 GiB), live set <= 2^35 entries
    _, pairs, sliced, st, params = search(ns, 32, live_cap=2.0 ** 35)
    out = dict(pairs=[list(p) for p in pairs], sliced=sliced, max_log2=32, params=params,
               flops_per_slice=st.flops_per_slice, total_flops=st.total_flops, log2_max=st.log2_max,
               peak_elems=st.peak_elems)
    with open(os.path.join(DATA, "config3_order.json"), "w") as f:
        json.dump(out, f)
    print("wrote config3_order.json", file=sys.stderr)


if __name__ == "__main__":
    main()
