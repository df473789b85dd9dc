"""Writes the frozen contraction order of the 53-qubit benchmark network
(rqcgen/data/config3_order.json) and its runner-up candidates
(rqcgen/data/config3_candidates.json).

Deterministic search (Supplement, "Tensor network contraction algorithm":
partition, slice, reconfigure, keep the best of many orders): recursive
bisection trees over a fixed grid of seeds, balance windows and leaf sizes;
each tree is reconfigured, sliced to 2^32 entries per tensor with
reconfiguration between slicing steps (live set <= 2^35 entries), and scored
by the kernel time model of rqcgen.optimize times the slice count.  The best
few are polished with larger reconfiguration windows.  The candidates file
feeds the measured choice among orders (one timed slice each on the GPU,
paper_2111_01066_amd.order_select); config3_order.json holds the chosen one.

  python -m rqcgen.make_orders [--jobs 8] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

from .network import network_structure
from .optimize import CostModel, _Net, optimize_tree
from .workloads import DATA, config3_circuit

MAX_LOG2 = 32
LIVE_CAP = 2.0 ** 35
ALPHA = 32.0


def _net():
    c, open_q, _ = config3_circuit()
    return _Net(network_structure(c, open_q))


def _trial(args):
    seed, lo, hi, leaf, kl = args
    net = _net()
    t = net.bisection_tree(seed, lo, hi, leaf, kl)
    r = optimize_tree(net, t, CostModel(ALPHA, MAX_LOG2), m=8, live_cap=LIVE_CAP,
                      source=f"bisection seed={seed} window=({lo},{hi}) leaf={leaf} kl={kl}")
    return args, r


def _polish(args):
    (seed, lo, hi, leaf, kl), m = args
    net = _net()
    t = net.bisection_tree(seed, lo, hi, leaf, kl)
    r = optimize_tree(net, t, CostModel(ALPHA, MAX_LOG2), m=m, live_cap=LIVE_CAP,
                      source=f"bisection seed={seed} window=({lo},{hi}) leaf={leaf} kl={kl} m={m}")
    return args[0], r


def _record(r, params):
    return dict(pairs=[list(p) for p in r.pairs], sliced=list(r.sliced), max_log2=MAX_LOG2, source=r.source,
                params=params, flops_per_slice=r.flops_per_slice, total_flops=r.total_flops,
                log2_max=r.log2_max, peak_elems=r.peak_elems, model_cost=r.total_cost, alpha=ALPHA)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--keep", type=int, default=6, help="candidates written for the measured choice")
    a = ap.parse_args()
    seeds = range(4) if a.quick else range(12)
    grid = [(s, lo, hi, leaf, kl) for s in seeds for (lo, hi) in ((0.3, 0.7), (0.35, 0.65), (0.4, 0.6), (0.25, 0.75))
            for leaf in (4, 8) for kl in (True, False)]
    res = []
    with ProcessPoolExecutor(a.jobs) as ex:
        for args, r in ex.map(_trial, grid):
            res.append((r.total_cost, args, r))
            print(f"  {r.source}: k={len(r.sliced)} flops {r.total_flops:.3e} model {r.total_cost:.3e}", flush=True)
    res.sort(key=lambda x: x[0])
    top = [x[1] for x in res[: a.keep]]
    with ProcessPoolExecutor(a.jobs) as ex:
        pol = list(ex.map(_polish, [(t, 10) for t in top]))
    final = []
    for (args, r0) in [(x[1], x[2]) for x in res[: a.keep]] + pol:
        final.append((r0.total_cost, args, r0))
    final.sort(key=lambda x: x[0])
    seen, cands = set(), []
    for cost, args, r in final:
        key = (tuple(map(tuple, r.pairs)), tuple(r.sliced))
        if key in seen:
            continue
        seen.add(key)
        cands.append(_record(r, dict(seed=args[0], lo=args[1], hi=args[2], leaf=args[3], kl=args[4])))
        if len(cands) == a.keep:
            break
    os.makedirs(DATA, exist_ok=True)
    with open(os.path.join(DATA, "config3_candidates.json"), "w") as f:
        json.dump(cands, f)
    with open(os.path.join(DATA, "config3_order.json"), "w") as f:
        json.dump(cands[0], f)
    for c in cands:
        print(f"candidate: {c['source']}: k={len(c['sliced'])} flops/slice {c['flops_per_slice']:.3e} "
              f"total {c['total_flops']:.3e} model {c['model_cost']:.3e}", file=sys.stderr)


if __name__ == "__main__":
    main()
