"""Measured choice among candidate contraction orders (Supplement, section
"Tensor network contraction algorithm": many orders are found, and the one
whose single slice runs fastest on the machine is used).

Each candidate (pairs, sliced wires) is planned through the library, one
slice is run to warm up, then `reps` slices are timed with events on the
current stream; the estimate of the whole job is the time per slice times
the slice count.  Plans use the planner's default kernel rules unless tune
is set (the autotuner then runs for every candidate).  All contraction work runs in the library's kernels.

  python -m paper_2111_01066_amd.order_select CANDIDATES.json OUT.json [--dtype c64] [--reps 2]
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def time_candidates(circuit, open_qubits, out_bits, candidates, dtype="c64", reps=2, tune=False, tune_db=None,
                    log=print):
    import torch

    from . import tnrcs
    out = []
    for i, c in enumerate(candidates):
        pairs = [tuple(p) for p in c["pairs"]]
        log(f"[order_select] candidate {i}: planning ({c.get('source', '')})")
        t0 = time.perf_counter()
        plan = tnrcs.Plan(circuit, pairs, c["sliced"], open_qubits, out_bits, dtype=dtype, tune=tune,
                          tune_db=tune_db)
        t_plan = time.perf_counter() - t0
        n = plan.info()["n_slices"]
        amp = torch.zeros(1 << len(open_qubits), dtype=torch.complex128, device="cuda")
        plan.contract(0, 1, amp)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.contract(1, 1 + reps, amp)
        e1.record(s)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        plan.close()
        rec = dict(index=i, source=c.get("source", ""), sec_per_slice=sec, n_slices=n,
                   time_to_amplitudes_s=sec * n, plan_s=t_plan, flops_per_slice=c.get("flops_per_slice"),
                   model_cost=c.get("model_cost"))
        log(f"[order_select] candidate {i}: {sec:.4f} s/slice x {n} slices = {sec * n:.1f} s "
            f"(plan {t_plan:.1f} s; {rec['source']})")
        out.append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("candidates")
    ap.add_argument("out")
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--reps", type=int, default=2)
    a = ap.parse_args()
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    from rqcgen.workloads import config3_circuit
    c, open_q, bits = config3_circuit()
    with open(a.candidates) as f:
        cands = json.load(f)
    res = time_candidates(c, open_q, bits, cands, dtype=a.dtype, reps=a.reps,
                          log=lambda *x: print(*x, file=sys.stderr, flush=True))
    best = min(res, key=lambda r: r["time_to_amplitudes_s"])
    with open(a.out, "w") as f:
        json.dump(dict(timings=res, chosen=best["index"]), f, indent=1)
    print(json.dumps(dict(chosen=best["index"], time_to_amplitudes_s=best["time_to_amplitudes_s"])))


if __name__ == "__main__":
    main()
