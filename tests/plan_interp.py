"""NumPy interpreter of a dry-run plan (test infrastructure).

Executes the planner's JSON step list (bind, permute, GEMM, gathered
contraction, accumulate) on flat complex128 arrays that stand for the device
regions, so the planner's index bookkeeping, layouts and arena offsets can be
checked against the oracle without a GPU.  It shares nothing with the oracle.
"""
import numpy as np


def dep(x, runs):
    x = np.asarray(x, dtype=np.int64)
    out = np.zeros_like(x)
    for src, dst, ln in runs:
        out |= ((x >> src) & ((1 << ln) - 1)) << dst
    return out


class PlanInterpreter:
    def __init__(self, plan):
        self.js = plan.json()
        js = self.js
        self.leaves = np.zeros(js["leaves_elems"], dtype=np.complex128)
        for i, d in enumerate(js["dev_leaves"]):
            n = 1 << len(d["layout"])
            self.leaves[d["stored_off"]:d["stored_off"] + n] = plan.leaf(i, n)
        self.bound = np.full(js["bound_elems"], np.nan, dtype=np.complex128)
        self.arena = np.full(js["arena_elems"], np.nan, dtype=np.complex128)

    ext = {}

    def region(self, ref):
        reg, off = ref
        if reg >= 3:
            return self.ext[reg], off
        return {0: self.arena, 1: self.leaves, 2: self.bound}[reg], off

    def run_ops(self):
        self._ops(self.js["ops"])

    def run_slice(self, s, amp):
        js = self.js
        for b in js["binds"]:
            off = 0
            for sb, p in zip(b["sbit"], b["pos"]):
                off |= ((s >> sb) & 1) << p
            self.bound[b["dst"]:b["dst"] + b["n"]] = self.leaves[b["src"] + off:b["src"] + off + b["n"]]
        self._ops(js["ops"])
        acc = js["accum"]
        rr, orr = self.region(acc["root"])
        y = np.arange(1 << acc["n_open"])
        v = rr[orr + dep(y, acc["y2root"])]
        assert not np.isnan(v).any()
        amp += v

    def _ops(self, ops):
        for op in ops:
            ra, oa = self.region(op["a"])
            rc, oc = self.region(op["c"])
            if op["kind"] == 0:  # permute
                r = op["rank"]
                o = np.arange(1 << r, dtype=np.int64)
                i = np.zeros_like(o)
                for q, p in enumerate(op["perm"]):
                    i |= ((o >> q) & 1) << p
                rc[oc:oc + (1 << r)] = ra[oa + i]
            elif op["kind"] == 1:  # gemm
                rb, ob = self.region(op["b"])
                M, N, K = op["M"], op["N"], op["K"]
                if op.get("ga"):  # A read in its stored layout
                    Ai = dep(np.arange(M), op["aM"])[:, None] | dep(np.arange(K), op["aK"])[None, :]
                    A = ra[oa + Ai]
                else:
                    A = ra[oa:oa + M * K].reshape(M, K)
                B = rb[ob:ob + N * K].reshape(N, K)
                assert not np.isnan(A).any() and not np.isnan(B).any()
                rc[oc:oc + M * N] = (A @ B.T).reshape(-1)
            else:  # gathered contraction
                rb, ob = self.region(op["b"])
                nM, nN, nK = op["nM"], op["nN"], op["nK"]
                m = np.arange(1 << nM)
                n = np.arange(1 << nN)
                k = np.arange(1 << nK)
                Ai = dep(m, op["aM"])[:, None] | dep(k, op["aK"])[None, :]
                Bi = dep(n, op["bN"])[:, None] | dep(k, op["bK"])[None, :]
                A = ra[oa + Ai]
                B = rb[ob + Bi]
                assert not np.isnan(A).any() and not np.isnan(B).any()
                rc[oc:oc + (1 << (nM + nN))] = (A @ B.T).reshape(-1)
