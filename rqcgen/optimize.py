"""Contraction-tree search with slicing and subtree reconfiguration (input
side: wire bookkeeping only, no tensor values).

The paper finds its orders with a partition-based search followed by index
slicing and subtree reconfiguration, and picks among many candidate orders
(Supplement, section "Tensor network contraction algorithm").  This module
is this project's own version of that pipeline:

1. the network is first simplified by the section's rule (rank-1 and rank-2
   tensors absorbed, pairs whose result is no larger than the larger operand
   pre-contracted);
2. starting trees over the simplified tensors come from seeded recursive
   bisection (spectral + Kernighan-Lin) and from a seeded randomized greedy;
3. subtree reconfiguration: for a node of the tree, its subtree is cut at up
   to ``m`` descendants (always opening the largest one) and the best binary
   tree over those pieces is found by dynamic programming over subsets; a
   better subtree replaces the old one.  Sweeps go over all nodes until the
   cost stops falling;
4. slicing interleaved with reconfiguration: while some intermediate exceeds
   the size bound, the wire whose slicing raises the total cost least (the
   per-slice cost times the slice count) is sliced, and the tree is
   reconfigured for the sliced network.

The cost of one pairwise step is a time model of the kernels that run it:
``2^|A u B|`` complex multiply-adds plus ``alpha`` times the entries of A, B
and C (each tensor moved once, the fused-kernel principle of Supplement
Fig. S7a); alpha is the ratio of the time to move one complex entry to the
time of one complex multiply-add (about 32 for complex64 on MI355X: 8 bytes
at ~5 TB/s against 8 flops at ~170 TFLOP/s).  Flop counts are reported
separately (one complex multiply-add = 8 flops).

Masks are Python ints over wire ids; every wire joins at most two tensors,
so the wires of a contracted set are the XOR of its members' masks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .network import NetworkStructure
from .order import _Bisect, _Greedy, _mask, live_peak, order_stats

INF = float("inf")


def _pc(x: int) -> int:
    return x.bit_count()


class Tree:
    """Binary contraction tree over base tensors 0..B-1 (internal nodes
    B..2B-2); mask[n] is the wire set of node n's tensor."""

    def __init__(self, base_masks: Sequence[int]):
        self.B = len(base_masks)
        self.mask: List[int] = list(base_masks) + [0] * (self.B - 1)
        self.left: List[int] = [-1] * (2 * self.B - 1)
        self.right: List[int] = [-1] * (2 * self.B - 1)
        self.parent: List[int] = [-1] * (2 * self.B - 1)
        self.root = -1

    def is_leaf(self, n: int) -> bool:
        return n < self.B

    def set_children(self, n: int, a: int, b: int):
        self.left[n], self.right[n] = a, b
        self.parent[a] = self.parent[b] = n
        self.mask[n] = self.mask[a] ^ self.mask[b]

    def internal(self) -> List[int]:
        return list(range(self.B, 2 * self.B - 1))

    def postorder(self) -> List[int]:
        out, stack = [], [(self.root, False)]
        while stack:
            n, done = stack.pop()
            if self.is_leaf(n):
                continue
            if done:
                out.append(n)
            else:
                stack.append((n, True))
                stack.append((self.right[n], False))
                stack.append((self.left[n], False))
        return out

    def copy(self) -> "Tree":
        t = Tree.__new__(Tree)
        t.B = self.B
        t.mask, t.left, t.right, t.parent = list(self.mask), list(self.left), list(self.right), list(self.parent)
        t.root = self.root
        return t


@dataclass
class CostModel:
    alpha: float = 32.0        # entry moves per multiply-add of time
    max_log2: int = 32         # bound on every per-slice tensor (entries, log2)

    def step(self, ma: int, mb: int, keep: int) -> float:
        sa, sb, sc = _pc(ma & keep), _pc(mb & keep), _pc((ma ^ mb) & keep)
        return 2.0 ** _pc((ma | mb) & keep) + self.alpha * (2.0 ** sa + 2.0 ** sb + 2.0 ** sc)


def tree_cost(t: Tree, cm: CostModel, keep: int) -> float:
    m, L, R = t.mask, t.left, t.right
    return sum(cm.step(m[L[n]], m[R[n]], keep) for n in range(t.B, 2 * t.B - 1))


def tree_flops(t: Tree, keep: int) -> float:
    m, L, R = t.mask, t.left, t.right
    return sum(8.0 * 2.0 ** _pc((m[L[n]] | m[R[n]]) & keep) for n in range(t.B, 2 * t.B - 1))


def tree_max_log2(t: Tree, keep: int) -> int:
    return max(_pc(m & keep) for m in t.mask)


# --------------------------------------------------------------- subtrees --

def _best_tree(fm: List[int], cm: CostModel, keep: int):
    """Cheapest binary tree over the pieces fm (DP over subsets).  Returns
    (cost, split) with split[s] the chosen first part of subset s."""
    k = len(fm)
    full = (1 << k) - 1
    sm = [0] * (full + 1)
    sz = [0] * (full + 1)
    for s in range(1, full + 1):
        i = (s & -s).bit_length() - 1
        sm[s] = sm[s ^ (1 << i)] ^ fm[i]
        sz[s] = _pc(sm[s] & keep)
    best = [INF] * (full + 1)
    split = [0] * (full + 1)
    for i in range(k):
        best[1 << i] = 0.0
    alpha, cap = cm.alpha, cm.max_log2
    for s in range(1, full + 1):
        if s & (s - 1) == 0:
            continue
        if sz[s] > cap and s != full:
            continue
        out = alpha * 2.0 ** sz[s]
        low = s & -s
        cur = INF
        arg = 0
        sub = (s - 1) & s
        while sub:
            if sub & low:
                o = s ^ sub
                c = best[sub] + best[o]
                if c < cur:
                    c += 2.0 ** _pc((sm[sub] | sm[o]) & keep) + alpha * (2.0 ** sz[sub] + 2.0 ** sz[o]) + out
                    if c < cur:
                        cur, arg = c, sub
            sub = (sub - 1) & s
        best[s] = cur
        split[s] = arg
    return best[full], split


def _frontier(t: Tree, r: int, m: int, keep: int) -> List[int]:
    fr = [r]
    while len(fr) < m:
        cand = [x for x in fr if not t.is_leaf(x)]
        if not cand:
            break
        x = max(cand, key=lambda n: (_pc(t.mask[n] & keep), n))
        fr.remove(x)
        fr += [t.left[x], t.right[x]]
    return fr


def _subtree_internal(t: Tree, r: int, fr: List[int]) -> List[int]:
    stop = set(fr)
    out, stack = [], [r]
    while stack:
        n = stack.pop()
        if n in stop and n != r:
            continue
        out.append(n)
        stack += [t.left[n], t.right[n]]
    return out


def _subtree_cost(t: Tree, nodes: List[int], cm: CostModel, keep: int) -> float:
    m, L, R = t.mask, t.left, t.right
    return sum(cm.step(m[L[n]], m[R[n]], keep) for n in nodes)


def reconfigure(t: Tree, cm: CostModel, keep: int, m: int = 8, sweeps: int = 8, rng=None,
                tol: float = 1e-4) -> float:
    """Subtree reconfiguration sweeps (in place); returns the final cost."""
    cost = tree_cost(t, cm, keep)
    for _ in range(sweeps):
        nodes = t.internal()
        if rng is not None:
            rng.shuffle(nodes)
        else:
            nodes.sort(key=lambda n: -_pc(t.mask[n] & keep))
        for r in nodes:
            fr = _frontier(t, r, m, keep)
            if len(fr) < 3:
                continue
            inner = _subtree_internal(t, r, fr)
            old = _subtree_cost(t, inner, cm, keep)
            new, split = _best_tree([t.mask[x] for x in fr], cm, keep)
            if new < old * (1 - 1e-9):
                _rebuild(t, r, fr, inner, split)
        c2 = tree_cost(t, cm, keep)
        done = c2 > cost * (1 - tol)
        cost = c2
        if done:
            break
    return cost


def _rebuild(t: Tree, r: int, fr: List[int], inner: List[int], split: List[int]):
    free = [n for n in inner if n != r]
    k = len(fr)

    def build(s: int, node: Optional[int]) -> int:
        if s & (s - 1) == 0:
            return fr[s.bit_length() - 1]
        a = split[s]
        b = s ^ a
        n = node if node is not None else free.pop()
        ca = build(a, None)
        cb = build(b, None)
        t.set_children(n, ca, cb)
        return n

    build((1 << k) - 1, r)
    assert not free


# ----------------------------------------------------------------- slicing --

def slice_reconfigure(t: Tree, cm: CostModel, keep: int, sliced: List[int], m: int = 8,
                      live_cap: Optional[float] = None, live_fn=None, forbid: int = 0) -> Tuple[int, List[int]]:
    """Slice wires one at a time (the one that raises total cost least among
    the wires of the largest intermediates), reconfiguring after each, until
    every tensor fits cm.max_log2 (and live_fn(keep) <= live_cap)."""
    while True:
        sizes = [_pc(x & keep) for x in t.mask]
        mx = max(sizes)
        over_live = live_cap is not None and mx <= cm.max_log2 and live_fn(keep) > live_cap
        if mx <= cm.max_log2 and not over_live:
            return keep, sliced
        big = [n for n, s in enumerate(sizes) if s == mx]
        cw = 0
        for n in big:
            cw |= t.mask[n]
        cw &= keep & ~forbid
        if not cw:
            raise RuntimeError("cannot slice further")
        cands = []
        w = cw
        while w:
            b = w & -w
            cands.append(b)
            w ^= b
        # score: total cost after slicing (2 x the per-slice cost)
        scored = []
        for b in cands:
            k2 = keep & ~b
            scored.append((tree_cost(t, cm, k2), b))
        scored.sort()
        b = scored[0][1]
        keep &= ~b
        sliced.append(b.bit_length() - 1)
        reconfigure(t, cm, keep, m=m, sweeps=2)


# ----------------------------------------------------------- whole search --

@dataclass
class SearchResult:
    pairs: List[Tuple[int, int]]
    sliced: List[int]
    total_cost: float          # time model x slice count
    total_flops: float
    flops_per_slice: float
    log2_max: int
    peak_elems: float
    source: str


class _Net:
    """The simplified network: base tensors, their SSA ids and the
    simplification pairs (shared by every tree)."""

    def __init__(self, ns: NetworkStructure):
        g = _Greedy(ns, np.random.default_rng(0), 0.0, 1.0)
        g.simplify()
        self.ns = ns
        self.simp_pairs = list(g.pairs)
        self.base_ids = sorted(g.masks)
        self.base_masks = [g.masks[i] for i in self.base_ids]
        self.id2base = {x: i for i, x in enumerate(self.base_ids)}
        self.next_id = g.next_id
        self.open_mask = _mask(ns.open_wires)
        allw = 0
        for mk in self.base_masks:
            allw |= mk
        self.all_wires = allw

    def tree_from_pairs(self, pairs_after: Sequence[Tuple[int, int]]) -> Tree:
        """Tree from SSA pairs that continue the simplification pairs."""
        t = Tree(self.base_masks)
        node_of = dict(self.id2base)
        nid = self.next_id
        nxt = t.B
        for a, b in pairs_after:
            t.set_children(nxt, node_of.pop(a), node_of.pop(b))
            node_of[nid] = nxt
            nid += 1
            nxt += 1
        (t.root,) = node_of.values()
        return t

    def pairs_from_tree(self, t: Tree) -> List[Tuple[int, int]]:
        pairs = list(self.simp_pairs)
        sid = {i: self.base_ids[i] for i in range(t.B)}
        nid = self.next_id
        for n in t.postorder():
            pairs.append((sid[t.left[n]], sid[t.right[n]]))
            sid[n] = nid
            nid += 1
        return pairs

    def greedy_tree(self, rng, temperature: float, costmod: float) -> Tree:
        """Seeded randomized greedy over the base tensors: repeatedly
        contract the connected pair with the smallest
        size(result) - costmod (size(a) + size(b)), perturbed by Gumbel
        noise of the given temperature on a log scale."""
        import heapq
        t = Tree(self.base_masks)
        owner: Dict[int, List[int]] = {}
        live = {}
        for i, mk in enumerate(self.base_masks):
            live[i] = mk
            w = mk & ~self.open_mask
            while w:
                b = w & -w
                owner.setdefault(b, []).append(i)
                w ^= b

        def score(a, b):
            ma, mb = live[a], live[b]
            c = 2.0 ** _pc(ma ^ mb) - costmod * (2.0 ** _pc(ma) + 2.0 ** _pc(mb))
            c = math.copysign(math.log1p(abs(c)), c)
            if temperature > 0:
                c -= temperature * -math.log(-math.log(rng.random() + 1e-300) + 1e-300)
            return c

        def nbrs(a):
            out = set()
            w = live[a] & ~self.open_mask
            while w:
                b = w & -w
                out.update(owner.get(b, ()))
                w ^= b
            out.discard(a)
            return out

        heap = []
        for a in live:
            for b in nbrs(a):
                if b > a:
                    heap.append((score(a, b), a, b))
        heapq.heapify(heap)
        nxt = t.B
        while heap:
            _, a, b = heapq.heappop(heap)
            if a not in live or b not in live:
                continue
            t.set_children(nxt, a, b)
            mc = live.pop(a) ^ live.pop(b)
            live[nxt] = mc
            w = (t.mask[a] | t.mask[b]) & ~self.open_mask
            while w:
                bit = w & -w
                lst = owner.get(bit)
                if lst is not None:
                    lst[:] = [x for x in lst if x != a and x != b]
                    if mc & bit:
                        lst.append(nxt)
                w ^= bit
            for d in nbrs(nxt):
                heapq.heappush(heap, (score(nxt, d), nxt, d))
            nxt += 1
        rest = sorted(live, key=lambda x: _pc(live[x]))
        while len(rest) > 1:
            a, b = rest[0], rest[1]
            t.set_children(nxt, a, b)
            live[nxt] = live.pop(a) ^ live.pop(b)
            rest = sorted(live, key=lambda x: _pc(live[x]))
            nxt += 1
        t.root = rest[0]
        return t

    def bisection_tree(self, seed: int, lo: float, hi: float, leaf_size: int, use_kl: bool) -> Tree:
        rng = np.random.default_rng(seed)
        b = _Bisect(self.ns, rng, lo, hi, leaf_size, use_kl)
        b.simplify()
        assert b.pairs == self.simp_pairs
        b.build(sorted(b.masks))
        return self.tree_from_pairs(b.pairs[len(self.simp_pairs):])


def optimize_tree(net: _Net, t: Tree, cm: CostModel, m: int = 8, live_cap: Optional[float] = None,
                  source: str = "", initial: Sequence[int] = ()) -> SearchResult:
    """Reconfigure, slice to cm.max_log2 with reconfiguration, reconfigure
    again.  `initial`: wires sliced from the start (kept first in the
    result's sliced list)."""
    keep = net.all_wires & ~_mask(initial)
    reconfigure(t, CostModel(cm.alpha, 64), keep, m=m, sweeps=6)
    sliced: List[int] = list(initial)

    def live_fn(kp):
        pairs = net.pairs_from_tree(t)
        sl = [w for w in range(kp.bit_length() + 1) if (net.all_wires >> w) & 1 and not (kp >> w) & 1]
        return live_peak(net.ns, pairs, sl)

    keep, sliced = slice_reconfigure(t, cm, keep, sliced, m=m, live_cap=live_cap, live_fn=live_fn,
                                     forbid=net.open_mask)
    reconfigure(t, cm, keep, m=m, sweeps=6)
    pairs = net.pairs_from_tree(t)
    st = order_stats(net.ns, pairs, sliced)
    per = tree_cost(t, cm, keep)
    return SearchResult(pairs, list(sliced), per * 2.0 ** len(sliced), st.total_flops, st.flops_per_slice,
                        st.log2_max, st.peak_elems, source)
