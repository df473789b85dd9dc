"""Contraction-order finder, index slicer and cost model (input side).

The paper obtains its orders from hypergraph partitioning plus slicing and
subtree reconfiguration (Supplement, section "Tensor network contraction
algorithm") with packages that are not available here.  This module is a
project-written replacement of lower quality: a seeded randomized greedy
pairwise order (the simplification rule of that section first), greedy index
slicing under a bound on the largest intermediate, and the cost model used to
score orders.  Everything here is integer/graph bookkeeping on wire sets; no
tensor values are touched.

Orders are in SSA form: step t contracts ids (pairs[t][0], pairs[t][1]) and
creates id n_leaves + t.
"""
from __future__ import annotations

import heapq
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .network import NetworkStructure


def _popcount(x: int) -> int:
    return bin(x).count("1")


def _mask(wires: Sequence[int]) -> int:
    m = 0
    for w in wires:
        m |= 1 << w
    return m


def _bits(mask: int) -> List[int]:
    out = []
    i = 0
    while mask:
        if mask & 1:
            out.append(i)
        mask >>= 1
        i += 1
    return out


@dataclass
class OrderStats:
    n_steps: int
    sliced: List[int]
    log2_max: int                # largest tensor of one slice (elements, log2)
    flops_per_slice: float       # 8 * 2^|A u B| summed over steps (complex MAC = 8 flops)
    total_flops: float           # flops_per_slice * 2^k
    peak_elems: float            # live-set peak of one slice (elements)
    k_hist: Dict[int, int] = field(default_factory=dict)   # contracted-size histogram


class _Greedy:
    def __init__(self, ns: NetworkStructure, rng: np.random.Generator,
                 temperature: float, alpha: float):
        self.ns = ns
        self.rng = rng
        self.temperature = temperature
        self.alpha = alpha
        self.open_mask = _mask(ns.open_wires)
        self.masks: Dict[int, int] = {}
        self.owners: Dict[int, set] = {}
        for i, ws in enumerate(ns.leaf_wires):
            self.masks[i] = _mask(ws)
            for w in ws:
                self.owners.setdefault(w, set()).add(i)
        self.next_id = ns.n_leaves
        self.pairs: List[Tuple[int, int]] = []

    def rank(self, t: int) -> int:
        return _popcount(self.masks[t])

    def neighbors(self, t: int) -> set:
        out = set()
        m = self.masks[t] & ~self.open_mask
        for w in _bits(m):
            out |= self.owners[w]
        out.discard(t)
        return out

    def contract(self, a: int, b: int) -> int:
        ma, mb = self.masks.pop(a), self.masks.pop(b)
        c = self.next_id
        self.next_id += 1
        mc = ma ^ mb
        for w in _bits(ma | mb):
            s = self.owners[w]
            s.discard(a)
            s.discard(b)
            if mc >> w & 1:
                s.add(c)
        self.masks[c] = mc
        self.pairs.append((a, b))
        return c

    def simplify(self):
        """Absorb rank-1/rank-2 tensors, and pre-contract pairs whose result
        rank is not above the larger operand rank (Supplement, TNC section)."""
        changed = True
        while changed:
            changed = False
            small = sorted(t for t in self.masks if self.rank(t) <= 2)
            for t in small:
                if t not in self.masks or self.rank(t) > 2:
                    continue
                nb = self.neighbors(t)
                if not nb:
                    continue
                u = max(nb, key=lambda x: (self.rank(x), -x))
                self.contract(t, u)
                changed = True
            for t in sorted(self.masks):
                if t not in self.masks:
                    continue
                for u in sorted(self.neighbors(t)):
                    if u not in self.masks or t not in self.masks:
                        continue
                    rc = _popcount(self.masks[t] ^ self.masks[u])
                    if rc <= max(self.rank(t), self.rank(u)) and min(self.rank(t), self.rank(u)) > 2:
                        self.contract(t, u)
                        changed = True
                        break

    def cost(self, a: int, b: int) -> float:
        ma, mb = self.masks[a], self.masks[b]
        sc = 2.0 ** _popcount(ma ^ mb)
        c = sc - self.alpha * (2.0 ** _popcount(ma) + 2.0 ** _popcount(mb))
        if self.temperature > 0:
            g = -math.log(-math.log(self.rng.random() + 1e-300) + 1e-300)
            # perturb on a log scale, keeping the sign
            c = math.copysign(math.log1p(abs(c)), c) - self.temperature * g
        return c

    def run(self):
        self.simplify()
        heap = []
        counter = 0
        for t in sorted(self.masks):
            for u in sorted(self.neighbors(t)):
                if u > t:
                    heapq.heappush(heap, (self.cost(t, u), counter, t, u))
                    counter += 1
        while heap:
            _, _, a, b = heapq.heappop(heap)
            if a not in self.masks or b not in self.masks:
                continue
            c = self.contract(a, b)
            for d in sorted(self.neighbors(c)):
                heapq.heappush(heap, (self.cost(c, d), counter, c, d))
                counter += 1
        # disconnected pieces: outer products, smallest first
        while len(self.masks) > 1:
            ts = sorted(self.masks, key=lambda t: (self.rank(t), t))
            self.contract(ts[0], ts[1])
        return self.pairs


def greedy_order(ns: NetworkStructure, seed: int = 0, temperature: float = 0.0,
                 alpha: float = 1.0) -> List[Tuple[int, int]]:
    """Seeded greedy pairwise order over the canonical leaves (SSA pairs)."""
    rng = np.random.default_rng(seed)
    return _Greedy(ns, rng, temperature, alpha).run()


def step_masks(ns: NetworkStructure, pairs: Sequence[Tuple[int, int]]):
    """Per step (mask A, mask B, mask C) as python ints over wire ids."""
    masks = [_mask(ws) for ws in ns.leaf_wires]
    out = []
    for a, b in pairs:
        ma, mb = masks[a], masks[b]
        mc = ma ^ mb
        masks.append(mc)
        out.append((ma, mb, mc))
    return out


def validate_order(ns: NetworkStructure, pairs: Sequence[Tuple[int, int]]) -> None:
    n = ns.n_leaves
    if len(pairs) != n - 1:
        raise ValueError(f"order has {len(pairs)} steps, expected {n - 1}")
    used = set()
    for t, (a, b) in enumerate(pairs):
        for x in (a, b):
            if not 0 <= x < n + t or x in used:
                raise ValueError(f"step {t}: bad or reused id {x}")
            used.add(x)
        if a == b:
            raise ValueError(f"step {t}: self contraction")


def order_stats(ns: NetworkStructure, pairs, sliced: Sequence[int] = ()) -> OrderStats:
    sm = step_masks(ns, pairs)
    smask = _mask(sliced)
    flops = 0.0
    lmax = 0
    khist: Dict[int, int] = {}
    for ma, mb, mc in sm:
        u = (ma | mb) & ~smask
        flops += 8.0 * 2.0 ** _popcount(u)
        lmax = max(lmax, _popcount(mc & ~smask), _popcount(ma & ~smask), _popcount(mb & ~smask))
        kk = _popcount(ma & mb & ~smask)
        khist[kk] = khist.get(kk, 0) + 1
    peak = live_peak(ns, pairs, sliced)
    k = len(sliced)
    return OrderStats(len(pairs), list(sliced), lmax, flops, flops * 2.0 ** k, peak, khist)


def live_peak(ns: NetworkStructure, pairs, sliced: Sequence[int] = ()) -> float:
    """Peak of the summed sizes of live intermediates (leaves excluded),
    counting both operands and the result of the running step."""
    smask = _mask(sliced)
    n = ns.n_leaves
    masks = [_mask(ws) for ws in ns.leaf_wires]
    size = {}
    live = 0.0
    peak = 0.0
    for t, (a, b) in enumerate(pairs):
        mc = masks[a] ^ masks[b]
        masks.append(mc)
        sc = 2.0 ** _popcount(mc & ~smask)
        peak = max(peak, live + sc)
        for x in (a, b):
            if x >= n:
                live -= size.pop(x)
        size[n + t] = sc
        live += sc
    return peak


def slice_to_fit(ns: NetworkStructure, pairs, max_log2: int,
                 max_live_elems: Optional[float] = None,
                 exclude: Sequence[int] = (), initial: Sequence[int] = ()) -> List[int]:
    """Greedy index slicing: repeatedly slice the wire that minimizes the total
    flop count (per-slice cost x number of slices) among the wires of the
    largest intermediates, until every tensor of one slice has at most
    2^max_log2 elements (and, optionally, the live-set peak fits)."""
    sm = step_masks(ns, pairs)
    n_steps = len(sm)
    open_mask = _mask(ns.open_wires) | _mask(exclude)
    all_wires = 0
    for ma, mb, mc in sm:
        all_wires |= ma | mb
    wires = [w for w in _bits(all_wires & ~open_mask)]
    widx = {w: i for i, w in enumerate(wires)}
    U = np.zeros((n_steps, len(wires)), dtype=bool)   # wire in A u B
    C = np.zeros((n_steps, len(wires)), dtype=bool)   # wire in C
    urank = np.zeros(n_steps, dtype=np.int64)
    crank = np.zeros(n_steps, dtype=np.int64)
    for i, (ma, mb, mc) in enumerate(sm):
        for w in _bits((ma | mb) & ~open_mask):
            U[i, widx[w]] = True
        for w in _bits(mc & ~open_mask):
            C[i, widx[w]] = True
        urank[i] = _popcount(ma | mb)
        crank[i] = _popcount(mc)
    sliced: List[int] = list(initial)
    sl = np.zeros(len(wires), dtype=bool)
    for w in initial:
        if w in widx:
            sl[widx[w]] = True
    while True:
        ur = urank - U[:, sl].sum(axis=1)
        cr = crank - C[:, sl].sum(axis=1)
        cmax = int(cr.max()) if n_steps else 0
        over_size = cmax > max_log2
        over_live = False
        if max_live_elems is not None and not over_size:
            over_live = live_peak(ns, pairs, sliced) > max_live_elems
        if not (over_size or over_live):
            return sliced
        big = cr == cmax
        cand = np.where(C[big].any(axis=0) & ~sl)[0]
        if cand.size == 0:
            raise RuntimeError("cannot slice further")
        f = 2.0 ** ur
        base = f.sum()
        # total flops after slicing w: 2 * (base - 0.5 * sum_{w in step} f)
        red = (U[:, cand] * f[:, None]).sum(axis=0)
        tot = 2.0 * (base - 0.5 * red)
        nbig = (C[big][:, cand]).sum(axis=0)
        key = np.lexsort((-nbig, tot))
        w = int(cand[key[0]])
        sl[w] = True
        sliced.append(wires[w])


@dataclass
class Plan:
    pairs: List[Tuple[int, int]]
    sliced: List[int]
    stats: OrderStats
    seed: int


def find_order(ns: NetworkStructure, max_log2: int, restarts: int = 32, seed: int = 0,
               max_live_elems: Optional[float] = None,
               temperatures: Sequence[float] = (0.0, 0.25, 0.5, 1.0)) -> Plan:
    """Best of several seeded greedy orders, each sliced to fit; scored by
    total flops (per-slice flops x slice count), ties by per-slice flops."""
    best = None
    for r in range(restarts):
        temp = temperatures[r % len(temperatures)] if r else 0.0
        pairs = greedy_order(ns, seed=seed * 100003 + r, temperature=temp)
        sliced = slice_to_fit(ns, pairs, max_log2, max_live_elems)
        st = order_stats(ns, pairs, sliced)
        key = (st.total_flops, st.flops_per_slice)
        if best is None or key < best[0]:
            best = (key, Plan(pairs, sliced, st, seed * 100003 + r))
    return best[1]


def _fiedler_split(nodes: List[int], adj: Dict[int, Dict[int, int]], lo: float, hi: float,
                   rng: np.random.Generator) -> Tuple[List[int], List[int]]:
    """Balanced bisection: sweep cut along the Fiedler vector of the induced
    subgraph's weighted Laplacian, cut chosen in the [lo, hi] size window."""
    n = len(nodes)
    pos = {v: i for i, v in enumerate(nodes)}
    L = np.zeros((n, n))
    for v in nodes:
        i = pos[v]
        for u, w in adj[v].items():
            j = pos.get(u)
            if j is not None:
                L[i, j] -= w
                L[i, i] += w
    # tiny random diagonal jitter breaks ties between equivalent splits
    L += np.diag(rng.random(n) * 1e-9)
    vals, vecs = np.linalg.eigh(L)
    f = vecs[:, 1]
    order = [nodes[i] for i in np.argsort(f, kind="stable")]
    left = set()
    cut = 0
    best = None
    a, b = max(1, int(math.floor(lo * n))), min(n - 1, int(math.ceil(hi * n)))
    for i in range(1, n):
        v = order[i - 1]
        wl = sum(w for u, w in adj[v].items() if u in left)
        wall = sum(w for u, w in adj[v].items() if u in pos)
        cut += (wall - wl) - wl
        left.add(v)
        if a <= i <= b:
            key = (cut, abs(2 * i - n))
            if best is None or key < best[0]:
                best = (key, i)
    i = best[1]
    return order[:i], order[i:]


def _kl_refine(nodes1, nodes2, adj, seed):
    import networkx as nx
    from networkx.algorithms.community import kernighan_lin_bisection
    G = nx.Graph()
    allv = set(nodes1) | set(nodes2)
    G.add_nodes_from(allv)
    for v in allv:
        for u, w in adj[v].items():
            if u in allv and u > v:
                G.add_edge(v, u, weight=w)
    p1, p2 = kernighan_lin_bisection(G, partition=(set(nodes1), set(nodes2)),
                                     weight="weight", seed=seed, max_iter=20)
    return sorted(p1), sorted(p2)


class _Bisect(_Greedy):
    """Recursive bisection of the simplified network into a contraction tree."""

    def __init__(self, ns, rng, lo, hi, leaf_size, use_kl):
        super().__init__(ns, rng, 0.0, 1.0)
        self.lo, self.hi = lo, hi
        self.leaf_size = leaf_size
        self.use_kl = use_kl

    def adjacency(self, nodes):
        adj = {v: {} for v in nodes}
        for v in nodes:
            for u in self.neighbors(v):
                if u in adj:
                    adj[v][u] = _popcount(self.masks[v] & self.masks[u])
        return adj

    def small_greedy(self, nodes: List[int]) -> int:
        live = list(nodes)
        while len(live) > 1:
            best = None
            for i in range(len(live)):
                for j in range(i + 1, len(live)):
                    ma, mb = self.masks[live[i]], self.masks[live[j]]
                    shared = ma & mb
                    rc = _popcount(ma ^ mb)
                    key = (0 if shared else 1, rc, _popcount(ma | mb))
                    if best is None or key < best[0]:
                        best = (key, i, j)
            _, i, j = best
            c = self.contract(live[i], live[j])
            live = [x for k, x in enumerate(live) if k not in (i, j)] + [c]
        return live[0]

    def components(self, nodes, adj):
        seen, comps = set(), []
        for v in nodes:
            if v in seen:
                continue
            stack, comp = [v], []
            seen.add(v)
            while stack:
                x = stack.pop()
                comp.append(x)
                for u in adj[x]:
                    if u not in seen:
                        seen.add(u)
                        stack.append(u)
            comps.append(sorted(comp))
        return comps

    def build(self, nodes: List[int]) -> int:
        if len(nodes) <= self.leaf_size:
            return self.small_greedy(nodes)
        adj = self.adjacency(nodes)
        comps = self.components(nodes, adj)
        if len(comps) > 1:
            comps.sort(key=len, reverse=True)
            g1, g2 = [], []
            for c in comps:
                (g1 if len(g1) <= len(g2) else g2).extend(c)
            n1, n2 = sorted(g1), sorted(g2)
        else:
            n1, n2 = _fiedler_split(nodes, adj, self.lo, self.hi, self.rng)
            if self.use_kl and len(nodes) > 4:
                n1, n2 = _kl_refine(n1, n2, adj, int(self.rng.integers(1 << 30)))
        a = self.build(n1)
        b = self.build(n2)
        return self.contract(a, b)

    def run(self):
        self.simplify()
        self.build(sorted(self.masks))
        return self.pairs


def bisection_order(ns: NetworkStructure, seed: int = 0, lo: float = 0.4, hi: float = 0.6,
                    leaf_size: int = 8, use_kl: bool = True) -> List[Tuple[int, int]]:
    """Seeded recursive-bisection order (spectral sweep cut + Kernighan-Lin),
    the simplification rule applied first."""
    rng = np.random.default_rng(seed)
    return _Bisect(ns, rng, lo, hi, leaf_size, use_kl).run()


def schroedinger_order(circuit, open_qubits: Sequence[int] = ()) -> List[Tuple[int, int]]:
    """Gate-by-gate (state-vector-like) SSA order over the canonical leaves:
    each qubit's |0> vector and the single-qubit gates between two two-qubit
    gates are first contracted into the next two-qubit gate (small steps),
    then every such block is contracted into the running state in circuit
    order; trailing single-qubit gates and the output vectors of closed
    qubits follow, and disjoint components are joined last.  The state has
    at most n indices, so this order suits networks with many open qubits,
    where graph-partitioning orders are poor."""
    n = circuit.n_qubits
    m = len(circuit.gates)
    open_set = set(int(q) for q in open_qubits)
    closed = [q for q in range(n) if q not in open_set]
    pairs: List[Tuple[int, int]] = []
    next_id = n + m + len(closed)

    def contract(a: int, b: int) -> int:
        nonlocal next_id
        pairs.append((a, b))
        next_id += 1
        return next_id - 1

    pending: List[Optional[int]] = list(range(n))   # small tensor not yet in the state, per qubit
    comp: Dict[int, int] = {}                         # qubit -> id of the state component holding it
    members: Dict[int, List[int]] = {}                # component id -> its qubits

    def merge_into_state(block: int, qubits: Sequence[int]):
        cur = block
        qs: List[int] = []
        seen = set()
        for q in qubits:
            c = comp.get(q)
            if c is not None and c not in seen:
                seen.add(c)
                cur = contract(c, cur)
                qs += members.pop(c)
        for q in qubits:
            if q not in qs:
                qs.append(q)
        members[cur] = qs
        for q in qs:
            comp[q] = cur

    for gi, g in enumerate(circuit.gates):
        leaf = n + gi
        if len(g.qubits) == 1:
            q = g.qubits[0]
            pending[q] = leaf if pending[q] is None else contract(pending[q], leaf)
            continue
        block = leaf
        for q in g.qubits:
            if pending[q] is not None:
                block = contract(block, pending[q])
                pending[q] = None
        merge_into_state(block, list(g.qubits))
    for j, q in enumerate(closed):
        out_leaf = n + m + j
        pending[q] = out_leaf if pending[q] is None else contract(pending[q], out_leaf)
    for q in range(n):
        if pending[q] is not None:
            merge_into_state(pending[q], [q])
            pending[q] = None
    roots = list(members)
    cur = roots[0]
    for r in roots[1:]:
        cur = contract(cur, r)
    return pairs
