"""Host-side checks of the contraction-tree search (rqcgen.optimize): the
subset dynamic program against a brute-force recursion over all splits, the
invariants of reconfiguration and slicing, orders that the FP64 oracle
contracts to the state-vector amplitudes, and the frozen 53-qubit order."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle.tn import contract_sliced
from rqcgen import make_rqc, network_structure, random_bitstrings
from rqcgen.optimize import CostModel, _Net, _best_tree, optimize_tree, reconfigure, tree_cost
from rqcgen.order import order_stats, validate_order
from rqcgen.workloads import DATA, config3



def _brute(items, cm, keep):
    if len(items) == 1:
        return 0.0
    best = float("inf")
    first, rest = items[0], items[1:]
    n = len(rest)
    for r in range(0, n):
        for combo in itertools.combinations(range(n), r):
            left = [first] + [rest[i] for i in combo]
            right = [rest[i] for i in range(n) if i not in combo]
            ml = 0
            for x in left:
                ml ^= x
            mr = 0
            for x in right:
                mr ^= x
            c = _brute(left, cm, keep) + _brute(right, cm, keep) + cm.step(ml, mr, keep)
            best = min(best, c)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_subset_dp_is_optimal(seed):
    rng = np.random.default_rng(seed)
    k = 5
    # random graph on k tensors: each wire joins two tensors (or is open)
    masks = [0] * k
    w = 0
    for a in range(k):
        for b in range(a + 1, k):
            for _ in range(rng.integers(0, 3)):
                masks[a] |= 1 << w
                masks[b] |= 1 << w
                w += 1
        for _ in range(rng.integers(0, 2)):
            masks[a] |= 1 << w
            w += 1
    keep = (1 << w) - 1
    for alpha in (0.0, 4.0):
        cm = CostModel(alpha, 64)
        got, _ = _best_tree(masks, cm, keep)
        assert got == pytest.approx(_brute(masks, cm, keep), rel=1e-12)


def _small_net(seed=0, open_q=(0, 5)):
    c = make_rqc(3, 4, 8, seed=seed)
    ns = network_structure(c, list(open_q))
    return c, ns, _Net(ns)


def test_tree_roundtrip_and_reconfigure_monotone():
    c, ns, net = _small_net()
    t = net.bisection_tree(0, 0.4, 0.6, 4, True)
    pairs = net.pairs_from_tree(t)
    validate_order(ns, pairs)
    t2 = net.tree_from_pairs(pairs[len(net.simp_pairs):])
    assert net.pairs_from_tree(t2) == pairs
    cm = CostModel(8.0, 64)
    before = tree_cost(t, cm, net.all_wires)
    after = reconfigure(t, cm, net.all_wires, m=6, sweeps=3)
    assert after <= before * (1 + 1e-12)
    validate_order(ns, net.pairs_from_tree(t))


@pytest.mark.parametrize("bound", [6, 8])
def test_sliced_orders_contract_to_the_state_vector(bound):
    c, ns, net = _small_net(seed=2)
    open_q = [0, 5]
    t = net.bisection_tree(1, 0.4, 0.6, 4, True)
    r = optimize_tree(net, t, CostModel(8.0, bound), m=6)
    validate_order(ns, r.pairs)
    st = order_stats(ns, r.pairs, r.sliced)
    assert st.log2_max <= bound
    assert not set(r.sliced) & set(ns.open_wires)
    bits = random_bitstrings(12, 1, seed=4)[0]
    leaves, ow = oracle.build_network(c, open_q, bits)
    got = contract_sliced(leaves, r.pairs, ow, r.sliced)
    ref = oracle.amplitudes_sv(c, open_q, bits)
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_frozen_config3_order():
    w = config3()
    ns = network_structure(w.circuit, w.open_qubits)
    validate_order(ns, w.pairs)
    with open(os.path.join(DATA, "config3_order.json")) as f:
        meta = json.load(f)
    st = order_stats(ns, w.pairs, w.sliced)
    assert st.log2_max <= 32
    assert st.peak_elems <= 2.0 ** 35
    assert st.flops_per_slice == pytest.approx(meta["flops_per_slice"], rel=1e-12)
    assert not set(w.sliced) & set(ns.open_wires)
    # the measured choice among the candidates picked this order
    with open(os.path.join(DATA, "config3_order_select.json")) as f:
        sel = json.load(f)
    with open(os.path.join(DATA, "config3_candidates.json")) as f:
        cands = json.load(f)
    chosen = cands[sel["chosen"]]
    assert [tuple(p) for p in chosen["pairs"]] == [tuple(p) for p in w.pairs]
    assert chosen["sliced"] == list(w.sliced)
    assert sel["chosen"] == min(sel["timings"], key=lambda r: r["time_to_amplitudes_s"])["index"]
