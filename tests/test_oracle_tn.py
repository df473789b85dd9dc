"""Pins for the oracle's tensor-network contraction: agreement with the state
vector (a different algorithm), the slicing identity, bunches vs single
amplitudes, and the Supplement's Eq. (matmul) worked example by brute force."""
import itertools

import numpy as np
import pytest

import oracle
from oracle.tn import contract_slice, slice_assignment
from rqcgen import (make_rqc, network_structure, greedy_order, slice_to_fit,
                    random_bitstrings, validate_order)
from rqcgen.order import bisection_order


def _setup(rows, cols, d, seed, open_q, bits, finder="greedy", oseed=0):
    c = make_rqc(rows, cols, d, seed)
    ns = network_structure(c, open_q)
    pairs = (greedy_order(ns, seed=oseed) if finder == "greedy"
             else bisection_order(ns, seed=oseed))
    validate_order(ns, pairs)
    leaves, ow = oracle.build_network(c, open_q, bits)
    assert [list(w) for _, w in leaves] == ns.leaf_wires
    assert ow == ns.open_wires
    return c, ns, pairs, leaves, ow


@pytest.mark.parametrize("finder", ["greedy", "bisection"])
def test_tn_all_open_equals_statevector(finder):
    c, ns, pairs, leaves, ow = _setup(3, 4, 8, 0, list(range(12)), None, finder)
    a = oracle.contract_network(leaves, pairs, ow)
    psi = oracle.statevector(c).reshape(-1)
    np.testing.assert_allclose(a, psi, atol=1e-12)


def test_tn_single_amplitudes_equal_statevector():
    c = make_rqc(4, 5, 8, 0)
    psi = oracle.statevector(c).reshape(-1)
    bs = random_bitstrings(20, 4, seed=1)
    for b in bs:
        c2, ns, pairs, leaves, ow = _setup(4, 5, 8, 0, [], b)
        a = oracle.contract_network(leaves, pairs, ow)
        idx = int("".join(map(str, b)), 2)
        assert a.shape == (1,)
        assert abs(a[0] - psi[idx]) < 1e-12


def test_bunch_equals_single_amplitudes():
    open_q = [3, 7, 11]
    bits = random_bitstrings(12, 1, seed=2)[0]
    c, ns, pairs, leaves, ow = _setup(3, 4, 10, 5, open_q, bits)
    bunch = oracle.contract_network(leaves, pairs, ow)
    ref = oracle.amplitudes_sv(c, open_q, bits)
    np.testing.assert_allclose(bunch, ref, atol=1e-12)
    for y in range(8):
        b = np.array(bits)
        for j, q in enumerate(open_q):
            b[q] = (y >> (2 - j)) & 1
        c2, ns2, p2, l2, o2 = _setup(3, 4, 10, 5, [], b)
        single = oracle.contract_network(l2, p2, o2)
        assert abs(single[0] - bunch[y]) < 1e-12


def test_sum_over_slices_equals_unsliced():
    open_q = [0, 5, 10, 15, 19]
    bits = random_bitstrings(20, 1, seed=3)[0]
    c, ns, pairs, leaves, ow = _setup(4, 5, 8, 1, open_q, bits, finder="bisection")
    full = oracle.contract_network(leaves, pairs, ow)
    sliced = slice_to_fit(ns, pairs, 13)
    assert 2 <= len(sliced) <= 8
    tot = oracle.contract_sliced(leaves, pairs, ow, sliced)
    np.testing.assert_allclose(tot, full, atol=1e-12)
    # a single slice equals the sum of its sub-slices
    extra = [w for w in range(ns.n_wires) if w not in sliced and w not in ow][:2]
    s = 5 % (1 << len(sliced))
    v1 = contract_slice(leaves, pairs, ow, sliced, s)
    v2 = contract_slice(leaves, pairs, ow, sliced, s, sub_sliced=extra)
    np.testing.assert_allclose(v1, v2, atol=1e-13)
    # slices are not all equal (the fixed bonds matter)
    v0 = contract_slice(leaves, pairs, ow, sliced, 0)
    assert np.max(np.abs(v0 - v1)) > 1e-6


def test_slice_assignment_convention():
    assert slice_assignment([7, 3, 9], 0b101) == {7: 1, 3: 0, 9: 1}


def test_matmul_worked_example_bruteforce():
    """Supplement Eq. (matmul): A[a,b,c,d,e,f] x B[a,h,i,e,j] over (a, e)
    gives C[b,c,d,f,h,i,j]; checked entry by entry against explicit sums."""
    rng = np.random.default_rng(7)
    A = rng.normal(size=(2,) * 6) + 1j * rng.normal(size=(2,) * 6)
    B = rng.normal(size=(2,) * 5) + 1j * rng.normal(size=(2,) * 5)
    a_, b_, c_, d_, e_, f_, h_, i_, j_ = range(9)
    C, wc = oracle.pairwise_contract(A, [a_, b_, c_, d_, e_, f_], B, [a_, h_, i_, e_, j_])
    assert wc == [b_, c_, d_, f_, h_, i_, j_]
    for b, c, d, f, h, i, j in itertools.product(range(2), repeat=7):
        s = 0
        for a, e in itertools.product(range(2), repeat=2):
            s += A[a, b, c, d, e, f] * B[a, h, i, e, j]
        assert abs(C[b, c, d, f, h, i, j] - s) < 1e-13


def test_disconnected_network_product_state():
    c = make_rqc(2, 2, 4, seed=1, two_qubit=False)
    open_q = [0, 1, 2, 3]
    ns = network_structure(c, open_q)
    pairs = greedy_order(ns, seed=0)
    validate_order(ns, pairs)
    leaves, ow = oracle.build_network(c, open_q, None)
    a = oracle.contract_network(leaves, pairs, ow)
    np.testing.assert_allclose(a, oracle.statevector(c).reshape(-1), atol=1e-14)


def test_contract_entries_matches_pairwise():
    rng = np.random.default_rng(11)
    la, lb, lc = [4, 0, 7, 2, 9], [7, 3, 4, 1], [9, 3, 0, 2, 1]
    A = rng.normal(size=(2,) * 5) + 1j * rng.normal(size=(2,) * 5)
    B = rng.normal(size=(2,) * 4) + 1j * rng.normal(size=(2,) * 4)
    C, wc = oracle.pairwise_contract(A, la, B, lb)
    C = np.transpose(C, [wc.index(l) for l in lc])
    coords = np.array(list(itertools.product(range(2), repeat=5)))
    got = oracle.tn.contract_entries(A, la, B, lb, lc, coords)
    np.testing.assert_allclose(got, C.reshape(-1), atol=1e-13)
    # no shared index: outer product
    got = oracle.tn.contract_entries(A[..., 0, 0], [4, 0, 7], B[0, 0], [3, 1], [4, 0, 7, 3, 1],
                                     coords[:, :5])
    ref = np.einsum("abc,de->abcde", A[..., 0, 0], B[0, 0]).reshape(-1)
    np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("rows,cols,d,seed,open_q", [(2, 3, 6, 1, list(range(6))), (3, 3, 5, 2, [0, 4]),
                                                     (2, 2, 4, 3, []), (3, 4, 8, 4, list(range(12)))])
def test_gate_by_gate_order_is_a_full_tree_and_exact(rows, cols, d, seed, open_q):
    """The gate-by-gate order (used for all-open networks) validates as a
    full SSA tree and contracts to the state-vector bunch; its largest
    intermediate has at most n + 4 indices."""
    from rqcgen.order import schroedinger_order, validate_order, order_stats
    c = make_rqc(rows, cols, d, seed=seed)
    bits = random_bitstrings(c.n_qubits, 1, seed=9)[0]
    ns = network_structure(c, open_q)
    pairs = schroedinger_order(c, open_q)
    validate_order(ns, pairs)
    assert order_stats(ns, pairs, []).log2_max <= c.n_qubits + 4
    leaves, ow = oracle.build_network(c, open_q, bits)
    got = oracle.contract_network(leaves, pairs, ow, {}).reshape(-1)
    np.testing.assert_allclose(got, oracle.amplitudes_sv(c, open_q, bits), rtol=0, atol=1e-12)
