"""Seeded input generators: the circuit layout rules of the Supplement's
circuit section (as read for rectangular grids), order validity and the
slicing bound."""
import numpy as np
import pytest

from rqcgen import (make_rqc, cycle_patterns, pattern_edges, network_structure, greedy_order,
                    slice_to_fit, order_stats, validate_order, make_uneven_batch, near_square_grid)
from rqcgen.order import bisection_order


def test_cycle_strings_match_printed_sequences():
    assert cycle_patterns(8) == "ABCDCDAB"
    assert cycle_patterns(12) == "ABCDCDABABCD"
    assert cycle_patterns(14) == "ABCDCDABABCDCD"


@pytest.mark.parametrize("rows,cols", [(4, 5), (6, 9), (5, 5)])
def test_patterns_are_matchings_covering_each_edge_once(rows, cols):
    present = [[True] * cols for _ in range(rows)]
    seen = {}
    for p in "ABCD":
        used = set()
        for a, b in pattern_edges(rows, cols, p, present):
            assert a not in used and b not in used
            used |= {a, b}
            seen[(a, b)] = seen.get((a, b), 0) + 1
    n_edges = rows * (cols - 1) + (rows - 1) * cols
    assert len(seen) == n_edges and set(seen.values()) == {1}


def test_missing_site_drops_its_edges():
    c = make_rqc(6, 9, 14, seed=3, n_missing=1)
    assert c.n_qubits == 53
    present_sites = set(c.sites)
    assert len(present_sites) == 53
    for g in c.gates:
        assert all(0 <= q < 53 for q in g.qubits)


def test_single_qubit_layers_no_immediate_repeat_and_seeded():
    c = make_rqc(4, 5, 12, seed=0)
    c2 = make_rqc(4, 5, 12, seed=0)
    assert [(g.name, g.qubits) for g in c.gates] == [(g.name, g.qubits) for g in c2.gates]
    last = {}
    layers = 0
    for g in c.gates:
        if len(g.qubits) == 1:
            q = g.qubits[0]
            assert last.get(q) != g.name
            last[q] = g.name
            layers += 1
    assert layers == 20 * 13
    c3 = make_rqc(4, 5, 12, seed=1)
    assert [g.name for g in c3.gates] != [g.name for g in c.gates]


def test_two_qubit_gate_count():
    c = make_rqc(4, 5, 8, seed=0)
    # 8 cycles = two full ABCD groups: every one of the 31 edges twice
    assert c.n_two_qubit == 62


@pytest.mark.parametrize("finder", ["greedy", "bisection"])
def test_orders_are_full_trees(finder):
    c = make_rqc(4, 5, 8, seed=0)
    ns = network_structure(c, [19])
    pairs = greedy_order(ns, 0) if finder == "greedy" else bisection_order(ns, 0)
    validate_order(ns, pairs)
    with pytest.raises(ValueError):
        validate_order(ns, pairs[:-1])


def test_slicer_respects_bound():
    c = make_rqc(5, 6, 10, seed=2)
    ns = network_structure(c, [0, 1, 2])
    pairs = bisection_order(ns, 0)
    for S in (12, 16, 20):
        sl = slice_to_fit(ns, pairs, S)
        st = order_stats(ns, pairs, sl)
        assert st.log2_max <= S
        assert not (set(sl) & set(ns.open_wires))


def test_uneven_batch_shapes():
    cs = make_uneven_batch(16)
    for c in cs:
        assert 24 <= c.n_qubits <= 40
        assert 10 <= c.cycles <= 20
        r, k = near_square_grid(c.n_qubits)
        assert c.rows == r and c.cols == k
