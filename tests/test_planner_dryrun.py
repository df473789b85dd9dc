"""The C++ planner on the CPU (dry-run plans, no device): its step list, run
by a NumPy interpreter over stand-in device regions, reproduces the oracle.
Also the C ABI's argument validation and exported symbols."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2111_01066_amd import tnrcs
from rqcgen import (make_rqc, network_structure, greedy_order, slice_to_fit, random_bitstrings,
                    Circuit, Gate)
from rqcgen.order import bisection_order
from tests.plan_interp import PlanInterpreter

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_plan(plan, n_slices, n_open):
    it = PlanInterpreter(plan)
    amp = np.zeros(1 << n_open, dtype=np.complex128)
    for s in range(n_slices):
        it.run_slice(s, amp)
    return amp


CASES = [
    # rows, cols, d, seed, open, finder, S, fold
    (4, 5, 8, 0, list(range(20)), "bisection", 40, 12),
    (4, 5, 8, 0, list(range(20)), "greedy", 40, 12),
    (4, 5, 8, 0, [], "bisection", 40, 12),
    (3, 4, 8, 1, [0, 5, 11], "bisection", 10, 12),
    (3, 4, 8, 1, [0, 5, 11], "greedy", 8, 4),
    (3, 4, 6, 2, [2, 3], "bisection", 9, 0),
    (2, 3, 10, 3, list(range(6)), "greedy", 40, 20),
]


@pytest.mark.parametrize("rows,cols,d,seed,open_q,finder,S,fold", CASES)
def test_dryrun_plan_matches_oracle(rows, cols, d, seed, open_q, finder, S, fold):
    c = make_rqc(rows, cols, d, seed)
    bits = random_bitstrings(c.n_qubits, 1, seed=seed + 100)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0) if finder == "bisection" else greedy_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, S)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dry_run=True, host_fold_log2=fold)
    info = plan.info()
    assert info["n_slices"] == 1 << len(sliced)
    assert info["n_host_steps"] + info["n_device_steps"] == len(pairs)
    amp = _run_plan(plan, info["n_slices"], len(open_q))
    ref = oracle.amplitudes_sv(c, open_q, bits)
    np.testing.assert_allclose(amp, ref, atol=1e-12)
    plan.close()


@pytest.mark.parametrize("dtype", ["c64", "f16s"])
@pytest.mark.parametrize("d,open_q,S", [(12, [], 22), (10, [0, 1, 2, 3, 4, 5], 20)])
def test_dryrun_dense_steps_present(d, open_q, S, dtype):
    c = make_rqc(4, 5, d, 5)
    bits = random_bitstrings(20, 1, seed=8)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, S)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dry_run=True, dtype=dtype)
    info = plan.info()
    assert info["n_dense"] > 0
    amp = _run_plan(plan, info["n_slices"], len(open_q))
    ref = oracle.amplitudes_sv(c, open_q, bits)
    np.testing.assert_allclose(amp, ref, atol=1e-12)


def test_single_leaf_and_tiny_networks():
    # one qubit, no gates, open: the amplitude vector is |0>
    c = Circuit(1, [])
    plan = tnrcs.Plan(c, [], [], [0], None, dry_run=True)
    np.testing.assert_allclose(_run_plan(plan, 1, 1), [1, 0])
    # one qubit, one gate, closed at 1
    c = Circuit(1, [Gate("sqrt_x", (0,), (), oracle.sqrt_x())])
    plan = tnrcs.Plan(c, [(0, 1), (3, 2)], [], [], [1], dry_run=True)
    np.testing.assert_allclose(_run_plan(plan, 1, 0), [-1j / np.sqrt(2)], atol=1e-15)


def test_set_output_bits_rebinds():
    c = make_rqc(3, 3, 6, 7)
    ns = network_structure(c, [4])
    pairs = bisection_order(ns, seed=0)
    b1 = random_bitstrings(9, 2, seed=3)
    plan = tnrcs.Plan(c, pairs, [], [4], b1[0], dry_run=True)
    np.testing.assert_allclose(_run_plan(plan, 1, 1), oracle.amplitudes_sv(c, [4], b1[0]), atol=1e-12)
    plan.set_output_bits(b1[1])
    np.testing.assert_allclose(_run_plan(plan, 1, 1), oracle.amplitudes_sv(c, [4], b1[1]), atol=1e-12)


def test_errors():
    c = make_rqc(2, 2, 4, 0)
    ns = network_structure(c, [0])
    pairs = greedy_order(ns, 0)
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs[:-1], [], [0], None, dry_run=True)
    assert e.value.code == -2
    bad = list(pairs)
    bad[-1] = (bad[-1][0], bad[-1][0])
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, bad, [], [0], None, dry_run=True)
    assert e.value.code == -2
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs, [ns.open_wires[0]], [0], None, dry_run=True)
    assert e.value.code == -1
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs, [10**6], [0], None, dry_run=True)
    assert e.value.code == -2
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs, [], [0, 0], None, dry_run=True)
    assert e.value.code == -1
    plan = tnrcs.Plan(c, pairs, [], [0], None, dry_run=True)
    with pytest.raises(tnrcs.TnError) as e:
        plan.contract(0, 1, 0, stream=0)
    assert e.value.code == -5


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tnrcs.h")).read()
    declared = set(re.findall(r"^(?:int|int64_t|void|const char\*)\s+(tn_\w+)\s*\(", header, flags=re.M))
    assert len(declared) >= 15
    lib = ctypes.CDLL(tnrcs.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(tnrcs.EXPORTED)


def test_batch_argument_checks_without_device():
    c = make_rqc(3, 4, 8, seed=1)
    ns = network_structure(c, [0])
    pairs = greedy_order(ns, seed=0)
    plan = tnrcs.Plan(c, pairs, [], [0], None, dry_run=True)
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Batch([plan], [(0, 1)], [0])
    assert e.value.code == -5
    with pytest.raises(ValueError):
        tnrcs.Batch([plan], [], [])
    # an empty batch is valid and launches nothing
    b = tnrcs.Batch([], [], [])
    b.run(stream=0)
    b.close()


def test_tuning_reserves_split_workspace_in_the_plan():
    c = make_rqc(4, 5, 12, seed=5)
    open_q = list(range(20))
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, 24)
    base = tnrcs.Plan(c, pairs, sliced, open_q, None, dry_run=True)
    tuned = tnrcs.Plan(c, pairs, sliced, open_q, None, dry_run=True, tune=True)
    g0 = [o for o in base.json()["ops"] if o["kind"] == 1]
    g1 = [o for o in tuned.json()["ops"] if o["kind"] == 1]
    assert len(g0) == len(g1) > 0
    for a, b in zip(g0, g1):
        assert (a["M"], a["N"], a["K"], a["split_k"]) == (b["M"], b["N"], b["K"], b["split_k"])
        assert a["split_max"] == a["split_k"] or a["split_k"] == 1
        assert b["split_max"] >= b["split_k"]
        # split slabs stay at least 256 deep and the workspace at most 2^28 entries
        if b["split_max"] > 1:
            assert b["K"] // b["split_max"] >= 256 and b["split_max"] * b["M"] * b["N"] <= 2 ** 28
    assert tuned.info()["arena_bytes"] >= base.info()["arena_bytes"]


def test_shift_outputs_on_dry_run_plan():
    c = make_rqc(3, 4, 8, seed=1)
    open_q = [0, 5, 11]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    plan = tnrcs.Plan(c, pairs, [], open_q, None, dtype="f16s", dry_run=True)
    before = [o["s_out"] for o in plan.json()["ops"] if o["kind"] != 0]
    plan.shift_outputs(3)
    after = [o["s_out"] for o in plan.json()["ops"] if o["kind"] != 0]
    assert before and after == [s + 3 for s in before]
    ops = plan.json()["ops"]
    i = next(j for j, o in enumerate(ops) if o["kind"] != 0)
    plan.shift_outputs(-2, op=i)
    assert plan.json()["ops"][i]["s_out"] == ops[i]["s_out"] - 2
    with pytest.raises(tnrcs.TnError):
        plan.shift_outputs(100)
    with pytest.raises(tnrcs.TnError):
        plan.shift_outputs(1, op=len(ops))
    perm = [j for j, o in enumerate(ops) if o["kind"] == 0]
    if perm:
        with pytest.raises(tnrcs.TnError):
            plan.shift_outputs(1, op=perm[0])


def _valid(nM, nN, nK):
    v = {2}
    if nM >= 6 and nN >= 6 and nK >= 4:
        v.add(1)
    if (nM + nN <= 6 and nK >= 4) or (nM + nN <= 12 and nK >= 12):
        v.add(4)
    if nN <= 4 and nK + nN <= 11 and nM >= 8:
        v.add(3)
    if nN <= 6 and 1 <= nK <= 10 and nM >= 7:
        v.add(5)
    return v


def _class_candidates(st):
    nM, nN, nK = st["nM"], st["nN"], st["nK"]
    v = _valid(nM, nN, nK)
    big = nM + nN > 22 or nK >= 16  # the gathered kernel is not timed on large steps or long sums
    if 1 in v:
        if nK > 6:
            return []
        c = {1} | (v & {5}) | (set() if big else {2})
    else:
        c = v & {2, 3, 4, 5}
        if big and c != {2}:
            c.discard(2)
    return sorted(c) if len(c) > 1 else []


def _default_class(st):
    nM, nN, nK = st["nM"], st["nN"], st["nK"]
    v = _valid(nM, nN, nK)
    if 1 in v and (nK >= 7 or nN >= 7 or 5 not in v):
        return 1
    if 4 in v and nK >= 10:
        return 4
    if 3 in v and nK + nN <= 4:
        return 3
    for k in (5, 3):
        if k in v:
            return k
    return 2


@pytest.mark.parametrize("dtype", ["c64", "f16s"])
@pytest.mark.parametrize("d,n_open,S,alt", [(8, 15, 16, 2), (12, 6, 15, 4)])
def test_step_classes_default_rule_and_forced_classes(tmp_path, dtype, d, n_open, S, alt):
    """Each device step's kernel class follows the planner's rule; class
    lines in a tuning database replace it (a dry-run plan applies them
    without timing), the forced plan still computes the amplitudes, and a
    line naming a class that the step does not admit is ignored.  Networks
    on 3x5 qubits where the alternative is the gathered kernel in place of
    permutes + GEMM (alt 2) or split-K in place of the gathered kernel
    (alt 4)."""
    c = make_rqc(3, 5, d, 0)
    open_q = list(range(15 - n_open, 15))
    bits = random_bitstrings(15, 1, seed=4)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, S)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dry_run=True, dtype=dtype)
    steps = plan.json()["steps"]
    assert len(steps) == plan.info()["n_device_steps"]
    for st in steps:
        assert st["cls"] == _default_class(st) and not st["tuned"]
        a, b, cc = (list(map(int, part.split("."))) if part else [] for part in st["key"].split("/"))
        assert a == list(range(len(a)))  # relabelled by first appearance
        assert len(cc) == st["nM"] + st["nN"] and len(set(a) & set(b)) == st["nK"]
    forced = {st["key"]: [k for k in _class_candidates(st) if k != st["cls"]][0]
              for st in steps if _class_candidates(st)}
    assert alt in forced.values()
    fixed = [st for st in steps if st["key"] not in forced]
    plan.close()
    code = {"c64": 0, "f16s": 1}[dtype]
    db = tmp_path / "tune.txt"
    with open(db, "w") as f:
        for key, k in forced.items():
            f.write(f"tnrcs-class {code} {key} {k} 0.0\n")
        for st in fixed:  # not admitted (no such class): ignored
            f.write(f"tnrcs-class {code} {st['key']} 9 0.0\n")
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dry_run=True, dtype=dtype, tune=True, tune_db=str(db))
    for st in plan.json()["steps"]:
        if st["key"] in forced:
            assert st["tuned"] and st["cls"] == forced[st["key"]]
        else:
            assert st["cls"] == _default_class(st)
    amp = _run_plan(plan, plan.info()["n_slices"], n_open)
    ref = oracle.amplitudes_sv(c, open_q, bits)
    np.testing.assert_allclose(amp, ref, atol=1e-12)
    plan.close()
