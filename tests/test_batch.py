"""Batches of plans (one captured graph over many circuits), plans sharing one
arena workspace, and the GEMM autotuner, on the GPU through the C ABI:
against per-plan runs of the same plans (bitwise: same kernels, same order)
and against the FP64 oracle."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.tn import build_network, contract_sliced  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen import make_rqc, make_uneven_batch, network_structure, random_bitstrings, slice_to_fit  # noqa: E402
from rqcgen.order import bisection_order  # noqa: E402
from rqcgen.workloads import config5, config5_table  # noqa: E402

DEV = "cuda"
TOL = {"c64": 1e-5, "f16s": 1e-2, "bf16s": 6e-2}


def _small_batch(count=8, s_max=9):
    """Small uneven circuits (10..18 qubits, 6..12 cycles), each sliced to
    between 1 and 8 wires, with state-vector references."""
    out = []
    for i, c in enumerate(make_uneven_batch(count, seed0=2000, n_range=(10, 18), d_range=(6, 12))):
        open_q = list(range(c.n_qubits - 6, c.n_qubits))
        bits = random_bitstrings(c.n_qubits, 1, seed=3000 + i)[0]
        ns = network_structure(c, open_q)
        pairs = bisection_order(ns, seed=0)
        S = s_max
        while len(slice_to_fit(ns, pairs, S)) > 8:
            S += 1
        sliced = slice_to_fit(ns, pairs, S)
        out.append((c, open_q, bits, pairs, sliced, oracle.amplitudes_sv(c, open_q, bits)))
    return out


@pytest.fixture(scope="module")
def small():
    return _small_batch()


def _shared_plans(cases, dtype, tune=False, tune_db=None, workspaces=1):
    """Plans on `workspaces` arena workspaces, dealt round-robin (plans on
    different workspaces go to different lanes of a batch graph)."""
    need = 0
    for c, open_q, bits, pairs, sliced, _ in cases:
        dry = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, dry_run=True, tune=tune)
        need = max(need, dry.info()["arena_bytes"])
        dry.close()
    ws = [torch.empty(max(need, 256), dtype=torch.uint8, device=DEV) for _ in range(workspaces)]
    plans = [tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, arena=ws[i % workspaces], tune=tune,
                        tune_db=tune_db)
             for i, (c, open_q, bits, pairs, sliced, _) in enumerate(cases)]
    return plans, ws


@pytest.mark.parametrize("workspaces", [1, 3])
@pytest.mark.parametrize("dtype", ["c64", "f16s"])
def test_batch_matches_per_plan_runs_and_oracle(small, dtype, workspaces):
    print(f"batch of {len(small)} small uneven circuits, {dtype}, {workspaces} arena workspace(s)", flush=True)
    plans, ws = _shared_plans(small, dtype, workspaces=workspaces)
    n_sl = [p.info()["n_slices"] for p in plans]
    assert any(n > 1 for n in n_sl)
    seq = [torch.zeros(64, dtype=torch.complex128, device=DEV) for _ in plans]
    for p, a, n in zip(plans, seq, n_sl):
        p.contract(0, n, a)
    torch.cuda.synchronize()
    amps = [torch.zeros(64, dtype=torch.complex128, device=DEV) for _ in plans]
    b = tnrcs.Batch(plans, [(0, n) for n in n_sl], amps)
    b.run()
    torch.cuda.synchronize()
    for i, (p, a, s) in enumerate(zip(plans, amps, seq)):
        got = a.cpu().numpy()
        assert np.array_equal(got, s.cpu().numpy()), i
        err = oracle.relative_error_norm(got, small[i][5])
        assert err < TOL[dtype], (i, err)
        assert p.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    # a second launch accumulates the same sums again, exactly as a second
    # round of per-plan runs does
    b.run()
    for p, a, n in zip(plans, seq, n_sl):
        p.contract(0, n, a)
    torch.cuda.synchronize()
    for a, s in zip(amps, seq):
        got, ref = a.cpu().numpy(), s.cpu().numpy()
        assert np.array_equal(got, ref)
    for i, a in enumerate(amps):
        err = oracle.relative_error_norm(a.cpu().numpy() / 2, small[i][5])
        assert err < TOL[dtype], (i, err)
    b.close()
    for p in plans:
        p.close()
    del ws


def test_batch_split_ranges_repeated_plans_and_one_shot(small):
    print("batch split ranges / repeated plans / one-shot", flush=True)
    cases = small[:3]
    plans, ws = _shared_plans(cases, "c64")
    n_sl = [p.info()["n_slices"] for p in plans]
    ref = [torch.zeros(64, dtype=torch.complex128, device=DEV) for _ in plans]
    for p, a, n in zip(plans, ref, n_sl):
        p.contract(0, n, a)
    # every plan twice, its range split in two, both halves into one buffer
    entries, ranges, amps = [], [], []
    out = [torch.zeros(64, dtype=torch.complex128, device=DEV) for _ in plans]
    for p, a, n in zip(plans, out, n_sl):
        h = n // 2
        entries += [p, p]
        ranges += [(0, h), (h, n)]
        amps += [a, a]
    tnrcs.tn_contract_batch(entries, ranges, amps)
    for a, r in zip(out, ref):
        assert np.array_equal(a.cpu().numpy(), r.cpu().numpy())
    # empty ranges are allowed and do nothing
    z = torch.zeros(64, dtype=torch.complex128, device=DEV)
    tnrcs.tn_contract_batch(plans[:1], [(1, 1)], [z])
    assert not z.abs().sum().item()
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Batch(plans[:1], [(0, n_sl[0] + 1)], [z])
    assert e.value.code == -1
    for p in plans:
        p.close()
    del ws


def test_arena_workspace_errors():
    c = make_rqc(4, 5, 8, seed=1)
    open_q = [0, 5, 11, 19]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    bits = random_bitstrings(20, 1, seed=2)[0]
    need = tnrcs.Plan(c, pairs, [], open_q, bits, dry_run=True).info()["arena_bytes"]
    assert need > 4096
    ws = torch.empty(need + 512, dtype=torch.uint8, device=DEV)
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs, [], open_q, bits, arena=ws[: need - 256])
    assert e.value.code == -3
    with pytest.raises(tnrcs.TnError) as e:
        tnrcs.Plan(c, pairs, [], open_q, bits, arena=int(ws.data_ptr()) + 8, arena_bytes=need)
    assert e.value.code == -1
    p = tnrcs.Plan(c, pairs, [], open_q, bits, arena=ws)
    a = torch.zeros(16, dtype=torch.complex128, device=DEV)
    p.contract(0, 1, a)
    torch.cuda.synchronize()
    ref = oracle.amplitudes_sv(c, open_q, bits)
    assert oracle.relative_error_norm(a.cpu().numpy(), ref) < TOL["c64"]
    p.close()


@pytest.mark.parametrize("dtype", ["c64", "f16s"])
def test_tuned_plan_vs_oracle_and_cache(tmp_path, dtype):
    c = make_rqc(4, 5, 12, seed=5)
    open_q = list(range(20))
    bits = np.zeros(20, dtype=np.uint8)
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, 24)
    db = str(tmp_path / "tune.txt")
    print(f"tuned 4x5 d=12 all open {dtype}", flush=True)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, tune=True, tune_db=db)
    gemms = [o for o in plan.json()["ops"] if o["kind"] == 1]
    assert gemms and all(o["tile"] in (64, 128) for o in gemms)
    assert all(1 <= o["split_k"] <= max(1, o["split_max"]) for o in gemms)
    lines = open(db).read().split("\n")
    # GEMM shapes of the plan and of the one-step plans the class tuner timed
    assert sum(ln.startswith("tnrcs-gemm") for ln in lines) >= len({(o["M"], o["N"], o["K"]) for o in gemms})
    # every step with more than one candidate class was timed once per key
    steps = plan.json()["steps"]
    tuned = [st for st in steps if st["tuned"]]
    assert {st["key"] for st in tuned} == {st["key"] for st in steps if _candidates(st)}
    cls_lines = [ln.split() for ln in lines if ln.startswith("tnrcs-class")]
    assert sorted(ln[2] for ln in cls_lines) == sorted({st["key"] for st in tuned})
    for st in tuned:
        assert st["cls"] in _candidates(st)
    amp = torch.zeros(1 << 20, dtype=torch.complex128, device=DEV)
    plan.contract(0, plan.info()["n_slices"], amp)
    torch.cuda.synchronize()
    ref = oracle.statevector(c).reshape(-1)
    err = oracle.relative_error_norm(amp.cpu().numpy(), ref)
    print(f"  relative error {err:.3e}", flush=True)
    assert err < TOL[dtype]
    # a second plan answers every shape from the database (same choices)
    again = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, tune=True, tune_db=db)
    g2 = [o for o in again.json()["ops"] if o["kind"] == 1]
    assert [(o["tile"], o["split_k"]) for o in g2] == [(o["tile"], o["split_k"]) for o in gemms]
    assert open(db).read().split("\n") == lines
    plan.close()
    again.close()


def _candidates(st):
    """Kernel classes the class tuner times for a step (1 GEMM, 2 gathered,
    3 skewed on the vector units, 4 split-K, 5 skewed on the matrix cores):
    the written rule of the planner's tests."""
    from tests.test_planner_dryrun import _class_candidates
    return _class_candidates(st)


@pytest.mark.parametrize("dtype", ["c64", "f16s"])
def test_forced_classes_vs_oracle(tmp_path, dtype):
    """Every step with an alternative class runs in a class other than the
    planner's rule (forced through class lines in the tuning database): the
    plan uses them and still matches the state vector."""
    c = make_rqc(4, 5, 12, seed=5)
    open_q = list(range(20))
    bits = np.zeros(20, dtype=np.uint8)
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, 24)
    dry = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, dry_run=True)
    forced = {}
    for st in dry.json()["steps"]:
        cand = _candidates(st)
        if cand:
            forced[st["key"]] = [k for k in cand if k != st["cls"]][0]
    dry.close()
    assert set(forced.values()) >= {2, 4}
    db = str(tmp_path / "tune.txt")
    code = {"c64": 0, "f16s": 1, "bf16s": 2}[dtype]
    with open(db, "w") as f:
        for key, k in forced.items():
            f.write(f"tnrcs-class {code} {key} {k} 0.0\n")
    print(f"forced classes {sorted(forced.values())} {dtype}", flush=True)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, tune=True, tune_db=db)
    steps = plan.json()["steps"]
    for st in steps:
        if st["key"] in forced:
            assert st["tuned"] and st["cls"] == forced[st["key"]], st
    kinds = {o["kind"] for o in plan.json()["ops"]}
    assert 4 in kinds and 2 in kinds
    amp = torch.zeros(1 << 20, dtype=torch.complex128, device=DEV)
    plan.contract(0, plan.info()["n_slices"], amp)
    torch.cuda.synchronize()
    err = oracle.relative_error_norm(amp.cpu().numpy(), oracle.statevector(c).reshape(-1))
    print(f"  relative error {err:.3e}", flush=True)
    assert err < TOL[dtype]
    assert plan.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    plan.close()


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
def test_forced_pingpong_gemm_vs_oracle(tmp_path, dtype):
    """The ping-pong 256x128 FP16/BF16 GEMM variant (tuning choice occ 3),
    forced through a GEMM line in the tuning database for every eligible
    step of a sliced 20-qubit network: the plan uses it and matches the
    state vector."""
    c = make_rqc(4, 5, 12, seed=5)
    open_q = list(range(20))
    bits = np.zeros(20, dtype=np.uint8)
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, 24)
    dry = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, dry_run=True, tune=True)
    code = {"f16s": 1, "bf16s": 2}[dtype]
    lines = [f"tnrcs-gemm {code} {o['M']} {o['N']} {o['K']} {o['form']} {o['split_max']} 128 1 3 0.0"
             for o in dry.json()["ops"]
             if o["kind"] == 1 and o["form"] == 1 and o["M"] % 256 == 0 and o["N"] % 128 == 0 and o["K"] % 32 == 0]
    dry.close()
    assert lines
    db = str(tmp_path / "tune.txt")
    with open(db, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"ping-pong GEMM forced on {len(lines)} shape(s), {dtype}", flush=True)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype, tune=True, tune_db=db)
    assert sum(o["kind"] == 1 and o["occ"] == 3 for o in plan.json()["ops"]) >= len(lines)
    amp = torch.zeros(1 << 20, dtype=torch.complex128, device=DEV)
    plan.contract(0, plan.info()["n_slices"], amp)
    torch.cuda.synchronize()
    err = oracle.relative_error_norm(amp.cpu().numpy(), oracle.statevector(c).reshape(-1))
    print(f"  relative error {err:.3e}", flush=True)
    assert err < TOL[dtype]
    assert plan.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    plan.close()


def test_config5_circuits_in_one_batch_vs_oracle():
    """Four of the 512 frozen config-5 circuits, scaled FP16 in one batch,
    against the oracle's pairwise FP64 contraction of the same order: 5
    (31 qubits, 10 cycles), 44 and 54 (28 qubits, 10 cycles), and 494 (32
    qubits, 17 cycles, one sliced wire, 2^27-entry intermediates; about
    1e12 flop for the oracle)."""
    t = config5_table()
    cand = [5, 44, 54, 494]
    assert np.diff(t["sliced_off"])[494] == 1
    ws_list = config5(indices=cand, table=t)
    cases = []
    for w in ws_list:
        leaves, ow = build_network(w.circuit, w.open_qubits, w.out_bits)
        ref = contract_sliced(leaves, w.pairs, ow, w.sliced)
        cases.append((w.circuit, w.open_qubits, w.out_bits, w.pairs, w.sliced, ref.reshape(-1)))
    print(f"config-5 circuits {cand} in one batch", flush=True)
    plans, ws = _shared_plans(cases, "f16s", tune=True)
    amps = [torch.zeros(64, dtype=torch.complex128, device=DEV) for _ in plans]
    tnrcs.tn_contract_batch(plans, [(0, p.info()["n_slices"]) for p in plans], amps)
    for i, (p, a) in enumerate(zip(plans, amps)):
        err = oracle.relative_error_norm(a.cpu().numpy(), cases[i][5])
        print(f"  circuit {cand[i]}: k={len(cases[i][4])} relative error {err:.3e}", flush=True)
        assert err < TOL["f16s"], (cand[i], err)
        p.close()
    del ws
