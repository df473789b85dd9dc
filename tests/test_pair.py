"""Pairwise contraction entry point (tn_pair_plan / tn_pair_run): CPU dry-run
interpretation vs numpy, and GPU parity (complex64 and scaled FP16), including
the rank-27 x rank-25 microbench shape on sampled outputs vs the oracle."""
import numpy as np
import pytest

import oracle
from paper_2111_01066_amd import tnrcs
from rqcgen.workloads import config2_pair
from tests.plan_interp import PlanInterpreter

# (labels A, labels B, labels C): dense, skinny, split-K, generic, outer product
CASES = [
    ([0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11], [12, 13, 14, 15, 16, 17, 18, 5, 6, 7, 8, 9, 10, 11],
     [0, 1, 2, 3, 4, 12, 13, 14, 15, 16, 17, 18]),
    ([3, 0, 8, 1, 9, 2, 10, 4, 11, 5, 12, 6], [6, 20, 0, 21], [3, 8, 1, 9, 2, 10, 4, 11, 5, 12, 20, 21]),
    ([0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12], [13, 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11],
     [12, 13]),
    ([5, 1, 7, 3], [3, 8, 5, 9], [9, 7, 8, 1]),
    ([0, 1, 2], [3, 4], [3, 0, 4, 1, 2]),
    # split-K: 64 outputs all on B's side, all on A's side, and 3+3 with interleaved K bits
    (list(range(12)), [20, 21, 22, 23, 24, 25] + list(range(12)), [20, 21, 22, 23, 24, 25]),
    ([30, 31, 32, 33, 34, 35] + list(range(11)), list(range(11)), [30, 31, 32, 33, 34, 35]),
    ([0, 40, 1, 2, 41, 3, 4, 5, 42, 6, 7, 8, 9, 10, 11], [43, 0, 1, 44, 2, 3, 4, 5, 6, 45, 7, 8, 9, 10, 11],
     [40, 41, 42, 43, 44, 45]),
    # gathered: long K with few outputs per side (K tabulated in two levels), and K = 8 with many outputs
    ([50, 51, 52] + list(range(13)), [53, 54, 55, 56, 57] + list(range(13)), [50, 53, 51, 54, 52, 55, 56, 57]),
    (list(range(60, 70)) + [0, 1, 2], list(range(70, 79)) + [0, 1, 2], list(range(60, 70)) + list(range(70, 79))),
    # dense with 64-wide free extents (the 64x64 GEMM tile, FP16 included)
    (list(range(80, 88)) + list(range(6)), list(range(90, 96)) + list(range(6)), list(range(80, 88)) + list(range(90, 96))),
] + [
    # skewed: A as [M bits, K bits] (contiguous rows; 1, 2 or 4 rows per thread and pass),
    # K bits elsewhere (gathered rows), no K at all, and the largest B (2^11 entries)
    (list(range(12)) + [100], [101, 100], list(range(12)) + [101]),
    (list(range(9)) + [100, 102, 104], [101, 100, 103, 102, 105, 104, 106], list(range(9)) + [101, 103, 105, 106]),
    (list(range(10)) + [100, 102], [102, 101, 100, 103, 104], list(range(10)) + [101, 103, 104]),
    (list(range(6)) + [200] + list(range(6, 11)) + [201], [201, 202, 200, 203], list(range(11)) + [202, 203]),
    (list(range(8)), [300, 301], list(range(8)) + [300, 301]),
    (list(range(8)) + list(range(400, 407)), list(range(400, 407)) + [410, 411, 412, 413],
     list(range(8)) + [410, 411, 412, 413]),
]
SKEWED = CASES[-6:]
# skewed on the matrix cores: 32 or 64 outputs per row (or fewer, padded),
# A with its lowest bits M bits (rows gathered across threads) or K bits
# (contiguous rows), B resident in LDS or staged chunk by chunk (2^14
# entries), the shortest K (2) and the fewest rows (128)
SKEW = [
    (list(range(200, 206)) + list(range(10)), list(range(300, 305)) + list(range(200, 206)),
     list(range(10)) + list(range(300, 305))),
    (list(range(9)) + list(range(210, 215)), list(range(310, 316)) + [212, 210, 214, 211, 213],
     list(range(9)) + list(range(310, 316))),
    (list(range(8)) + list(range(220, 229)), [320, 228, 321, 227, 322, 220, 221, 323, 222, 223, 324, 224, 225, 226],
     list(range(8)) + list(range(320, 325))),
    ([230, 0, 1, 231, 2, 3, 4, 232, 5, 6, 7, 233, 8, 9, 10, 11], [330, 231, 331, 230, 233, 332, 232],
     list(range(12)) + [330, 331, 332]),
    (list(range(7)) + [240], list(range(340, 346)) + [240], list(range(7)) + list(range(340, 346))),
]
CASES = CASES + SKEW
# gathered with output tiles (both free extents >= 64, at most 16 terms, too
# wide for the skewed kernels): an outer product, and K = 4 with the
# operands' bits interleaved
TILED = [
    (list(range(7)), list(range(20, 27)), list(range(7)) + list(range(20, 27))),
    ([0, 500, 1, 2, 501, 3, 4, 5, 6, 7], [30, 500, 31, 32, 33, 501, 34, 35, 36], list(range(8)) + list(range(30, 37))),
]
# split-K into at most 8 x 8 outputs whose operands do not hold their
# contracted wires lowest and in one order: both are read in place, chunk by
# chunk (no permute).  B scattered; a free wire among A's low wires and B's
# contracted wires in reverse order; no free wire on A's side; a sum of 2^20
# terms (8 chunks per block) with both operands shuffled
_SH = [int(x) for x in np.random.default_rng(7).permutation(20)]
_SH2 = [int(x) for x in np.random.default_rng(8).permutation(20)]
ALIGN = [
    ([20, 21, 22] + list(range(12)), [30, 31, 32] + [5, 0, 9, 2, 11, 7, 1, 4, 10, 3, 8, 6],
     [20, 21, 22, 30, 31, 32]),
    ([50, 0, 1, 51, 2, 3, 4, 5, 6, 7, 8, 9, 52, 10, 11, 12, 13],
     [13, 60, 11, 12, 9, 10, 61, 7, 8, 5, 6, 3, 4, 1, 2, 0], [50, 51, 52, 60, 61]),
    ([3, 0, 8, 1, 9, 2, 10, 4, 11, 5, 12, 6, 7], [70, 71, 72] + list(range(13)), [70, 71, 72]),
    ([80, 81] + _SH, [90] + _SH2[:10] + [91, 92] + _SH2[10:], [80, 81, 90, 91, 92]),
]
# dense with an A of 2^20+ entries whose contracted wires are not its lowest
# block and at least 32 terms: the GEMM reads A in place (no permute of A);
# K interleaved with M, K above M, K split around M in scattered order; A's
# two lowest wires are (row, k), (row, row), (k, k) and (k, row), the four
# ways the 16-bit kernel deinterleaves a 16-byte load
GATHER = [
    ([600, 0, 601, 602, 1, 603, 2, 604, 605, 3, 606, 607, 4, 608, 609, 5, 610, 611, 6, 612],
     list(range(700, 707)) + [3, 1, 0, 2, 6, 5, 4], list(range(600, 613)) + list(range(700, 707))),
    ([600, 0, 601, 602, 1, 603, 2, 604, 605, 3, 606, 607, 4, 608, 609, 5, 610, 611, 6, 612, 7, 613],
     list(range(700, 707)) + [3, 1, 0, 2, 6, 7, 5, 4], list(range(600, 614)) + list(range(700, 707))),
    (list(range(7)) + list(range(620, 634)), [0, 1, 2, 3, 4, 5, 6] + list(range(720, 727)),
     list(range(620, 634)) + list(range(720, 727))),
    ([8, 0] + list(range(640, 652)) + [7, 1, 6, 2, 5, 3, 4],
     list(range(740, 748)) + [4, 3, 5, 2, 6, 1, 7, 0, 8], list(range(640, 652)) + list(range(740, 748))),
    ([0, 1, 2, 3, 4] + list(range(660, 673)) + [5, 673, 6], [6, 5, 4, 3, 2, 1, 0] + list(range(760, 767)),
     list(range(660, 674)) + list(range(760, 767))),
    # the shortest sum read in place: 32 terms
    ([680, 681, 0, 682, 683, 1, 684, 685, 2, 686, 687, 3] + list(range(688, 695)) + [4],
     list(range(780, 787)) + [4, 3, 2, 1, 0], list(range(680, 695)) + list(range(780, 787))),
]
# long sums into more than 64 outputs: split-K over groups of 64 outputs
# (512 and 2048 outputs; one operand's contracted wires scattered), and a
# GEMM with a 64-wide extent whose K is split over 64x64-tile slabs
WIDE = [
    ([800, 801, 802, 803, 804] + list(range(12)), [810, 811, 812, 813] + list(range(12)),
     [800, 801, 802, 803, 804, 810, 811, 812, 813]),
    ([820, 821, 822, 823, 824, 825] + list(range(12)), [5, 830, 0, 831, 9, 832, 833, 834, 2, 11, 1, 3, 4, 6, 7, 8, 10],
     [830, 820, 831, 821, 832, 822, 833, 823, 834, 824, 825]),
    (list(range(900, 909)) + list(range(14)), list(range(910, 916)) + list(range(14)),
     list(range(900, 909)) + list(range(910, 916))),
]
CASES = CASES + TILED + ALIGN + GATHER + WIDE


def _rand(rng, r):
    return rng.standard_normal(1 << r) + 1j * rng.standard_normal(1 << r)


def _ref(A, la, B, lb, lc):
    C, wc = oracle.pairwise_contract(A.reshape((2,) * len(la)), la, B.reshape((2,) * len(lb)), lb)
    return np.transpose(C, [wc.index(l) for l in lc]).reshape(-1) if lc else C.reshape(-1)


@pytest.mark.parametrize("la,lb,lc", CASES)
def test_pair_dryrun(la, lb, lc):
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
    rng = np.random.default_rng(len(la) * 7 + len(lb))
    A, B = _rand(rng, len(la)), _rand(rng, len(lb))
    it = PlanInterpreter.__new__(PlanInterpreter)
    it.js = pp.json()
    it.arena = np.full(it.js["arena_elems"], np.nan, dtype=np.complex128)
    it.leaves = it.bound = np.zeros(0, dtype=np.complex128)
    C = np.full(1 << len(lc), np.nan, dtype=np.complex128)
    it.ext = {3: A, 4: B, 5: C}
    it.run_ops()
    np.testing.assert_allclose(C, _ref(A, la, B, lb, lc), atol=1e-12)
    pp.close()


@pytest.mark.parametrize("la,lb,lc", SKEWED)
def test_pair_skewed_cases_plan_a_skewed_kernel(la, lb, lc):
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
    assert [o["kind"] for o in pp.json()["ops"]] in ([3], [5])
    pp.close()


@pytest.mark.parametrize("la,lb,lc", SKEW)
def test_pair_skew_cases_plan_the_matrix_core_kernel(la, lb, lc):
    """A is read in place; a B whose low contracted wires are scattered is
    first permuted when the sum has 2^7 terms or more (B is staged chunk by
    chunk then)."""
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
    ops = pp.json()["ops"]
    kinds = [o["kind"] for o in ops]
    if kinds[0] == 0:
        assert kinds == [0, 5] and ops[0]["a"] == [4, 0] and ops[1]["nK"] >= 7
    else:
        assert kinds == [5]
    pp.close()


@pytest.mark.parametrize("la,lb,lc", TILED)
def test_pair_tiled_cases_plan_the_gathered_kernel(la, lb, lc):
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
    ops = pp.json()["ops"]
    g = [o for o in ops if o["kind"] == 2]
    assert len(g) == 1 and g[0]["nM"] >= 6 and g[0]["nN"] >= 6 and g[0]["nK"] <= 4
    pp.close()


@pytest.mark.parametrize("la,lb,lc", ALIGN)
def test_pair_splitk_reads_scattered_operands_in_place(la, lb, lc):
    for dt in ("c64", "f16s"):
        pp = tnrcs.PairPlan(la, lb, lc, dry_run=True, dtype=dt)
        ops = pp.json()["ops"]
        sk = [o for o in ops if o["kind"] == 4]
        assert len(sk) == 1 and sorted([sk[0]["a"], sk[0]["b"]]) == [[3, 0], [4, 0]]  # the caller's A and B
        assert all(o["a"] not in ([3, 0], [4, 0]) for o in ops if o["kind"] == 0)  # neither is permuted
        pp.close()


@pytest.mark.parametrize("la,lb,lc", GATHER)
def test_pair_gather_cases_read_a_in_place(la, lb, lc):
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
    ops = pp.json()["ops"]
    g = [o for o in ops if o["kind"] == 1]
    assert len(g) == 1 and g[0]["ga"] == 1 and g[0]["a"] == [3, 0]  # the caller's A, not a permuted copy
    assert all(o["a"] != [3, 0] for o in ops if o["kind"] == 0)
    pp.close()
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True, dtype="f16s")
    assert [o["ga"] for o in pp.json()["ops"] if o["kind"] == 1] == [1]
    pp.close()
    # the 16-bit in-place kernel is 4M only: a forced 3M form permutes A
    pp = tnrcs.PairPlan(la, lb, lc, dry_run=True, dtype="f16s", gemm_form="3m")
    assert all(o.get("ga", 0) == 0 for o in pp.json()["ops"])
    pp.close()


def test_pair_wide_cases_plan_split_k_and_split_gemm():
    kinds = []
    for la, lb, lc in WIDE:
        pp = tnrcs.PairPlan(la, lb, lc, dry_run=True)
        kinds.append([(o["kind"], o.get("split_k", 0)) for o in pp.json()["ops"] if o["kind"] != 0])
        pp.close()
    assert kinds[0] == [(4, 0)] and kinds[1] == [(4, 0)]
    assert kinds[2][0][0] == 1 and kinds[2][0][1] > 1  # a 512 x 64 GEMM, K split


def test_pair_rejects_bad_labels():
    with pytest.raises(tnrcs.TnError):
        tnrcs.PairPlan([0, 1], [1, 2], [0], dry_run=True)
    with pytest.raises(tnrcs.TnError):
        tnrcs.PairPlan([0, 0], [1, 2], [1, 2], dry_run=True)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
@pytest.mark.parametrize("la,lb,lc", CASES)
def test_pair_gpu(la, lb, lc, dtype):
    import torch
    rng = np.random.default_rng(len(la) * 5 + len(lb))
    A, B = _rand(rng, len(la)), _rand(rng, len(lb))
    print(f"pair {dtype} ranks {len(la)}x{len(lb)}->{len(lc)}", flush=True)
    pp = tnrcs.PairPlan(la, lb, lc, dtype=dtype)
    if dtype == "c64":
        dA = torch.from_numpy(A.astype(np.complex64)).cuda()
        dB = torch.from_numpy(B.astype(np.complex64)).cuda()
        dC = torch.empty(1 << len(lc), dtype=torch.complex64, device="cuda")
        pp.run(dA, dB, dC, batch=1)
        torch.cuda.synchronize()
        C = dC.cpu().numpy().astype(np.complex128)
        ref = _ref(A.astype(np.complex64).astype(np.complex128), la, B.astype(np.complex64).astype(np.complex128),
                   lb, lc)
        tol = 1e-5
    else:
        half = torch.float16 if dtype == "f16s" else torch.bfloat16

        def pairs(z):
            return torch.stack([torch.from_numpy(z.real.copy()), torch.from_numpy(z.imag.copy())], -1).to(half).cuda()
        dA, dB = pairs(A), pairs(B)
        Aq = dA.float().cpu().numpy()
        Bq = dB.float().cpu().numpy()
        Aq, Bq = Aq[..., 0] + 1j * Aq[..., 1], Bq[..., 0] + 1j * Bq[..., 1]
        ref = _ref(Aq, la, Bq, lb, lc)
        scale = 2.0 ** -int(np.ceil(np.log2(np.abs(ref).max())) - 12)
        dC = torch.empty((1 << len(lc), 2), dtype=half, device="cuda")
        pp.run(dA, dB, dC, batch=1, out_scale=scale)
        torch.cuda.synchronize()
        Cq = dC.float().cpu().numpy().astype(np.float64) / scale
        C = Cq[..., 0] + 1j * Cq[..., 1]
        # the output's own rounding (unit roundoff 2^-11 / 2^-8) dominates
        tol = 2e-3 if dtype == "f16s" else 8e-3
    assert oracle.relative_error_norm(C, ref) < tol
    pp.close()


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["c64", "f16s"])
def test_config2_microbench_sampled_entries(dtype):
    """Rank-27 x rank-25 pairs sharing 12 indices, 32 pairs per call, output in
    a seeded random order; 512 sampled output entries per pair for 4 pairs
    computed one by one by the oracle in FP64 (on the storage format's
    rounded inputs for scaled FP16)."""
    import torch
    la, lb, lc = config2_pair(seed=2)
    n_pairs = 32
    pp = tnrcs.PairPlan(la, lb, lc, dtype=dtype)
    info = pp.info()
    print(f"config 2 {dtype}: dense={info['n_dense']} permutes={info['n_permute']}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(2)
    s = 0.5 ** 0.5
    A = torch.complex(torch.randn(n_pairs, 1 << 27, generator=g, device="cuda") * s,
                      torch.randn(n_pairs, 1 << 27, generator=g, device="cuda") * s)
    B = torch.complex(torch.randn(n_pairs, 1 << 25, generator=g, device="cuda") * s,
                      torch.randn(n_pairs, 1 << 25, generator=g, device="cuda") * s)
    scale = 1.0
    if dtype == "c64":
        C = torch.empty(n_pairs, 1 << 28, dtype=torch.complex64, device="cuda")
        pp.run(A, B, C, batch=n_pairs)
    else:
        # (re, im) FP16 pairs; the oracle sees the rounded values
        Ah = torch.view_as_real(A).to(torch.float16)
        Bh = torch.view_as_real(B).to(torch.float16)
        A = torch.view_as_complex(Ah.float().contiguous())
        B = torch.view_as_complex(Bh.float().contiguous())
        scale = 2.0 ** -3  # |C| ~ sqrt(4096): the stored output stays well inside FP16
        Ch = torch.empty(n_pairs, 1 << 28, 2, dtype=torch.float16, device="cuda")
        pp.run(Ah, Bh, Ch, batch=n_pairs, out_scale=scale)
        torch.cuda.synchronize()
        del Ah, Bh
        C = Ch
    torch.cuda.synchronize()
    shared = [l for l in la if l in lb]
    rng = np.random.default_rng(7)
    for pair in (0, 9, 20, 31):
        coords = rng.integers(0, 2, size=(512, 28))
        # flat offsets of every (coordinate, shared assignment) in A and B
        sh = np.array(np.meshgrid(*[[0, 1]] * 12, indexing="ij")).reshape(12, -1).T  # 4096 x 12
        def flat(labels, c_row):
            fixed = dict(zip(lc, c_row))
            idx = np.zeros(4096, dtype=np.int64)
            for pos, l in enumerate(labels):
                w = len(labels) - 1 - pos
                bit = sh[:, shared.index(l)] if l in shared else np.full(4096, fixed[l])
                idx |= bit.astype(np.int64) << w
            return idx
        ia = np.stack([flat(la, c) for c in coords])
        ib = np.stack([flat(lb, c) for c in coords])
        sa = A[pair][torch.from_numpy(ia).cuda()].cpu().numpy().astype(np.complex128)
        sb = B[pair][torch.from_numpy(ib).cuda()].cpu().numpy().astype(np.complex128)
        ref = np.array([oracle.tn.contract_entry(sa[i].reshape((2,) * 12), shared, sb[i].reshape((2,) * 12), shared)
                        for i in range(len(coords))])
        oc = np.zeros(len(coords), dtype=np.int64)
        for pos in range(28):
            oc |= coords[:, pos].astype(np.int64) << (27 - pos)
        sel = C[pair][torch.from_numpy(oc).cuda()]
        if dtype != "c64":
            sel = torch.view_as_complex(sel.float().contiguous())
        got = sel.cpu().numpy().astype(np.complex128) / scale
        err = oracle.relative_error_norm(got, ref)
        print(f"  pair {pair}: relative error {err:.2e}", flush=True)
        # complex64: the 1e-5 bar; scaled FP16: the output's own rounding (unit roundoff 2^-11) dominates
        assert err < (1e-5 if dtype == "c64" else 2e-3)
    pp.close()
