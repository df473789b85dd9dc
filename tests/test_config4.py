"""The 30-qubit all-open cross-check of the precision study on the GPU: the
whole pipeline (plan, device contraction of all 2^30 amplitudes, FP64
reductions) in complex64, scaled FP16 and scaled BF16, against the oracle's
FP64 state vector through the stored fixture tests/golden/config4_30q.npz
(sampled amplitudes and cross-entropy values)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen.workloads import config4, config4_uniform_indices  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4_30q.npz")
TOL = {"c64": 1e-5, "f16s": 1e-2, "bf16s": 6e-2}
N = 2 ** 30


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("fixture not generated (python -m tests.golden.make_config4_golden)")
    with np.load(GOLDEN, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _xeb(amp, idx):
    """F = 2^n <|a(x)|^2> - 1 and its standard error, FP64 sums on the GPU."""
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    tnrcs.tn_amp_xeb(amp, N, idx, idx.numel(), out)
    s1, s2 = out.cpu().numpy()
    m = idx.numel()
    f = N * s1 / m - 1.0
    var = N * N * s2 / m - (f + 1.0) ** 2
    return f, float(np.sqrt(max(var, 0.0) / m))


@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
def test_config4_30q_all_open_vs_statevector(golden, dtype):
    w = config4()
    print(f"config 4 ({w.name}) {dtype}", flush=True)
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, dtype=dtype)
    amp = torch.zeros(N, dtype=torch.complex128, device="cuda")
    plan.contract(0, 1, amp)
    torch.cuda.synchronize()
    flags = plan.status()
    plan.close()
    assert flags & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    # norm of the whole output (FP64 sum over 2^30 entries on the GPU)
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    tnrcs.tn_amp_norm2(amp, N, nrm)
    assert abs(nrm.item() - float(golden["norm"])) < 2 * TOL[dtype], nrm.item()
    # sampled amplitudes against the state vector
    ideal = torch.from_numpy(golden["ideal_idx"].astype(np.int64)).cuda()
    uni = torch.from_numpy(config4_uniform_indices()).cuda()
    n_amp = golden["ideal_amp"].size
    stride = int(golden["ideal_amp_stride"])
    for name, idx, sub in (("ideal", ideal, ideal[::stride][:n_amp]), ("uniform", uni, uni[:n_amp])):
        got = amp[sub].cpu().numpy()
        err = oracle.relative_error_norm(got, golden[f"{name}_amp"])
        f, se = _xeb(amp, idx)
        ref = float(golden[f"xeb_{name}"])
        print(f"  {name}: amplitude error {err:.2e}, XEB {f:.5f} (FP64 {ref:.5f}, s.e. {se:.5f})", flush=True)
        assert err < TOL[dtype], (name, err)
        # equal XEB error: the estimate moves by less than one standard error
        assert abs(f - ref) < se, (name, f, ref, se)
    if dtype == "c64":
        # frugal rejection sampling over 2^14 random bunches of 64 (the 6
        # lowest qubits open): the kept bit strings' N <p> - 1 is that of
        # Porter-Thomas reweighted by min(1, N p / M)
        from oracle.stats import frugal_accepted_mean_pt
        rng = np.random.default_rng(9)
        starts = rng.integers(0, N // 64, size=1 << 14) * 64
        cand = torch.from_numpy((starts[:, None] + np.arange(64)[None, :]).reshape(-1)).cuda()
        u = torch.from_numpy(rng.random(cand.numel())).cuda()
        out = torch.empty(cand.numel(), dtype=torch.int64, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        tnrcs.tn_amp_frugal(amp, N, cand, cand.numel(), u, float(N), 10.0, out, cnt)
        kept = out[: int(cnt.item())]
        f, se = _xeb(amp, kept)
        want = frugal_accepted_mean_pt(10.0) - 1.0
        print(f"  frugal sampling: {kept.numel()} kept of {cand.numel()}, XEB {f:.4f} (expected {want:.4f}, "
              f"s.e. {se:.4f})", flush=True)
        assert abs(f - want) < 4 * se
    del amp
    torch.cuda.empty_cache()
