"""Frugal rejection sampling on the GPU (tn_amp_frugal) against the oracle's
decisions on the same amplitudes and the same uniforms: the kept multiset is
identical (the decision is an FP64 comparison evaluated the same way on both
sides), including repeated candidates, out-of-range candidates (never kept)
and the empty list."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.stats import frugal_accept, frugal_acceptance_pt  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402

DEV = "cuda"


def _gpu_frugal(a, cand, u, scale, m):
    da = torch.from_numpy(a).to(DEV)
    n_cand = len(u)
    di = None if cand is None else torch.from_numpy(np.asarray(cand, dtype=np.int64)).to(DEV)
    du = torch.from_numpy(np.asarray(u, dtype=np.float64)).to(DEV)
    out = torch.full((max(n_cand, 1),), -7, dtype=torch.int64, device=DEV)
    cnt = torch.full((1,), 123, dtype=torch.int64, device=DEV)
    tnrcs.tn_amp_frugal(da, a.size, di, n_cand, du, scale, m, out, cnt)
    torch.cuda.synchronize()
    k = int(cnt.item())
    return np.sort(out[:k].cpu().numpy())


@pytest.mark.parametrize("m", [1.0, 10.0])
def test_frugal_matches_oracle_decisions(m):
    rng = np.random.default_rng(21)
    n = 1 << 18
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0 * n)
    # every amplitude once
    u = rng.random(n)
    got = _gpu_frugal(a, None, u, float(n), m)
    want = np.sort(frugal_accept(a, np.arange(n), u, float(n), m))
    assert np.array_equal(got, want)
    assert abs(got.size / n - frugal_acceptance_pt(m)) < 0.01
    # a random candidate list with repeats
    cand = rng.integers(0, n, size=300_000)
    u2 = rng.random(cand.size)
    got = _gpu_frugal(a, cand, u2, float(n), m)
    assert np.array_equal(got, np.sort(frugal_accept(a, cand, u2, float(n), m)))


def test_frugal_edge_cases():
    rng = np.random.default_rng(4)
    n = 1000
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0 * n)
    cand = np.array([-1, 5, n, 7, n + 100, 5], dtype=np.int64)
    u = np.zeros(cand.size)  # u = 0: every in-range candidate with p > 0 is kept
    got = _gpu_frugal(a, cand, u, float(n), 10.0)
    assert got.tolist() == [5, 5, 7]
    assert _gpu_frugal(a, np.zeros(0, dtype=np.int64), np.zeros(0), float(n), 10.0).size == 0
    with pytest.raises(tnrcs.TnError):
        _gpu_frugal(a, None, np.zeros(n), float(n), 0.0)
