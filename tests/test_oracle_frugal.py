"""Frugal rejection sampling in the oracle, pinned by what the Porter-Thomas
law fixes: the acceptance rate (1 - e^-M)/M, the mean of N p over accepted
candidates, the limits M -> 0 (everything with p > 0 accepted) and u = 0,
and a brute-force per-candidate loop on a tiny case."""
import numpy as np
import pytest

from oracle.stats import frugal_accept, frugal_acceptance_pt, frugal_accepted_mean_pt


def _pt_amplitudes(n, rng):
    """Amplitudes whose N|a|^2 is Exp(1) (complex Gaussian entries), N = n."""
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0 * n)
    return a


@pytest.mark.parametrize("m", [1.0, 4.0, 10.0])
def test_acceptance_rate_and_accepted_mean_match_porter_thomas(m):
    rng = np.random.default_rng(11)
    n = 1 << 20
    a = _pt_amplitudes(n, rng)
    u = rng.random(n)
    acc = frugal_accept(a, np.arange(n), u, float(n), m)
    rate = acc.size / n
    p = frugal_acceptance_pt(m)
    assert abs(rate - p) < 4 * np.sqrt(p * (1 - p) / n)
    x = n * np.abs(a[acc]) ** 2
    assert abs(x.mean() - frugal_accepted_mean_pt(m)) < 4 * x.std() / np.sqrt(x.size)


def test_closed_forms_at_limits():
    assert abs(frugal_acceptance_pt(1e-9) - 1.0) < 1e-8       # tiny M: every candidate
    assert abs(frugal_accepted_mean_pt(60.0) - 2.0) < 1e-12   # large M: N sum p^2 = 2


def test_degenerate_cases():
    rng = np.random.default_rng(3)
    a = _pt_amplitudes(4096, rng)
    a[7] = 0.0
    u = rng.random(4096)
    # M -> 0: every candidate with p > 0 is accepted
    acc = frugal_accept(a, np.arange(4096), u, 4096.0, 1e-300)
    assert acc.tolist() == [i for i in range(4096) if i != 7]
    # u = 0: accepted iff p > 0, whatever M
    acc = frugal_accept(a, np.arange(4096), np.zeros(4096), 4096.0, 1e6)
    assert 7 not in acc and acc.size == 4095
    # empty candidate list
    assert frugal_accept(a, np.zeros(0, dtype=np.int64), np.zeros(0), 4096.0, 10.0).size == 0


def test_brute_force_tiny():
    rng = np.random.default_rng(5)
    a = _pt_amplitudes(64, rng)
    cand = rng.integers(0, 64, size=200)
    u = rng.random(200)
    want = []
    for j in range(200):
        z = complex(a[cand[j]])
        if u[j] * 10.0 < (z.real * z.real + z.imag * z.imag) * 64.0:
            want.append(int(cand[j]))
    assert frugal_accept(a, cand, u, 64.0, 10.0).tolist() == want
