"""Pins for the oracle's statistics: the Table II relative-error convention
(printed values, within print rounding), the Porter-Thomas family of
Eq. (fxeb), and XEB on ideal/uniform samples of a deep circuit."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from rqcgen import make_rqc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_amplitudes.txt")


def _half_ulp(text: str) -> float:
    mant, _, exp = text.lower().partition("e")
    dec = len(mant.split(".")[1]) if "." in mant else 0
    return 0.5 * 10.0 ** (-dec) * 10.0 ** int(exp or 0)


def _rows():
    out = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        out.append(line.split())
    return out


def _range_over_rounding_box(fields, fn):
    vals = [float(x) for x in fields]
    hs = [_half_ulp(x) for x in fields]
    grids = [np.linspace(v - h, v + h, 5) for v, h in zip(vals, hs)]
    lo, hi = np.inf, -np.inf
    for ar, ai, br, bi in itertools.product(*grids):
        r = fn(complex(br, bi), complex(ar, ai))
        lo, hi = min(lo, r), max(hi, r)
    return lo, hi


def test_table2_relative_error_convention():
    rows = _rows()
    assert len(rows) == 5
    for r in rows:
        ref, ours, pct = r[0:2], r[2:4], r[4]
        fields = ref + ours
        lo, hi = _range_over_rounding_box(
            fields, lambda a, b: float(oracle.relative_error_each(a, b)) * 100)
        p, hp = float(pct), _half_ulp(pct)
        assert lo - hp <= p <= hi + hp, (r, lo, hi)


def test_table2_rejects_probability_convention():
    """|p_a - p_b| / p_b (probabilities) does not reproduce the table."""
    bad = 0
    for r in _rows():
        lo, hi = _range_over_rounding_box(
            r[0:4], lambda a, b: abs(abs(a) ** 2 - abs(b) ** 2) / abs(b) ** 2 * 100)
        p, hp = float(r[4]), _half_ulp(r[4])
        if not (lo - hp <= p <= hi + hp):
            bad += 1
    assert bad >= 1


def test_porter_thomas_density_normalised_with_mean_one_plus_f():
    x = np.linspace(0, 60, 600001)
    for f in (0.0, 0.0073, 0.5, 1.0):
        p = oracle.porter_thomas_pdf(x, f)
        assert abs(np.trapezoid(p, x) - 1.0) < 1e-8
        assert abs(np.trapezoid(x * p, x) - (1.0 + f)) < 1e-8


def test_relative_error_norm_basic():
    b = np.array([1 + 1j, 2, -1j])
    assert oracle.relative_error_norm(b, b) == 0.0
    a = b * (1 + 1e-3)
    assert abs(oracle.relative_error_norm(a, b) - 1e-3) < 1e-12


@pytest.fixture(scope="module")
def deep20():
    c = make_rqc(4, 5, 20, seed=11)
    psi = oracle.statevector(c).reshape(-1)
    return c, np.abs(psi) ** 2


def test_porter_thomas_collision_moment(deep20):
    _, p = deep20
    m = oracle.collision_moment(p)
    assert abs(m - 2.0) < 0.1


def test_porter_thomas_ks(deep20):
    from scipy import stats
    _, p = deep20
    x = p.size * p
    ks = stats.kstest(x, "expon")
    assert ks.statistic < 0.01


def test_xeb_ideal_and_uniform(deep20):
    c, p = deep20
    rng = np.random.default_rng(5)
    ideal = rng.choice(p.size, size=100000, p=p / p.sum())
    f_ideal = oracle.xeb_fidelity(p[ideal], c.n_qubits)
    se = oracle.stats.xeb_stderr(p[ideal], c.n_qubits)
    assert abs(f_ideal - oracle.collision_moment(p) + 1.0) < 4 * se
    assert abs(f_ideal - 1.0) < 0.1
    uni = rng.integers(0, p.size, size=100000)
    f_uni = oracle.xeb_fidelity(p[uni], c.n_qubits)
    se_u = oracle.stats.xeb_stderr(p[uni], c.n_qubits)
    assert abs(f_uni) < 4 * se_u


def test_xeb_stderr_porter_thomas_closed_forms():
    """The standard error of the XEB estimate against closed forms: with
    x = N p, uniform samples of a Porter-Thomas distribution have x ~ Exp(1)
    (variance 1, s.e. 1/sqrt(n)), ideal samples have density x e^-x
    (Gamma(2, 1): variance 2, s.e. sqrt(2/n)); and the estimate itself has
    means 0 and 1 (Eq. (fxeb) with F = 0 and F = 1)."""
    rng = np.random.default_rng(12)
    n, nq = 400_000, 30
    N = 2.0 ** nq
    x_uni = rng.exponential(1.0, n)
    x_ideal = rng.gamma(2.0, 1.0, n)
    se_u = oracle.stats.xeb_stderr(x_uni / N, nq)
    se_i = oracle.stats.xeb_stderr(x_ideal / N, nq)
    assert se_u == pytest.approx(1.0 / np.sqrt(n), rel=0.01)
    assert se_i == pytest.approx(np.sqrt(2.0 / n), rel=0.01)
    assert abs(oracle.stats.xeb_fidelity(x_uni / N, nq)) < 4 * se_u
    assert abs(oracle.stats.xeb_fidelity(x_ideal / N, nq) - 1.0) < 4 * se_i
