"""Pins of the stored 30-qubit fixture (tests/golden/config4_30q.npz, written
by the oracle's state vector) against what random-circuit statistics fix:
the state is normalised; a deep random circuit's output distribution is
Porter-Thomas, so the collision moment N sum p^2 is close to 2 (main text,
Eq. (fxeb) and its discussion); bit strings sampled from the ideal
distribution give a cross-entropy fidelity near 1 and uniform ones near 0,
each within a few standard errors; the ideal-sample estimate agrees with
the collision moment minus one (both estimate N sum p^2 - 1)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4_30q.npz")


@pytest.fixture(scope="module")
def g():
    if not os.path.exists(GOLDEN):
        pytest.skip("fixture not generated (python -m tests.golden.make_config4_golden)")
    with np.load(GOLDEN, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_fixture_shapes(g):
    assert int(g["n_qubits"]) == 30
    idx = g["ideal_idx"]
    assert idx.size == 100_000 and idx.min() >= 0 and idx.max() < 2 ** 30
    assert np.all(np.diff(idx) >= 0)   # drawn by inverse CDF from sorted uniforms
    assert g["ideal_amp"].size == 10_000 and g["uniform_amp"].size == 10_000


def test_norm_and_porter_thomas(g):
    assert abs(float(g["norm"]) - 1.0) < 1e-10
    assert abs(float(g["collision_moment"]) - 2.0) < 0.05


def test_xeb_on_ideal_and_uniform_samples(g):
    N = 2.0 ** 30
    # standard errors from the stored amplitudes: Var(N p) over each set
    x_i = N * np.abs(g["ideal_amp"]) ** 2
    x_u = N * np.abs(g["uniform_amp"]) ** 2
    se_i = x_i.std() / np.sqrt(100_000)
    se_u = x_u.std() / np.sqrt(100_000)
    assert abs(float(g["xeb_ideal"]) - 1.0) < 3 * se_i
    assert abs(float(g["xeb_uniform"])) < 3 * se_u
    assert abs(float(g["xeb_ideal"]) - (float(g["collision_moment"]) - 1.0)) < 3 * se_i
    # the stored amplitude subsets follow the same statistics
    assert abs(x_u.mean() - 1.0) < 3 * x_u.std() / np.sqrt(x_u.size)
    assert abs(x_i.mean() - 2.0) < 3 * x_i.std() / np.sqrt(x_i.size)
