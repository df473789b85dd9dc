"""Writes tests/golden/config4_30q.npz from the FP64 oracle only.

The 30-qubit cross-check network of the precision study: a 5x6 grid, 14
cycles, seed 4, every qubit open.  The oracle's state vector gives the ideal
distribution; 1e5 bit strings are drawn from it (numpy default_rng(5), by
inverse CDF over the basis order, in increasing index order) and 1e5
uniformly (default_rng(6)).  Stored (compact): the ideal sample indices
(int32), the FP64 amplitudes of every 10th ideal sample and of the first 1e4
uniform samples, the collision moment N sum p^2, the norm, and N <p> - 1 over
each full sample set.  The uniform indices are re-drawn from the same seed.

  python -m tests.golden.make_config4_golden      (about 16 GiB of RAM per copy of the state)
  python -m tests.golden.make_config4_golden --compact FULL.npz
      (re-store a full record written by an earlier version: selection only)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from rqcgen import make_rqc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_30q.npz")


def main(n_samples=100_000):
    c = make_rqc(5, 6, 14, seed=4)
    psi = oracle.statevector(c).reshape(-1)
    n = c.n_qubits
    N = float(2 ** n)
    # probabilities, then their running sum in place (inverse-CDF sampling)
    cdf = np.abs(psi) ** 2
    moment = N * float(np.sum(cdf * cdf))
    norm = float(np.sum(cdf))
    np.cumsum(cdf, out=cdf)
    u = np.sort(np.random.default_rng(5).random(n_samples)) * cdf[-1]
    ideal = np.minimum(np.searchsorted(cdf, u, side="right"), cdf.size - 1).astype(np.int64)
    del cdf
    uni = np.random.default_rng(6).integers(0, 2 ** n, size=n_samples, dtype=np.int64)
    a_ideal = psi[ideal].copy()
    a_uni = psi[uni].copy()
    save(ideal, a_ideal, uni, a_uni, moment, norm, n)


def save(ideal, a_ideal, uni, a_uni, moment, norm, n, n_amp=10_000):
    N = float(2 ** n)
    p_i, p_u = np.abs(a_ideal) ** 2, np.abs(a_uni) ** 2
    stride = len(ideal) // n_amp
    np.savez_compressed(OUT, ideal_idx=ideal.astype(np.int32), ideal_amp=a_ideal[::stride][:n_amp],
                        ideal_amp_stride=stride, uniform_amp=a_uni[:n_amp], collision_moment=moment, norm=norm,
                        xeb_ideal=N * p_i.mean() - 1.0, xeb_uniform=N * p_u.mean() - 1.0, n_qubits=n)
    print(f"wrote {OUT}: norm {norm:.15f}, N sum p^2 {moment:.4f}, XEB ideal {N * p_i.mean() - 1:.4f}, "
          f"uniform {N * p_u.mean() - 1:.4f}")


def compact(full_path):
    with np.load(full_path, allow_pickle=False) as z:
        save(z["ideal_idx"], z["ideal_amp"], z["uniform_idx"], z["uniform_amp"], float(z["collision_moment"]),
             float(z["norm"]), int(z["n_qubits"]))


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--compact":
        compact(sys.argv[2])
    else:
        main()
