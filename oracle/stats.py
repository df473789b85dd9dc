"""Statistics of output amplitudes (main text, "Verifying quantum supremacy
circuits", Eq. (fxeb); Supplement Table II).

* Porter-Thomas family: density of x = N p (N = 2^n) for XEB fidelity F is
  P(x|F) = (F x + 1 - F) exp(-x).  Its mean is 1 + F, so F is estimated by
  N <p(x_i)> - 1 over sampled bit strings x_i.
* Relative error of an amplitude a against a reference b: |a - b| / |b|
  (the convention that reproduces Table II's last column within print
  rounding); the norm-wise form ||a - b|| / ||b|| over a set of amplitudes.
"""
from __future__ import annotations

import numpy as np


def porter_thomas_pdf(x, fidelity: float):
    x = np.asarray(x, dtype=np.float64)
    return (fidelity * x + 1.0 - fidelity) * np.exp(-x)


def xeb_fidelity(probs, n_qubits: int) -> float:
    """N <p> - 1 over the probabilities of the sampled bit strings."""
    p = np.asarray(probs, dtype=np.float64)
    return float((2.0 ** n_qubits) * p.mean() - 1.0)


def xeb_stderr(probs, n_qubits: int) -> float:
    x = (2.0 ** n_qubits) * np.asarray(probs, dtype=np.float64)
    return float(x.std(ddof=1) / np.sqrt(x.size))


def collision_moment(probs_all) -> float:
    """N sum_x p(x)^2 over the full distribution (2 for Porter-Thomas)."""
    p = np.asarray(probs_all, dtype=np.float64).reshape(-1)
    return float(p.size * np.sum(p * p))


def relative_error_each(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.abs(a - b) / np.abs(b)


def relative_error_norm(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
