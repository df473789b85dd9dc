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


def frugal_accept(amps, candidates, uniforms, scale: float, m: float) -> np.ndarray:
    """Frugal rejection sampling over a bunch of amplitudes (main text: one
    perfect sample is drawn from a bunch of 64 amplitudes by frugal sampling,
    after the works it cites).  Candidate j, the amplitude amps[candidates[j]],
    is accepted when u_j * m < scale * |a|^2, i.e. with probability
    min(1, N p / m) for scale = N = 2^n and u_j uniform on [0, 1).  The
    product and sum are taken in FP64 as written (re*re + im*im, then times
    scale).  Returns the accepted amplitude indices in candidate order."""
    cand = np.asarray(candidates, dtype=np.int64)
    a = np.asarray(amps, dtype=np.complex128)[cand]
    x = (a.real * a.real + a.imag * a.imag) * scale
    keep = np.asarray(uniforms, dtype=np.float64) * m < x
    return cand[keep]


def frugal_acceptance_pt(m: float) -> float:
    """Acceptance probability of one candidate when N p follows the
    Porter-Thomas law Exp(1): E[min(1, x/m)] = (1 - e^-m) / m."""
    return float(-np.expm1(-m) / m)


def frugal_accepted_mean_pt(m: float) -> float:
    """Mean of x = N p over accepted candidates under Porter-Thomas:
    E[x min(x, m)] / E[min(x, m)] = (2 - (m + 2) e^-m) / (1 - e^-m)."""
    return float((2.0 - (m + 2.0) * np.exp(-m)) / -np.expm1(-m))
