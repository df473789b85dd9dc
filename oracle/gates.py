"""Gate matrices in FP64 (Supplement, section "Random quantum circuits").

Written directly from the printed definitions:

* sqrt(X) = (sqrt2/2) [[1, -i], [-i, 1]]
* sqrt(Y) = (sqrt2/2) [[1, -1], [1, 1]]
* sqrt(W) = (sqrt2/2) [[1, -(sqrt2/2)(1+i)], [(sqrt2/2)(1-i), 1]]
* the 5-parameter fSim gate.  The printed matrix writes the same phase
  exp(i(D+ + D-)) on both middle diagonal entries, which is not unitary when
  D- is nonzero; we read the second one as exp(i(D+ - D-)), the form that is
  unitary for all parameters.  Every circuit here uses D+ = D- = D-off = 0,
  where both readings coincide.

Two-qubit matrices act on |q0 q1> with q0 the more significant bit.
"""
from __future__ import annotations

import cmath
import math

import numpy as np


def sqrt_x() -> np.ndarray:
    s = math.sqrt(2.0) / 2.0
    return s * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)


def sqrt_y() -> np.ndarray:
    s = math.sqrt(2.0) / 2.0
    return s * np.array([[1, -1], [1, 1]], dtype=np.complex128)


def sqrt_w() -> np.ndarray:
    s = math.sqrt(2.0) / 2.0
    return s * np.array([[1, -s * (1 + 1j)], [s * (1 - 1j), 1]], dtype=np.complex128)


def fsim(theta: float, phi: float, d_plus: float = 0.0, d_minus: float = 0.0,
         d_minus_off: float = 0.0) -> np.ndarray:
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = cmath.exp(1j * (d_plus + d_minus)) * math.cos(theta)
    m[1, 2] = -1j * cmath.exp(1j * (d_plus - d_minus_off)) * math.sin(theta)
    m[2, 1] = -1j * cmath.exp(1j * (d_plus + d_minus_off)) * math.sin(theta)
    m[2, 2] = cmath.exp(1j * (d_plus - d_minus)) * math.cos(theta)
    m[3, 3] = cmath.exp(1j * (2.0 * d_plus - phi))
    return m


def gate_matrix(name: str, params=()) -> np.ndarray:
    if name == "sqrt_x":
        return sqrt_x()
    if name == "sqrt_y":
        return sqrt_y()
    if name == "sqrt_w":
        return sqrt_w()
    if name == "fsim":
        return fsim(*params)
    raise ValueError(f"oracle: unknown gate {name!r}")
