"""Polynomial approximation of D = C^1/2 (oracle; test infrastructure only).

The paper replaces D (D^2 = C) by a degree-g polynomial p_g(C) that fits
sqrt(x) on the interval holding the spectrum of C, and leaves the fitting
procedure open (paragraph after Eq. 12).  Reading taken here: Chebyshev
interpolation of sqrt(x) at the g + 1 Chebyshev points of the first kind on
[lo, hi], written in the Chebyshev basis,

    p_g(x) = sum_{j=0}^{g} c_j T_j(t),   t = (2x - (hi + lo)) / (hi - lo),

    c_j = (2 - [j = 0]) / (g + 1) * sum_{k=0}^{g} f(x_k) cos(j theta_k),
    theta_k = pi (k + 1/2) / (g + 1),  x_k = (hi + lo)/2 + (hi - lo)/2 cos(theta_k).

This is the same polynomial as the paper's monomial form a_0 I + sum a_k C^k,
evaluated in a stable basis.  The interval is an input: lo = (min Delta)^2 is a
rigorous lower bound on the spectrum because K is positive semidefinite, and
hi must bound max Omega_s^2 from above.
"""
from __future__ import annotations

import numpy as np


def interp_coeffs(f, lo: float, hi: float, g: int) -> np.ndarray:
    """Chebyshev-basis coefficients c_0..c_g of the degree-g interpolant of f
    at the first-kind Chebyshev points of [lo, hi]."""
    k = np.arange(g + 1)
    theta = np.pi * (k + 0.5) / (g + 1)
    x = 0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(theta)
    fx = np.array([f(xi) for xi in x], dtype=np.float64)
    c = np.empty(g + 1)
    for j in range(g + 1):
        c[j] = 2.0 / (g + 1) * np.sum(fx * np.cos(j * theta))
    c[0] *= 0.5
    return c


def sqrt_coeffs(lo: float, hi: float, g: int) -> np.ndarray:
    """Coefficients of p_g ~ sqrt on [lo, hi]."""
    return interp_coeffs(np.sqrt, lo, hi, g)


def nodes(lo: float, hi: float, g: int) -> np.ndarray:
    k = np.arange(g + 1)
    return 0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(np.pi * (k + 0.5) / (g + 1))


def eval_scalar(c: np.ndarray, lo: float, hi: float, x) -> np.ndarray:
    """p(x) for scalars/arrays by the three-term recurrence
    T_0 = 1, T_1 = t, T_{j+1} = 2 t T_j - T_{j-1}."""
    x = np.asarray(x, dtype=np.float64)
    t = (2.0 * x - (hi + lo)) / (hi - lo)
    tm1 = np.ones_like(t)
    acc = c[0] * tm1
    if len(c) == 1:
        return acc
    tj = t.copy()
    acc = acc + c[1] * tj
    for j in range(2, len(c)):
        tn = 2.0 * t * tj - tm1
        acc = acc + c[j] * tn
        tm1, tj = tj, tn
    return acc


def eval_matrix(c: np.ndarray, lo: float, hi: float, cmat: np.ndarray) -> np.ndarray:
    """p(C) for a dense symmetric matrix, same recurrence with matrices."""
    n = cmat.shape[0]
    eye = np.eye(n)
    t = (2.0 * cmat - (hi + lo) * eye) / (hi - lo)
    tm1 = eye
    acc = c[0] * eye
    if len(c) == 1:
        return acc
    tj = t.copy()
    acc = acc + c[1] * tj
    for j in range(2, len(c)):
        tn = 2.0 * (t @ tj) - tm1
        acc = acc + c[j] * tn
        tm1, tj = tj, tn
    return 0.5 * (acc + acc.T)


def apply(c: np.ndarray, lo: float, hi: float, matvec, x: np.ndarray) -> np.ndarray:
    """p(C) x given only x -> C x, by the same recurrence on vectors."""
    def ct(v):
        return (2.0 * matvec(v) - (hi + lo) * v) / (hi - lo)
    tm1 = x
    acc = c[0] * x
    if len(c) == 1:
        return acc
    tj = ct(x)
    acc = acc + c[1] * tj
    for j in range(2, len(c)):
        tn = 2.0 * ct(tj) - tm1
        acc = acc + c[j] * tn
        tm1, tj = tj, tn
    return acc
