"""Pins of the oracle's polynomial replacement p_g(C) ~ C^1/2.

* interpolation of a polynomial of degree <= g is exact;
* the coefficients equal numpy's own Chebyshev interpolation (a library
  routine) after the affine map to [-1, 1];
* p_g reproduces sqrt at the interpolation nodes;
* the error over [lo, hi] falls as g grows (the synthetic analogue of the
  paper's convergence in g);
* p_g of a symmetric matrix has eigenvalues p_g(eigenvalues), and the
  matrix-free recurrence equals the dense polynomial.
"""
import numpy as np
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev as CH


def test_polynomials_are_reproduced():
    lo, hi = 0.3, 2.9
    f = lambda x: 2 * x ** 3 - x ** 2 + 0.5 * x - 4
    for g in (3, 5, 9):
        c = CH.interp_coeffs(f, lo, hi, g)
        xs = np.linspace(lo, hi, 37)
        assert np.max(np.abs(CH.eval_scalar(c, lo, hi, xs) - f(xs))) < 1e-12


def test_matches_numpy_chebinterpolate():
    lo, hi = 0.02, 0.71
    for g in (4, 7, 12):
        ours = CH.sqrt_coeffs(lo, hi, g)
        ref = npcheb.chebinterpolate(lambda t: np.sqrt(0.5 * (hi + lo) + 0.5 * (hi - lo) * t), g)
        assert np.max(np.abs(ours - ref)) < 1e-14


def test_exact_at_nodes_and_converges():
    lo, hi = 0.0226, 0.711
    errs = []
    for g in (3, 5, 7, 12, 20):
        c = CH.sqrt_coeffs(lo, hi, g)
        xk = CH.nodes(lo, hi, g)
        assert np.max(np.abs(CH.eval_scalar(c, lo, hi, xk) - np.sqrt(xk))) < 1e-14
        xs = np.linspace(lo, hi, 2001)
        errs.append(np.max(np.abs(CH.eval_scalar(c, lo, hi, xs) / np.sqrt(xs) - 1)))
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[2] < 3e-2      # g = 7
    assert errs[-1] < 1e-4     # g = 20


def test_matrix_function_and_matrix_free():
    rng = np.random.default_rng(4)
    n = 12
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.linspace(0.05, 1.3, n)
    a = (q * ev) @ q.T
    a = 0.5 * (a + a.T)
    lo, hi = 0.04, 1.31
    c = CH.sqrt_coeffs(lo, hi, 7)
    pm = CH.eval_matrix(c, lo, hi, a)
    assert np.allclose(np.linalg.eigvalsh(pm), np.sort(CH.eval_scalar(c, lo, hi, ev)), atol=1e-13)
    x = rng.standard_normal(n)
    assert np.max(np.abs(CH.apply(c, lo, hi, lambda v: a @ v, x) - pm @ x)) < 1e-12
