"""Pins of the oracle's Hartree potential (periodic 4 pi / G^2 kernel).

Each pin is fixed by mathematics, not by re-running the oracle's formula:
plane waves are eigenfunctions of the Coulomb operator with eigenvalue
4 pi / |G|^2; a constant density has no G != 0 component; and an explicit
DFT-matrix evaluation on tiny grids does not use the FFT library.
"""
import numpy as np
import pytest

from oracle import poisson as P


def _coords(shape, h):
    nx, ny, nz = shape
    x = np.arange(nx)[:, None, None] * h
    y = np.arange(ny)[None, :, None] * h
    z = np.arange(nz)[None, None, :] * h
    return x, y, z


@pytest.mark.parametrize("shape,h,k", [
    ((24, 24, 24), 0.5, (1, 0, 0)),
    ((24, 24, 24), 0.5, (2, -3, 5)),
    ((16, 12, 10), 0.4, (0, 6, 0)),      # Nyquist plane along y
    ((16, 12, 10), 0.4, (8, 6, 5)),      # Nyquist along every axis
    ((9, 15, 7), 0.3, (4, -7, 3)),       # odd grids
])
def test_plane_wave_is_eigenfunction(shape, h, k):
    x, y, z = _coords(shape, h)
    lens = [n * h for n in shape]
    g = [2 * np.pi * ki / li for ki, li in zip(k, lens)]
    g2 = sum(gi * gi for gi in g)
    for fn in (np.cos, np.sin):
        rho = fn(g[0] * x + g[1] * y + g[2] * z)
        if np.max(np.abs(rho)) < 1e-12:      # sin at Nyquist vanishes on the grid
            continue
        v = P.poisson(rho.reshape(-1), shape, h).reshape(shape)
        expect = 4 * np.pi / g2 * rho
        assert np.max(np.abs(v - expect)) <= 1e-12 * np.max(np.abs(expect))


def test_constant_density_has_zero_potential():
    shape, h = (8, 10, 6), 0.5
    v = P.poisson(np.full(np.prod(shape), 3.7), shape, h)
    assert np.max(np.abs(v)) < 1e-13


def test_kernel_scale_is_linear():
    rng = np.random.default_rng(1)
    shape, h = (8, 8, 8), 0.6
    rho = rng.standard_normal(512)
    v1 = P.poisson(rho, shape, h)
    v2 = P.poisson(rho, shape, h, scale=2.5)
    assert np.max(np.abs(v2 - 2.5 * v1)) <= 1e-14 * np.max(np.abs(v2))
    assert np.max(np.abs(P.poisson(rho, shape, h, scale=0.0))) == 0.0


@pytest.mark.parametrize("shape,h", [((6, 4, 5), 0.7), ((4, 4, 4), 0.5), ((3, 8, 2), 1.1)])
def test_fft_matches_explicit_dft(shape, h):
    rng = np.random.default_rng(2)
    rho = rng.standard_normal(int(np.prod(shape)))
    a = P.poisson(rho, shape, h)
    b = P.poisson_bruteforce(rho, shape, h)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_potential_is_real_and_self_adjoint():
    """sum_r a V[b] = sum_r b V[a]: the Coulomb operator is symmetric."""
    rng = np.random.default_rng(3)
    shape, h = (10, 12, 8), 0.45
    a = rng.standard_normal(960)
    b = rng.standard_normal(960)
    lhs = a @ P.poisson(b, shape, h)
    rhs = b @ P.poisson(a, shape, h)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # positive semidefinite: the Hartree energy of any density is >= 0
    assert a @ P.poisson(a, shape, h) > 0
