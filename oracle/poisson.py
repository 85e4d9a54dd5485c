"""Hartree potential of a real grid density (oracle; test infrastructure only).

The paper writes the electron-repulsion integral with the bare Coulomb kernel
1/|r - r'| (Eq. 3, the definition of B and of the (kl|nm) integrals).  The
workloads here are periodic cubic boxes, so the kernel is read as the periodic
one, v(G) = 4 pi / |G|^2 with the G = 0 term dropped.  Reciprocal vectors
follow numpy's ``fftfreq`` convention: G_i = 2 pi * fftfreq(n_i, d=h), so the
Nyquist index of an even grid takes the negative frequency (its |G|^2 is the
same either way).

    V[rho](r) = IFFT[ v(G) FFT[rho](G) ](r)

approximates  int rho(r') / |r - r'| d^3r'  (no dV factor: the FFT pair is
the discrete convolution with the Fourier-series Green's function).
"""
from __future__ import annotations

import numpy as np


def g_squared(shape, h: float) -> np.ndarray:
    """|G|^2 on the FFT grid of a cubic-cell grid with spacing h (bohr)."""
    nx, ny, nz = shape
    gx = 2.0 * np.pi * np.fft.fftfreq(nx, d=h)
    gy = 2.0 * np.pi * np.fft.fftfreq(ny, d=h)
    gz = 2.0 * np.pi * np.fft.fftfreq(nz, d=h)
    return gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2


def coulomb_kernel(shape, h: float, scale: float = 1.0) -> np.ndarray:
    """v(G) = scale * 4 pi / |G|^2, with v(0) = 0."""
    g2 = g_squared(shape, h)
    v = np.zeros_like(g2)
    nz = g2 > 0
    v[nz] = scale * 4.0 * np.pi / g2[nz]
    return v


def poisson(rho: np.ndarray, shape, h: float, scale: float = 1.0) -> np.ndarray:
    """Hartree potential of one or more real densities.

    ``rho`` is [..., N_r] (C order, z fastest); returns the same shape.
    """
    lead = rho.shape[:-1]
    r3 = rho.reshape(lead + tuple(shape))
    axes = (-3, -2, -1)
    v = coulomb_kernel(shape, h, scale)
    out = np.fft.ifftn(v * np.fft.fftn(r3, axes=axes), axes=axes)
    # a contiguous copy: the real part is a strided view, which numpy's
    # matrix product would not hand to BLAS
    return np.ascontiguousarray(out.real).reshape(rho.shape)


def dft_matrix(n: int) -> np.ndarray:
    """Explicit n-point DFT matrix, F[k, j] = exp(-2 pi i j k / n)."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def poisson_bruteforce(rho: np.ndarray, shape, h: float, scale: float = 1.0) -> np.ndarray:
    """Same potential with explicit DFT matrices along each axis (no FFT
    library); for tiny grids only.  Used to pin ``poisson``."""
    nx, ny, nz = shape
    fx, fy, fz = dft_matrix(nx), dft_matrix(ny), dft_matrix(nz)
    r3 = rho.reshape(shape).astype(np.complex128)
    rk = np.einsum("ai,bj,ck,ijk->abc", fx, fy, fz, r3)
    # explicit |G|^2 from integer frequencies, independent of fftfreq
    def freqs(n):
        k = np.arange(n)
        return np.where(k <= n // 2, k, k - n) * (2.0 * np.pi / (n * h))
    # for even n the Nyquist entry k = n/2 has |G| = pi/h either way
    g2 = (freqs(nx)[:, None, None] ** 2 + freqs(ny)[None, :, None] ** 2
          + freqs(nz)[None, None, :] ** 2)
    v = np.where(g2 > 0, scale * 4.0 * np.pi / np.where(g2 > 0, g2, 1.0), 0.0)
    vk = v * rk
    back = np.einsum("ai,bj,ck,ijk->abc", fx.conj(), fy.conj(), fz.conj(), vk)
    back /= nx * ny * nz
    return back.real.reshape(rho.shape)
