"""ctypes binding of ``libgwl.so`` (the C ABI in ``include/gwl.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch is used for device memory (tensors passed by pointer) and
for the current HIP stream.  If the shared library is missing the import
fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgwl.so")

GWL_OK, GWL_EINVAL, GWL_ENOMEM, GWL_EDEVICE, GWL_ENUMERIC, GWL_ESTATE, GWL_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
FP64, MIXED_F16, MIXED_BF16X3, MIXED_FP32 = 0, 1, 2, 3
REORTH = {"none": 0, "local": 1, "full": 2}
KEY_PRECISION, KEY_REORTH, KEY_BLOCK, KEY_POLY_LO, KEY_POLY_HI, KEY_POLY_DEGREE = 1, 2, 3, 4, 5, 6
KEY_N_VC, KEY_LAST_MS_TOTAL, KEY_LAST_C_MATVECS, KEY_GEMM_SPLITK, KEY_KERNELS = 7, 9, 10, 11, 12
KEY_PROFILE = 13
KEY_GRAPHS, KEY_TUNED_BLOCK, KEY_TUNED_SPLITK, KEY_BF16_TILE, KEY_TDA = 23, 24, 25, 26, 27
KEY_QUADRATURE, KEY_ISDF, KEY_ISDF_NMU, KEY_TUNED_TILE = 28, 29, 30, 31
KEY_ADJOINT_STORE, KEY_ADJOINT_STORED, KEY_HI_RESIDUAL, KEY_SCHEDULER = 32, 33, 34, 35
KEY_PROF = {"gemm1": (14, 15, 16), "gemm2": (17, 18, 19), "fft": (20, 21, 22)}
# "mixed" is the built 16-bit path; the last two are named by the ABI and
# refused by the library (GWL_EUNSUPPORTED)
PRECISIONS = {"fp64": FP64, "mixed": MIXED_F16, "bf16x3": MIXED_BF16X3, "fp32": MIXED_FP32}


class GwlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gwl error {code}: {msg}")
        self.code = code


class _Grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("lx", ct.c_double), ("ly", ct.c_double), ("lz", ct.c_double)]


class _Options(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("poly_degree", ct.c_int),
                ("poly_lo", ct.c_double), ("poly_hi", ct.c_double),
                ("reorth", ct.c_int), ("block", ct.c_int),
                ("kernel_scale", ct.c_double), ("stream", ct.c_void_p)]


_lib = None

_P = ct.c_void_p
_I = ct.c_int
_D = ct.c_double
_SIGS = {
    "gwl_default_options": (None, [ct.POINTER(_Options)]),
    "gwl_setup": (_I, [_P, _I, _I, _I, _I, _P, ct.POINTER(_Grid), ct.POINTER(_Options), ct.POINTER(_P)]),
    "gwl_sigma_c": (_I, [_P, _P, _I, _P, _I, _D, _I, _P]),
    "gwl_sigma_c_range": (_I, [_P, _P, _I, _I, _I, _P, _I, _D, _I, _P]),
    "gwl_lanczos_pairs": (_I, [_P, _P, _P, _P, _I, _P, _P, _P, _P, _I]),
    "gwl_sigma_from_coeffs": (_I, [_P, _P, _I, _P, _P, _P, _P, _I, _P, _I, _D, _P]),
    "gwl_sigma_from_coeffs_noalloc": (_I, [_P, _P, _I, _P, _P, _P, _P, _I, _P, _I, _D, _P]),
    "gwl_sigma_c_vjp": (_I, [_P, _P, _I, _P, _I, _D, _I, _P, _P, _P, _P]),
    "gwl_sigma_c_vjp_forward": (_I, [_P, _P, _I, _I, _I, _P, _I, _D, _I, _P]),
    "gwl_sigma_c_vjp_backward": (_I, [_P, _P, _P, _P]),
    "gwl_sigma_c_range_vjp": (_I, [_P, _P, _I, _I, _I, _P, _I, _D, _I, _P, _P, _P, _P]),
    "gwl_poisson": (_I, [_P, _P, _P, _I, _I]),
    "gwl_apply_c": (_I, [_P, _P, _P, _I, _I]),
    "gwl_pair_density": (_I, [_P, _P, _P, _I, _I]),
    "gwl_potential_product": (_I, [_P, _P, _P, _I, _I]),
    "gwl_apply_d": (_I, [_P, _P, _P, _I, _I]),
    "gwl_coupling": (_I, [_P, _P, _P, _I, _P]),
    "gwl_sigma_x": (_I, [_P, _P, _I, _P]),
    "gwl_isdf_setup": (_I, [_P, _P, _I]),
    "gwl_sigma_c_offdiag": (_I, [_P, _I, _I, _P, _I, _D, _I, _P]),
    "gwl_isdf_kmeans": (_I, [_P, _P, _I, _I, _P, _P, _P]),
    "gwl_isdf_qrcp": (_I, [_P, _P, _P, _I, _I, _P]),
    "gwl_qp_solve": (_I, [_P, _I, _P, _D, _D, _D, _P, _P]),
    "gwl_set_option": (_I, [_P, _I, _D]),
    "gwl_query": (_I, [_P, _I, ct.POINTER(_D)]),
    "gwl_last_error": (ct.c_char_p, []),
    "gwl_destroy": (None, [_P]),
}


def lib():
    """Load libgwl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with "
                              "`python -m paper_2310_20103_amd.build` first")
        h = ct.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _check(code: int):
    if code != GWL_OK:
        raise GwlError(code, lib().gwl_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _sync_torch():
    """Device tensors are produced on torch's stream; the library runs on its
    own stream, so wait for torch's pending work before handing pointers over."""
    import torch
    torch.cuda.synchronize()


def _dev(t, dtype=None):
    """Pointer of a contiguous torch device tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ct.c_void_p(t.data_ptr())


class Context:
    """One orbital set on the GPU (``gwl_setup``); see ``include/gwl.h``.

    orbitals: [n_orb, nx*ny*nz] float64/float32, numpy (host) or torch (GPU).
    energies_ev: [n_orb]; grid: (nx, ny, nz); box: edge(s) in bohr.
    """

    def __init__(self, orbitals, energies_ev, n_occ: int, grid: Sequence[int], box,
                 precision: str = "fp64", poly_degree: int = 7, poly_lo: float = 0.0,
                 poly_hi: float = 0.0, reorth: str = "full", block: int = 0,
                 kernel_scale: float = 1.0, stream=None):
        L = lib()
        self._h = ct.c_void_p()
        e = _f64(energies_ev)
        nx, ny, nz = (int(g) for g in grid)
        bx = (float(box),) * 3 if np.isscalar(box) else tuple(float(b) for b in box)
        gr = _Grid(nx, ny, nz, *bx)
        op = _Options()
        L.gwl_default_options(ct.byref(op))
        op.precision = PRECISIONS[precision]
        op.poly_degree = int(poly_degree)
        op.poly_lo = float(poly_lo)
        op.poly_hi = float(poly_hi)
        op.reorth = REORTH[reorth]
        op.block = int(block)
        op.kernel_scale = float(kernel_scale)
        op.stream = stream
        keep = None
        try:
            import torch
            is_t = isinstance(orbitals, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_t = False
        if is_t:
            t = orbitals.contiguous()
            if t.is_cuda:
                _sync_torch()
            keep = t
            n_orb = t.shape[0]
            dt = 8 if t.dtype == torch.float64 else 4
            if t.dtype not in (torch.float64, torch.float32):
                raise TypeError("orbitals must be float64 or float32")
            ptr, on_dev = ct.c_void_p(t.data_ptr()), int(t.is_cuda)
        else:
            a = np.ascontiguousarray(orbitals)
            if a.dtype not in (np.float64, np.float32):
                a = a.astype(np.float64)
            keep = a
            n_orb = a.shape[0]
            dt = a.dtype.itemsize
            ptr, on_dev = _ptr(a), 0
        if e.shape[0] != n_orb:
            raise ValueError("energies and orbitals disagree on n_orb")
        _check(L.gwl_setup(ptr, dt, on_dev, int(n_orb), int(n_occ), _ptr(e), ct.byref(gr),
                           ct.byref(op), ct.byref(self._h)))
        del keep
        self.n_orb, self.n_occ = int(n_orb), int(n_occ)
        self.orb_itemsize = int(dt)
        self.n_emp = self.n_orb - self.n_occ
        self.n_vc = self.n_occ * self.n_emp
        self.grid = (nx, ny, nz)
        self.n_r = nx * ny * nz

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gwl_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- options ------------------------------------------------------------
    def set_option(self, key: int, value: float):
        _check(lib().gwl_set_option(self._h, int(key), float(value)))

    def query(self, key: int) -> float:
        out = ct.c_double()
        _check(lib().gwl_query(self._h, int(key), ct.byref(out)))
        return out.value

    @property
    def interval(self):
        return self.query(KEY_POLY_LO), self.query(KEY_POLY_HI)

    def set_precision(self, p: str):
        self.set_option(KEY_PRECISION, PRECISIONS[p])

    def set_reorth(self, r: str):
        self.set_option(KEY_REORTH, REORTH[r])

    def set_block(self, b: int):
        self.set_option(KEY_BLOCK, b)

    def set_tda(self, on: bool):
        """Tamm-Dancoff approximation on (Lanczos on A = Delta + K) or off."""
        self.set_option(KEY_TDA, 1 if on else 0)

    def isdf_setup(self, points):
        """ISDF of the pair densities at the given grid-point indices; turns
        the ISDF product on."""
        p = _i32(points)
        _check(lib().gwl_isdf_setup(self._h, _ptr(p), len(p)))

    def isdf_qrcp(self, gv, gc, n_mu: int):
        """ISDF points by column-pivoted QR of the pair densities sketched with
        the random factors gv [N_v, p], gc [N_c, p]; increasing grid indices."""
        a, b = _f64(gv), _f64(gc)
        if a.shape[0] != self.n_occ or b.shape[0] != self.n_emp or a.shape[1] != b.shape[1]:
            raise ValueError("gv must be [n_occ, p] and gc [n_emp, p]")
        out = np.zeros(int(n_mu), dtype=np.int32)
        _check(lib().gwl_isdf_qrcp(self._h, _ptr(a), _ptr(b), int(a.shape[1]), int(n_mu),
                                   _ptr(out)))
        return out

    def isdf_kmeans(self, init_points, max_iter=50):
        """Weighted K-means interpolation points from the initial centroids
        (grid indices): (strictly increasing points, assignment passes)."""
        p = _i32(init_points)
        out = np.zeros(len(p), dtype=np.int32)
        n_pts, n_as = ct.c_int(0), ct.c_int(0)
        _check(lib().gwl_isdf_kmeans(self._h, _ptr(p), len(p), int(max_iter), _ptr(out),
                                     ct.byref(n_pts), ct.byref(n_as)))
        return out[:n_pts.value].copy(), n_as.value

    def set_isdf(self, on: bool):
        self.set_option(KEY_ISDF, 1 if on else 0)

    def set_quadrature(self, on: bool):
        """Lanczos on C with Gauss quadrature (on) or Lanczos on p_g(C) (off)."""
        self.set_option(KEY_QUADRATURE, 1 if on else 0)

    def profile_totals(self):
        """{kernel: (event ms, launches, pair vectors)} of the last call when
        profiling is on (set_option(KEY_PROFILE, 1))."""
        return {k: tuple(self.query(q) for q in keys) for k, keys in KEY_PROF.items()}

    # -- the path -----------------------------------------------------------
    def sigma_c(self, qp_states, omega_ev, eta_ev: float, n_lanczos: int) -> np.ndarray:
        """Sigma^corr_mm(omega) in eV, complex128 [n_qp, n_omega]."""
        q = _i32(qp_states)
        om = _f64(omega_ev)
        out = np.zeros((len(q), len(om), 2), dtype=np.float64)
        _check(lib().gwl_sigma_c(self._h, _ptr(q), len(q), _ptr(om), len(om), float(eta_ev),
                                 int(n_lanczos), _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def sigma_c_offdiag(self, m: int, m2: int, omega_ev, eta_ev: float,
                        n_lanczos: int) -> np.ndarray:
        """Off-diagonal Sigma^corr_mm2(omega) in eV, complex128 [n_omega]."""
        om = _f64(omega_ev)
        out = np.zeros((len(om), 2), dtype=np.float64)
        _check(lib().gwl_sigma_c_offdiag(self._h, int(m), int(m2), _ptr(om), len(om),
                                         float(eta_ev), int(n_lanczos), _ptr(out)))
        return out[:, 0] + 1j * out[:, 1]

    def sigma_c_range(self, qp_states, n_begin: int, n_end: int, omega_ev, eta_ev: float,
                      n_lanczos: int) -> np.ndarray:
        """Sum of Sigma_mm(omega, n) over n in [n_begin, n_end), eV, [n_qp, n_omega]."""
        q = _i32(qp_states)
        om = _f64(omega_ev)
        out = np.zeros((len(q), len(om), 2), dtype=np.float64)
        _check(lib().gwl_sigma_c_range(self._h, _ptr(q), len(q), int(n_begin), int(n_end),
                                       _ptr(om), len(om), float(eta_ev), int(n_lanczos),
                                       _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def sigma_c_vjp(self, qp_states, omega_ev, eta_ev: float, n_lanczos: int, grad_sigma,
                    device="cuda", n_range=None):
        """Reverse-mode derivative of l = sum Re(conj(G) Sigma): returns
        (Sigma [n_qp, n_omega] complex eV, dl/d energies [n_orb] per eV,
        dl/d orbitals [n_orb, N_r] on the device, in the orbitals' dtype).
        n_range = (n_begin, n_end) differentiates the partial n-sum of
        sigma_c_range instead."""
        import torch
        q = _i32(qp_states)
        om = _f64(omega_ev)
        G = np.asarray(grad_sigma, dtype=np.complex128).reshape(len(q), len(om))
        g2 = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1))
        sig = np.zeros((len(q), len(om), 2))
        ge = np.zeros(self.n_orb)
        gdt = torch.float64 if self.orb_itemsize == 8 else torch.float32
        go = torch.empty((self.n_orb, self.n_r), dtype=gdt, device=device)
        _sync_torch()
        if n_range is None:
            _check(lib().gwl_sigma_c_vjp(self._h, _ptr(q), len(q), _ptr(om), len(om),
                                         float(eta_ev), int(n_lanczos), _ptr(g2), _ptr(sig),
                                         _ptr(ge), _dev(go, gdt)))
        else:
            _check(lib().gwl_sigma_c_range_vjp(self._h, _ptr(q), len(q), int(n_range[0]),
                                               int(n_range[1]), _ptr(om), len(om),
                                               float(eta_ev), int(n_lanczos), _ptr(g2),
                                               _ptr(sig), _ptr(ge), _dev(go, gdt)))
        return sig[..., 0] + 1j * sig[..., 1], ge, go

    def sigma_c_vjp_forward(self, qp_states, omega_ev, eta_ev: float, n_lanczos: int,
                            n_range=None):
        """The forward of sigma_c_vjp alone: returns Sigma [n_qp, n_omega]
        complex eV and keeps the recurrence's checkpoints in the context for
        sigma_c_vjp_backward."""
        q = _i32(qp_states)
        om = _f64(omega_ev)
        n0, n1 = (0, self.n_orb) if n_range is None else (int(n_range[0]), int(n_range[1]))
        sig = np.zeros((len(q), len(om), 2))
        _sync_torch()
        _check(lib().gwl_sigma_c_vjp_forward(self._h, _ptr(q), len(q), n0, n1, _ptr(om),
                                             len(om), float(eta_ev), int(n_lanczos), _ptr(sig)))
        self._vjp_shape = (len(q), len(om))
        return sig[..., 0] + 1j * sig[..., 1]

    def sigma_c_vjp_backward(self, grad_sigma, device="cuda"):
        """(dl/d energies [n_orb] per eV, dl/d orbitals [n_orb, N_r] on the
        device) for the cotangent grad_sigma of the last sigma_c_vjp_forward."""
        import torch
        G = np.asarray(grad_sigma, dtype=np.complex128)
        shape = getattr(self, "_vjp_shape", None)
        if shape is not None:  # (without a saved forward the library reports the error)
            G = G.reshape(shape)
        g2 = np.ascontiguousarray(np.stack([G.real, G.imag], axis=-1))
        ge = np.zeros(self.n_orb)
        gdt = torch.float64 if self.orb_itemsize == 8 else torch.float32
        go = torch.empty((self.n_orb, self.n_r), dtype=gdt, device=device)
        _sync_torch()
        _check(lib().gwl_sigma_c_vjp_backward(self._h, _ptr(g2), _ptr(ge), _dev(go, gdt)))
        return ge, go

    def lanczos_pairs(self, m_idx, n_idx, lengths, ld: Optional[int] = None):
        """(alpha [P, ld], beta [P, ld], norm2 [P], out_len [P]) in hartree units."""
        m, n, ln = _i32(m_idx), _i32(n_idx), _i32(lengths)
        P = len(m)
        ld = int(ld or (ln.max() if P else 1))
        a = np.zeros((P, ld))
        b = np.zeros((P, ld))
        n2 = np.zeros(P)
        ol = np.zeros(P, dtype=np.int32)
        _check(lib().gwl_lanczos_pairs(self._h, _ptr(m), _ptr(n), _ptr(ln), P, _ptr(a), _ptr(b),
                                       _ptr(n2), _ptr(ol), ld))
        return a, b, n2, ol

    def sigma_from_coeffs(self, n_idx, alpha, beta, norm2, lens, omega_ev, eta_ev):
        """Sigma(omega, n) per pair in eV, complex128 [P, n_omega]."""
        n = _i32(n_idx)
        a, b, n2 = _f64(alpha), _f64(beta), _f64(norm2)
        ln = _i32(lens)
        om = _f64(omega_ev)
        out = np.zeros((len(n), len(om), 2))
        _check(lib().gwl_sigma_from_coeffs(self._h, _ptr(n), len(n), _ptr(a), _ptr(b), _ptr(n2),
                                           _ptr(ln), a.shape[1], _ptr(om), len(om), float(eta_ev),
                                           _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def sigma_from_coeffs_noalloc(self, n_idx, alpha, beta, norm2, lens, omega_ev, eta_ev):
        """As sigma_from_coeffs, through the entry point that allocates no
        device memory (its buffers live in a fixed per-device array)."""
        n = _i32(n_idx)
        a, b, n2 = _f64(alpha), _f64(beta), _f64(norm2)
        ln = _i32(lens)
        om = _f64(omega_ev)
        out = np.zeros((len(n), len(om), 2))
        _check(lib().gwl_sigma_from_coeffs_noalloc(self._h, _ptr(n), len(n), _ptr(a), _ptr(b),
                                                   _ptr(n2), _ptr(ln), a.shape[1], _ptr(om),
                                                   len(om), float(eta_ev), _ptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    # -- components (device tensors) ----------------------------------------
    def poisson(self, rho, precision: str = "fp64"):
        import torch
        p = PRECISIONS[precision]
        dt = torch.float64 if p == FP64 else torch.float32
        out = torch.empty_like(rho)
        _sync_torch()
        _check(lib().gwl_poisson(self._h, _dev(rho, dt), _dev(out, dt), int(rho.shape[0]), p))
        return out

    def pair_density(self, x, precision: str = "fp64"):
        """rho_b(r) = sum_vc phi_v(r) phi_c(r) (Delta^1/2 x_b)_vc for device
        pair vectors x [n_vec][N_vc] (float64); float64 [n_vec][N_r]."""
        import torch
        out = torch.empty((x.shape[0], self.n_r), dtype=torch.float64, device=x.device)
        _sync_torch()
        _check(lib().gwl_pair_density(self._h, _dev(x, torch.float64), _dev(out, torch.float64),
                                      int(x.shape[0]), PRECISIONS[precision]))
        return out

    def potential_product(self, v, precision: str = "fp64"):
        """y_b,vc = dV sum_r phi_v(r) V_b(r) phi_c(r) for device potentials
        v [n_vec][N_r] (float64); float64 [n_vec][N_vc]."""
        import torch
        out = torch.empty((v.shape[0], self.n_vc), dtype=torch.float64, device=v.device)
        _sync_torch()
        _check(lib().gwl_potential_product(self._h, _dev(v, torch.float64),
                                           _dev(out, torch.float64), int(v.shape[0]),
                                           PRECISIONS[precision]))
        return out

    def apply_c(self, x, precision: str = "fp64"):
        import torch
        out = torch.empty_like(x)
        _sync_torch()
        _check(lib().gwl_apply_c(self._h, _dev(x, torch.float64), _dev(out, torch.float64),
                                 int(x.shape[0]), PRECISIONS[precision]))
        return out

    def apply_d(self, x, precision: str = "fp64"):
        import torch
        out = torch.empty_like(x)
        _sync_torch()
        _check(lib().gwl_apply_d(self._h, _dev(x, torch.float64), _dev(out, torch.float64),
                                 int(x.shape[0]), PRECISIONS[precision]))
        return out

    def sigma_x(self, qp_states):
        """Exchange self-energy Sigma^ex_mm (eV) for each state."""
        q = _i32(qp_states)
        out = np.zeros(len(q))
        if len(q):
            _check(lib().gwl_sigma_x(self._h, _ptr(q), len(q), _ptr(out)))
        return out

    def coupling(self, m_idx, n_idx, device="cuda"):
        import torch
        m, n = _i32(m_idx), _i32(n_idx)
        out = torch.empty((len(m), self.n_vc), dtype=torch.float64, device=device)
        _sync_torch()
        _check(lib().gwl_coupling(self._h, _ptr(m), _ptr(n), len(m), _dev(out, torch.float64)))
        return out


_COEFF_KEYS = ("m", "n", "alpha", "beta", "norm2", "lens")


def save_coefficients(path, m_idx, n_idx, alpha, beta, norm2, lens, **meta):
    """Write the Lanczos coefficients of (m, n) start vectors (the output of
    Context.lanczos_pairs) to an .npz file.  They fix Sigma on any frequency
    grid and broadening (the continued fraction of Eq. 14), so
    Context.sigma_from_coeffs on the loaded arrays resumes without another
    Lanczos run.  meta: scalars or lists describing the run (interval,
    degree, precision, grid, ...), stored as JSON."""
    import json
    arrays = {"m": _i32(m_idx), "n": _i32(n_idx), "alpha": _f64(alpha), "beta": _f64(beta),
              "norm2": _f64(norm2), "lens": _i32(lens)}
    P = len(arrays["n"])
    if not (len(arrays["m"]) == P and arrays["alpha"].shape == arrays["beta"].shape
            and arrays["alpha"].ndim == 2 and arrays["alpha"].shape[0] == P
            and len(arrays["norm2"]) == P and len(arrays["lens"]) == P):
        raise ValueError("coefficient arrays of inconsistent shapes")
    np.savez(path, meta=np.array(json.dumps(meta)), **arrays)


def load_coefficients(path):
    """(arrays, meta) from save_coefficients: arrays holds m, n, alpha, beta,
    norm2, lens; nothing in the file is executed (no pickled objects)."""
    import json
    with np.load(path, allow_pickle=False) as f:
        arrays = {k: f[k] for k in _COEFF_KEYS}
        meta = json.loads(str(f["meta"]))
    return arrays, meta


def qp_solve(omega_ev, sigma_c, eps_ev: float, sigma_x_ev: float, vxc_ev: float = 0.0):
    """(E_qp, Z) from the graphical solution on the frequency grid (eV);
    raises GwlError when the equation has no root on the grid."""
    om = _f64(omega_ev)
    sc = np.asarray(sigma_c, dtype=np.complex128).reshape(len(om))
    s2 = np.ascontiguousarray(np.stack([sc.real, sc.imag], axis=-1))
    e = np.zeros(1)
    z = np.zeros(1)
    _check(lib().gwl_qp_solve(_ptr(om), len(om), _ptr(s2), float(eps_ev), float(sigma_x_ev),
                              float(vxc_ev), _ptr(e), _ptr(z)))
    return float(e[0]), float(z[0])
