"""torch.autograd binding of Sigma_c and its hand-written adjoint.

``sigma_c(energies_ev, orbitals, ...)`` returns Sigma^corr_mm(omega) (eV,
complex128 [n_qp, n_omega]) as a differentiable function of the orbital
energies [n_orb] and the orbital grid values [n_orb, N_r] (float64 tensors,
the orbitals on the GPU).  The forward builds a library context from the
given values and evaluates Sigma in FP64 without reorthogonalisation (the
recurrence of Eq. 13 that the adjoint differentiates): gwl_sigma_c when no
gradient is needed, else gwl_sigma_c_vjp_forward, which keeps only the
recurrence's checkpoints (q_{k-1}, q_k every ceil(sqrt(L)) steps); the
backward calls gwl_sigma_c_vjp_backward, which recomputes the Lanczos vectors
from those checkpoints instead of storing them or running the forward again,
and returns dl/d energies and dl/d orbitals for the real loss l whose
gradient with respect to Sigma arrives as grad_output (dl/dRe Sigma + i
dl/dIm Sigma).  The Chebyshev interval [poly_lo, poly_hi]
is an argument: an interval estimated from the operator would itself depend
on the inputs.  All arithmetic runs in the library's kernels; this module
only moves arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class _SigmaC(torch.autograd.Function):
    @staticmethod
    def forward(fctx, energies_ev, orbitals, cfg):
        # (set by sigma_c from the grad mode outside this forward, which runs
        # with gradients off)
        need = cfg["need_grad"] and (fctx.needs_input_grad[0] or fctx.needs_input_grad[1])
        gctx = B.Context(orbitals.detach().contiguous(), energies_ev.detach().cpu().numpy(),
                         cfg["n_occ"], cfg["grid"], cfg["box"], precision="fp64",
                         poly_degree=cfg["poly_degree"], poly_lo=cfg["poly_lo"],
                         poly_hi=cfg["poly_hi"], reorth="none")
        try:
            if need:
                sig = gctx.sigma_c_vjp_forward(cfg["qp_states"], cfg["omega_ev"],
                                               cfg["eta_ev"], cfg["n_lanczos"])
            else:
                sig = gctx.sigma_c(cfg["qp_states"], cfg["omega_ev"], cfg["eta_ev"],
                                   cfg["n_lanczos"])
        except Exception:
            gctx.close()
            raise
        if need:
            fctx.gwl = gctx
            fctx.cfg = cfg
            fctx.e_dev = energies_ev.device
            fctx.o_dev = orbitals.device
        else:
            gctx.close()
        return torch.from_numpy(sig).to(energies_ev.device)

    @staticmethod
    def backward(fctx, grad_sigma):
        gctx, cfg = fctx.gwl, fctx.cfg
        fctx.gwl = None
        try:
            ge, go = gctx.sigma_c_vjp_backward(grad_sigma.detach().cpu().numpy(),
                                               device=fctx.o_dev)
        finally:
            gctx.close()
        ge_t = torch.from_numpy(ge).to(fctx.e_dev) if fctx.needs_input_grad[0] else None
        go_t = go if fctx.needs_input_grad[1] else None
        return ge_t, go_t, None


def sigma_c(energies_ev: torch.Tensor, orbitals: torch.Tensor, n_occ: int, grid, box,
            qp_states, omega_ev, eta_ev: float, n_lanczos: int, poly_lo: float,
            poly_hi: float, poly_degree: int = 7) -> torch.Tensor:
    """Differentiable Sigma^corr_mm(omega), eV, complex128 [n_qp, n_omega].

    energies_ev: float64 [n_orb]; orbitals: float64 [n_orb, nx*ny*nz] on the
    GPU (grid-normalised, as for Context); the other arguments as for
    Context and Context.sigma_c; poly_lo < poly_hi in hartree^2 must bracket
    the spectrum of C."""
    if not (poly_hi > poly_lo > 0):
        raise ValueError("need 0 < poly_lo < poly_hi (a fixed Chebyshev interval)")
    cfg = {"n_occ": int(n_occ), "grid": tuple(int(g) for g in grid),
           "box": tuple(float(b) for b in box), "qp_states": [int(q) for q in qp_states],
           "omega_ev": np.asarray(omega_ev, dtype=np.float64), "eta_ev": float(eta_ev),
           "n_lanczos": int(n_lanczos), "poly_lo": float(poly_lo), "poly_hi": float(poly_hi),
           "poly_degree": int(poly_degree),
           "need_grad": torch.is_grad_enabled()
           and (energies_ev.requires_grad or orbitals.requires_grad)}
    return _SigmaC.apply(energies_ev, orbitals, cfg)
