#!/usr/bin/env python3
"""Throughput of the Lanczos full-frequency GW self-energy on one MI355X.

Workload (grid64_v128c512): 64^3 grid in a 24 bohr box, 128 occupied + 512
empty seeded orthonormal real orbitals (pair dimension 65,536), Lanczos on
p_7(C) with L = 200 steps, 2,000 frequencies in [-20, 20] eV, broadening
0.05 eV, full reorthogonalisation.  Arithmetic: both GEMMs on FP16 operands
(power-of-two scaled), FP32 accumulation, FP32 FFT, FP64 Lanczos recurrence /
Chebyshev combination / continued fraction.

One step = one block of B start vectors (m, n) of one quasiparticle state m
through the whole path: coupling vectors P_nm, L Lanczos steps on p_g(C)
(g factored C-products each), continued fraction at every frequency and the
sum over n.  N_orb / B steps make one spectrum Sigma_mm(omega); the metric is
spectra per second.

Also reported: the plain FP64 GPU path end to end on one block at two short
Lanczos lengths, extrapolated linearly in L to spectra/s; Sigma of the FP64
and mixed GPU paths against the FP64 oracle on a sample of full-size start
vectors and on two smooth-orbital cases where Sigma is eV-sized; the roofline
fraction of the dominant kernel (HIP events on the library's stream); and the
FP64 CPU oracle on a bounded sample.

Two further measurements print their own line:
  --mode uneven   batched start vectors with uneven Lanczos lengths
                  (grid64_v128c512_pairs1024: drawn (m, n) pairs, lengths
                  U[50, 300]); vector-steps/s for B in {32, 64, 128, 256}, with
                  and without graph replay, on the first --pairs pairs.
  --mode adjoint  forward Sigma_c and its vector-Jacobian product in FP64 on
                  grid48_v64c256 (48^3 grid, 64 + 256 orbitals, L = 120,
                  32 frequencies) for one quasiparticle state; the ratio of
                  the two times.
  --mode isdf     smooth orbitals of grid48_v64c256 (or --workload) with the
                  K product on N_mu = r N_orb seeded grid points (ISDF, FP64;
                  r = --isdf-ratio, 4 by default as in the paper's runs):
                  setup time, spectra/s over --steps blocks against the grid
                  FP64 product on a window, and the ISDF error of Sigma
                  against the grid product on a sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_16BIT_TFLOPS = 2500.0  # MI355X dense FP16 / BF16 MFMA
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 matrix
METRIC = "Sigma_c spectra/s & matvec TFLOP/s, mixed vs FP64 on 1 GPU at 1e-3 eV"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload, block):
    """HBM bytes per launch of `kernel` from the counter summary committed in
    profiles/ (FETCH_SIZE and WRITE_SIZE passes scaled by a plain-copy
    calibration).  None when there is no summary, when it was taken at another
    block size, or when the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for ln in f:
            if ":" in ln and not ln.startswith(" "):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2310_20103_amd", "csrc", kv.get("source", "?"))
    if not os.path.exists(src) or int(kv.get("block", -1)) != block:
        return None
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != kv.get("source_sha256"):
            return None
    return float(kv["hbm_bytes_per_launch"])


def oracle_threads():
    """Threads the oracle's BLAS runs with (numpy's FFT runs on one)."""
    cores = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()] + [1])
    except Exception:
        pass
    return int(cores)


def oracle_vector(wl, pr, m, n, steps, lo, hi, omega):
    """The FP64 oracle (matrix-free route) for one start vector (m, n):
    its Lanczos coefficients on p_g(C), Sigma_mm(omega, n) in eV and the time."""
    from oracle import sigma as S
    t0 = time.perf_counter()
    (a, b, n2), = pr.lanczos_coeffs(m, steps, lo, hi, wl.poly_degree, reorth="full",
                                    route="matfree", n_list=[n])
    sig = S.sigma_n_from_tridiag(a, b, n2, np.asarray(omega) / S.HARTREE_EV, pr.eps[n],
                                 pr.eta(n), wl.eta / S.HARTREE_EV) * S.HARTREE_EV
    return sig, time.perf_counter() - t0


def cpu_baseline(wl, seconds, m, ns, steps):
    """The oracle's time for len(ns) start vectors over `steps` Lanczos steps
    each (coupling vectors included), extrapolated to spectra/s."""
    per_spectrum = seconds / (len(ns) * steps) * wl.n_lanczos * wl.n_orb
    return {
        "value": 1.0 / per_spectrum, "unit": "spectra/s", "cores": oracle_threads(),
        "kind": "oracle",
        "sample": (f"oracle matrix-free Lanczos on p_{wl.poly_degree}(C), {len(ns)} start "
                   f"vectors (m={m}, n in {list(ns)}), {steps} steps each incl. the coupling "
                   f"vector, {seconds:.1f} s, extrapolated x {wl.n_lanczos} steps x "
                   f"{wl.n_orb} vectors; BLAS on the stated threads, FFT on one"),
    }


def run_sched(args):
    """Vector-steps/s of the two schedulers (refill schedule uploaded once with
    whole-step graph replay, against the host-driven loop) for B in {32, 64,
    128, 256}: on the small workload (24^3, 8 + 32 orbitals: every (m, n) pair
    of all 40 states, L = 64, kernels of microseconds, so launch and host
    costs show) and on the first --pairs drawn pairs of the uneven workload
    (lengths U[50, 300], headline orbitals)."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    out = []
    for name in ("grid24_v8c32", "grid64_v128c512_pairs1024"):
        wl = gi.workload(name)
        sysm = gi.make_system(wl)
        box = tuple(k * wl.h for k in wl.grid)
        if name == "grid24_v8c32":
            m = np.repeat(np.arange(wl.n_orb), wl.n_orb)
            n = np.tile(np.arange(wl.n_orb), wl.n_orb)
            lens = np.full(m.size, wl.n_lanczos)
            prec = "fp64"
        else:
            P = min(args.pairs, wl.n_pairs)
            ex = sysm.extras
            m, n, lens = ex["m_idx"][:P], ex["n_idx"][:P], ex["lengths"][:P]
            prec = "mixed"
        ctx = G.Context(sysm.phi, sysm.energies_ev, wl.n_occ, wl.grid, box, precision=prec,
                        poly_degree=wl.poly_degree, reorth="full")
        for B in (32, 64, 128, 256):
            for sched in (1, 0):
                ctx.set_block(B)
                ctx.set_option(G.KEY_SCHEDULER, sched)
                ctx.lanczos_pairs(m[:B], n[:B], [2] * min(B, len(m)))
                torch.cuda.synchronize()
                t = time.perf_counter()
                ctx.lanczos_pairs(m, n, lens)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                vs = float(np.sum(lens))
                out.append({"workload": name, "precision": prec, "block": B,
                            "scheduler": "tables+step graphs" if sched else "host loop",
                            "seconds": round(dt, 3), "vector_steps_per_s": round(vs / dt, 1)})
                log(f"sched {name} B={B} sched={sched}: {dt:.2f}s, {vs / dt:.0f} vector-steps/s")
        ctx.close()
    print(json.dumps({
        "metric": "Lanczos vector-steps/s by scheduler", "unit": "vector-steps/s",
        "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
        "config": {"reorth": "full", "small": "all 1600 (m, n) pairs of grid24_v8c32, L=64, FP64",
                   "uneven": f"first {min(args.pairs, 1024)} pairs of grid64_v128c512_pairs1024, mixed"},
        "runs": out}), flush=True)


def run_uneven(args):
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    wl = gi.workload("grid64_v128c512_pairs1024")
    sysm = gi.make_system(wl)
    ex = sysm.extras
    P = min(args.pairs, wl.n_pairs)
    m, n, lens = ex["m_idx"][:P], ex["n_idx"][:P], ex["lengths"][:P]
    box = tuple(k * wl.h for k in wl.grid)
    ctx = G.Context(sysm.phi, sysm.energies_ev, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full")
    runs = []
    cases = ((32, 1), (64, 1), (128, 1), (256, 1), (128, 0))
    if args.uneven_blocks:
        cases = tuple((int(b), 1) for b in args.uneven_blocks.split(","))
    for B, graphs in cases:
        ctx.set_block(B)
        ctx.set_option(G.KEY_GRAPHS, graphs)
        ctx.lanczos_pairs(m[:B], n[:B], [1] * min(B, P))
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.lanczos_pairs(m, n, lens)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        vs = float(np.sum(lens))
        runs.append({"block": B, "graphs": bool(graphs), "seconds": round(dt, 3),
                     "vector_steps_per_s": round(vs / dt, 2),
                     "partial_spectra_per_s": round(P / wl.n_orb / dt, 6),
                     "matvec_tflops": round(4.0 * wl.n_r * wl.n_occ * wl.n_emp
                                            * ctx.query(G.KEY_LAST_C_MATVECS) / dt / 1e12, 1)})
        log(f"uneven B={B} graphs={graphs}: {dt:.1f}s")
    ctx.close()
    best = max(runs, key=lambda r: r["vector_steps_per_s"])
    print(json.dumps({
        "metric": "Lanczos vector-steps/s, uneven lengths, mixed precision", "unit": "vector-steps/s",
        "value": best["vector_steps_per_s"], "n_gpus": 1, "higher_is_better": True,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": wl.name, "pairs": int(P), "lengths": "U[50, 300]",
                   "vector_steps": int(np.sum(lens)), "poly_degree": wl.poly_degree,
                   "reorth": "full"},
        "runs": runs}), flush=True)


def run_adjoint(args):
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    wl = gi.workload(args.adjoint_workload)
    L = args.adjoint_lanczos or wl.n_lanczos
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    omega = gi.omega_grid(wl)
    if args.adjoint_omega:
        omega = np.linspace(omega[0], omega[-1], args.adjoint_omega)
    box = tuple(k * wl.h for k in wl.grid)
    m = [int(qp[0])]
    n_end = args.adjoint_vectors or wl.n_orb
    rng = np.random.default_rng([wl.seed, 9])
    cot = rng.standard_normal((1, len(omega))) + 1j * rng.standard_normal((1, len(omega)))
    log(f"adjoint: {wl.name}, {n_end} start vectors, L = {L}, {len(omega)} frequencies")
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="fp64",
                    poly_degree=wl.poly_degree, reorth="none", block=args.block)
    ctx.lanczos_pairs([m[0]] * 2, [0, 1], [1, 1])
    if args.adjoint_store:
        ctx.set_option(G.KEY_ADJOINT_STORE, 1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sig = ctx.sigma_c_range(m, 0, n_end, omega, wl.eta, L)
    t_fwd = time.perf_counter() - t
    log(f"adjoint: forward {t_fwd:.1f}s")
    t = time.perf_counter()
    sig2, ge, go = ctx.sigma_c_vjp(m, omega, wl.eta, L, cot, n_range=(0, n_end))
    torch.cuda.synchronize()
    t_vjp = time.perf_counter() - t
    iterates = "stored" if ctx.query(G.KEY_ADJOINT_STORED) == 1 else "recomputed"
    log(f"adjoint: vjp {t_vjp:.1f}s, iterates {iterates}")
    same = float(np.max(np.abs(sig2 - sig)) / max(np.max(np.abs(sig)), 1e-300))
    # the split form: forward keeping checkpoints, then the backward alone
    split = None
    if not args.adjoint_store:
        go_one = go.cpu().numpy()
        del go
        t = time.perf_counter()
        sig3 = ctx.sigma_c_vjp_forward(m, omega, wl.eta, L, n_range=(0, n_end))
        t_sf = time.perf_counter() - t
        log(f"adjoint: split forward {t_sf:.1f}s")
        t = time.perf_counter()
        ge3, go3 = ctx.sigma_c_vjp_backward(cot)
        torch.cuda.synchronize()
        t_sb = time.perf_counter() - t
        log(f"adjoint: split backward {t_sb:.1f}s")
        split = {"forward_s": round(t_sf, 3), "backward_s": round(t_sb, 3),
                 "backward_over_forward": round(t_sb / t_fwd, 3),
                 "forward_plus_backward_over_forward": round((t_sf + t_sb) / t_fwd, 3),
                 "equals_one_call": bool(np.array_equal(sig3, sig2) and np.array_equal(ge3, ge)
                                         and np.array_equal(go3.cpu().numpy(), go_one))}
        go = torch.from_numpy(go_one)
        del go3
    ctx.set_reorth("full")
    t = time.perf_counter()
    ctx.sigma_c_range(m, 0, n_end, omega, wl.eta, L)
    t_full = time.perf_counter() - t
    lo, hi = ctx.interval
    ctx.close()
    # central differences of the same forward (FP64, no reorthogonalisation,
    # the interval held fixed) along seeded random directions, step 1e-5
    h = 1e-5

    def loss(e, p):
        with G.Context(p, e, wl.n_occ, wl.grid, box, precision="fp64",
                       poly_degree=wl.poly_degree, poly_lo=lo, poly_hi=hi, reorth="none",
                       block=args.block) as c:
            return float(np.sum((np.conj(cot) * c.sigma_c_range(m, 0, n_end, omega, wl.eta,
                                                                L)).real))

    de = rng.standard_normal(wl.n_orb)
    dp = rng.standard_normal(phi.shape) * float(np.mean(np.abs(phi)))
    fd_e = (loss(eps + h * de, phi) - loss(eps - h * de, phi)) / (2 * h)
    log("adjoint: energy direction done")
    fd_p = (loss(eps, phi + h * dp) - loss(eps, phi - h * dp)) / (2 * h)
    log("adjoint: orbital direction done")
    an_e = float(ge @ de)
    an_p = float(np.sum(go.cpu().numpy() * dp))
    print(json.dumps({
        "metric": "Sigma_c vector-Jacobian product time / forward time, FP64", "unit": "ratio",
        "value": round(t_vjp / t_fwd, 3), "n_gpus": 1, "higher_is_better": False,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "qp_states": 1, "start_vectors": n_end,
                   "n_lanczos": L, "n_omega": len(omega), "block": args.block,
                   "iterates": iterates},
        "forward_s": round(t_fwd, 3), "vjp_s_incl_forward": round(t_vjp, 3),
        "forward_full_reorth_s": round(t_full, 3),
        "vjp_sigma_vs_forward_rel": same, "split": split,
        "fd_check": {"step": h, "energies": {"fd": fd_e, "vjp": an_e,
                                             "rel": abs(fd_e - an_e) / max(abs(fd_e), 1e-300)},
                     "orbitals": {"fd": fd_p, "vjp": an_p,
                                  "rel": abs(fd_p - an_p) / max(abs(fd_p), 1e-300)}},
        "grad_norms": {"energies": float(np.linalg.norm(ge)),
                       "orbitals": float(torch.linalg.norm(go).item())}}), flush=True)


def smooth_stress_error(G, gi):
    """FP64 and mixed GPU Sigma against the oracle's Sigma_L on smooth-orbital
    variants (eV-sized Sigma, where the 1e-3 eV bar binds): the 24^3, 8 + 32
    workload (both QP states, L = 64, 200 frequencies, full method and the
    Tamm-Dancoff option against the GPU FP64 result) and the 32^3, 32 + 128
    headline-shaped case (one QP state, L = 100, 400 frequencies)."""
    import oracle
    out = {}
    for name, nq, tda_too in (("grid24_v8c32", 2, True), ("grid32_v32c128", 1, False)):
        wl = gi.workload(name, name=name + "_smooth", smooth_sigma=1.0)
        sysm = gi.make_system(wl)
        pr = oracle.Problem(sysm.phi, sysm.energies_ev, wl.n_occ, wl.grid, wl.h)
        lo, hi = oracle.default_interval(pr)
        qp = [int(q) for q in sysm.qp_states[:nq]]
        refs = np.array([pr.sigma_lanczos(m, sysm.omega_ev, wl.eta, wl.n_lanczos, lo, hi,
                                          wl.poly_degree, route="measure") for m in qp])
        box = tuple(k * wl.h for k in wl.grid)
        ctx = G.Context(sysm.phi, sysm.energies_ev, wl.n_occ, wl.grid, box, precision="fp64",
                        poly_degree=wl.poly_degree, poly_lo=lo, poly_hi=hi, reorth="full")
        res = {}
        for p in ("fp64", "mixed"):
            ctx.set_precision(p)
            res[p] = ctx.sigma_c(qp, sysm.omega_ev, wl.eta, wl.n_lanczos)
        case = {"case": (f"{wl.grid[0]}^3, {wl.n_occ}+{wl.n_emp} smooth orbitals, {len(qp)} "
                         f"QP states, L={wl.n_lanczos}, {wl.n_omega} omega"),
                "max_abs_sigma_ev": float(np.max(np.abs(refs))),
                "fp64_vs_oracle_rel": float(np.max(np.abs(res["fp64"] - refs))
                                            / np.max(np.abs(refs))),
                "mixed_vs_oracle_abs_ev": float(np.max(np.abs(res["mixed"] - refs)))}
        if tda_too:
            ctx.set_tda(True)
            t = {}
            for p in ("fp64", "mixed"):
                ctx.set_precision(p)
                t[p] = ctx.sigma_c(qp, sysm.omega_ev, wl.eta, wl.n_lanczos)
            case["tda_mixed_vs_fp64_abs_ev"] = float(np.max(np.abs(t["mixed"] - t["fp64"])))
        ctx.close()
        out[name] = case
        log(f"smooth {name}: mixed vs oracle {case['mixed_vs_oracle_abs_ev']:.2e} eV")
    return out


def run_isdf(args):
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    base = args.workload if args.workload != "grid64_v128c512" else "grid48_v64c256"
    wl = gi.workload(base, name=base + "_smooth", smooth_sigma=1.0)
    t = time.perf_counter()
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    omega = gi.omega_grid(wl)
    n_mu = min(wl.n_r, args.isdf_ratio * wl.n_orb)
    pts = gi.random_grid_points(n_mu, wl.n_r, seed=wl.seed)
    log(f"isdf inputs {time.perf_counter() - t:.1f}s")
    box = tuple(k * wl.h for k in wl.grid)
    B = min(args.block, wl.n_orb)
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="fp64",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    # accuracy sample on the grid first (same interval for both products)
    ns = list(np.linspace(0, wl.n_orb - 1, 8).astype(int))
    m0 = int(qp[0])
    acc_L = 40
    a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
    s_grid = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    lo, hi = ctx.interval
    ctx.close()
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="fp64",
                    poly_degree=wl.poly_degree, poly_lo=lo, poly_hi=hi, reorth="full", block=B)
    # grid FP64 window for comparison: B vectors x 2 Lanczos steps
    ctx.lanczos_pairs([m0] * B, list(range(B)), [1] * B)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.lanczos_pairs([m0] * B, list(range(B)), [2] * B)
    torch.cuda.synchronize()
    grid_value = 1.0 / ((time.perf_counter() - t) / (2 * B) * wl.n_lanczos * wl.n_orb)
    log(f"grid fp64 window: {grid_value:.3g} spectra/s")
    torch.cuda.synchronize()
    t = time.perf_counter()
    km_iters = None
    if args.isdf_points == "kmeans":
        pts, km_iters = ctx.isdf_kmeans(pts, 50)
        n_mu = len(pts)
        torch.cuda.synchronize()
        log(f"isdf kmeans {time.perf_counter() - t:.1f}s, {km_iters} passes, {n_mu} points")
    elif args.isdf_points == "qrcp":
        rng = np.random.default_rng([wl.seed, 5])
        pts = ctx.isdf_qrcp(rng.standard_normal((wl.n_occ, n_mu + 16)),
                            rng.standard_normal((wl.n_emp, n_mu + 16)), n_mu)
        torch.cuda.synchronize()
        log(f"isdf qrcp {time.perf_counter() - t:.1f}s, {n_mu} points")
    ctx.isdf_setup(pts)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    log(f"isdf setup {t_setup:.1f}s")
    a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
    s_isdf = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    ctx.lanczos_pairs([m0] * B, list(range(B)), [1] * B)
    torch.cuda.synchronize()
    t = time.perf_counter()
    n_vec = 0
    for s in range(args.steps):
        n0 = (s * B) % wl.n_orb
        n1 = min(wl.n_orb, n0 + B)
        ctx.sigma_c_range([m0], n0, n1, omega, wl.eta, wl.n_lanczos)
        n_vec += n1 - n0
        log(f"isdf step {s} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ctx.close()
    print(json.dumps({
        "metric": "Sigma_c spectra/s with the ISDF product, FP64", "unit": "spectra/s",
        "value": round(n_vec / wl.n_orb / dt, 6), "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.grid), "n_occ": wl.n_occ,
                   "n_emp": wl.n_emp, "n_mu": n_mu,
                   "points": ("weighted K-means from seeded random grid points, "
                              f"{km_iters} assignment passes") if km_iters else
                   ("column-pivoted QR of a sketch (p = N_mu + 16)"
                    if args.isdf_points == "qrcp" else "seeded random grid points"),
                   "n_lanczos": wl.n_lanczos, "n_omega": wl.n_omega, "block": B,
                   "steps": args.steps},
        "ms_per_step": round(dt / max(args.steps, 1) * 1e3, 1),
        "setup_s": round(t_setup, 2),  # includes the K-means selection
        "grid_fp64_spectra_per_s": grid_value,
        "isdf_vs_grid_fp64": round(n_vec / wl.n_orb / dt / grid_value, 2),
        "isdf_vs_grid_sigma": {"max_abs_diff_ev": float(np.max(np.abs(s_isdf - s_grid))),
                               "max_abs_sigma_ev": float(np.max(np.abs(s_grid))),
                               "sample": f"8 start vectors, L={acc_L}, FP64, all omega"}}),
          flush=True)


def run_isdf_sweep(args):
    """Sigma error of the ISDF product against the grid product as the point
    count N_mu = r N_orb grows, for three point selections (seeded random
    points, weighted K-means from them, column-pivoted QR of a sketch), on
    the smooth-orbital variant of grid48_v64c256 (FP64): 8 start vectors of
    one QP state at L = 40, every frequency; selection + setup time."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    base = args.workload if args.workload != "grid64_v128c512" else "grid48_v64c256"
    wl = gi.workload(base, name=base + "_smooth", smooth_sigma=1.0)
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    omega = gi.omega_grid(wl)
    box = tuple(k * wl.h for k in wl.grid)
    ns = list(np.linspace(0, wl.n_orb - 1, 8).astype(int))
    m0 = int(qp[0])
    acc_L = 40
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="fp64",
                    poly_degree=wl.poly_degree, reorth="full", block=64)
    a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
    s_grid = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    smax = float(np.max(np.abs(s_grid)))
    rows = []
    for r in (2, 4, 8, 16):
        n_mu = min(wl.n_r, r * wl.n_orb)
        for how in ("random", "kmeans", "qrcp"):
            torch.cuda.synchronize()
            t = time.perf_counter()
            pts = gi.random_grid_points(n_mu, wl.n_r, seed=wl.seed)
            if how == "kmeans":
                pts, _ = ctx.isdf_kmeans(pts, 50)
            elif how == "qrcp":
                rng = np.random.default_rng([wl.seed, 5])
                pts = ctx.isdf_qrcp(rng.standard_normal((wl.n_occ, n_mu + 16)),
                                    rng.standard_normal((wl.n_emp, n_mu + 16)), n_mu)
            ctx.isdf_setup(pts)
            torch.cuda.synchronize()
            t_sel = time.perf_counter() - t
            ctx.set_option(G.KEY_ISDF, 1)
            a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
            s_is = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
            ctx.set_option(G.KEY_ISDF, 0)
            err = float(np.max(np.abs(s_is - s_grid)))
            rows.append({"r": r, "n_mu": int(len(pts)), "points": how,
                         "max_abs_err_ev": err, "rel_err": err / smax,
                         "select_and_setup_s": round(t_sel, 2)})
            log(f"isdf sweep r={r} {how}: {err:.3e} eV ({t_sel:.1f}s)")
    ctx.close()
    print(json.dumps({
        "metric": "Sigma_c error of the ISDF product against the grid product, FP64",
        "unit": "eV", "n_gpus": 1, "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.grid), "n_occ": wl.n_occ,
                   "n_emp": wl.n_emp, "sample": f"8 start vectors of m={m0}, L={acc_L}, "
                   f"{wl.n_omega} omega", "max_abs_sigma_ev": smax},
        "rows": rows}), flush=True)


def calibration_copy():
    """One elementwise kernel that reads 256 MiB and writes 256 MiB (the
    scale of the FETCH_SIZE and WRITE_SIZE counters)."""
    import torch
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    log("calibration copy of 256 MiB done")


def run_density(args):
    """The first GEMM with its fused row-dot alone (gwl_pair_density, mixed
    precision) at the headline launch configuration: --block pair vectors per
    launch on the headline orbitals, --steps launches timed (the cast and the
    partial sum around it included); with --calibrate-copy first, for counter
    runs."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    if args.calibrate_copy:
        calibration_copy()
    wl = gi.workload(args.workload)
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    box = tuple(k * wl.h for k in wl.grid)
    B = min(args.block, wl.n_vc)
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    x = torch.tensor(gi.random_pair_vectors(B, wl.n_vc, seed=3), device="cuda")
    ctx.pair_density(x, "mixed")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        ctx.pair_density(x, "mixed")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / max(args.steps, 1)
    ctx.close()
    flop = 2.0 * wl.n_r * wl.n_occ * wl.n_emp * B
    print(json.dumps({
        "metric": "first GEMM + row-dot (pair densities), mixed", "unit": "ms per launch",
        "value": round(dt * 1e3, 4), "n_gpus": 1, "higher_is_better": False, "dtype": "f16",
        "data": "synthetic", "tflops": round(flop / dt / 1e12, 1),
        "config": {"workload": wl.name, "block": B, "launches": args.steps}}), flush=True)


def run_potential(args):
    """The second GEMM alone (gwl_potential_product, mixed precision) at the
    headline launch configuration: --block seeded potentials per launch on the
    headline orbitals, --steps launches timed (the FP16 rounding of the
    potentials and the partial sum around it included); with --calibrate-copy
    first, for counter runs."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    if args.calibrate_copy:
        calibration_copy()
    wl = gi.workload(args.workload)
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    box = tuple(k * wl.h for k in wl.grid)
    B = min(args.block, wl.n_vc)
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    v = torch.tensor(np.random.default_rng(4).standard_normal((B, wl.n_r)), device="cuda")
    ctx.potential_product(v, "mixed")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        ctx.potential_product(v, "mixed")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / max(args.steps, 1)
    ctx.close()
    flop = 2.0 * wl.n_r * wl.n_occ * wl.n_emp * B
    print(json.dumps({
        "metric": "second GEMM (potential product), mixed", "unit": "ms per launch",
        "value": round(dt * 1e3, 4), "n_gpus": 1, "higher_is_better": False, "dtype": "f16",
        "data": "synthetic", "tflops": round(flop / dt / 1e12, 1),
        "config": {"workload": wl.name, "block": B, "launches": args.steps}}), flush=True)


def run_large(args):
    """The 128^3, 512 + 1,024-orbital configuration (FP32 orbitals, pair dim
    524,288): a steady-state window of the mixed-precision path at B vectors,
    extrapolated to the full spectrum, and the mixed-vs-FP64 error on a
    sample.  The window is the difference of a 1-step and a (1 + k)-step
    Lanczos run over the same B start vectors, so the coupling-vector build
    and the setup drop out."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    wl = gi.workload("grid128_v512c1024")
    t = time.perf_counter()
    phi = gi.make_orbitals(wl, dtype=np.float32, progress=log)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    omega = gi.omega_grid(wl)
    log(f"large inputs {time.perf_counter() - t:.1f}s ({phi.nbytes / 2**30:.1f} GiB FP32 orbitals)")
    B = min(args.block, wl.n_orb)
    box = tuple(k * wl.h for k in wl.grid)
    t = time.perf_counter()
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    del phi
    log(f"large setup {time.perf_counter() - t:.1f}s, interval {ctx.interval}")
    m0 = int(qp[0])
    pairs = ([m0] * B, list(range(B)))
    k = max(1, args.steps)

    def run(L):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.lanczos_pairs(pairs[0], pairs[1], [L] * B)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    run(1)
    if args.large_splits:
        # second-GEMM split sweep: one profiled 2-step window per split
        for sk in (int(x) for x in args.large_splits.split(",")):
            ctx.set_option(G.KEY_GEMM_SPLITK, sk)
            run(1)
            ctx.set_option(G.KEY_PROFILE, 1)
            run(2)
            tot = ctx.profile_totals()
            ctx.set_option(G.KEY_PROFILE, 0)
            log(f"large split {sk}: gemm2 {tot['gemm2'][0] / tot['gemm2'][1]:.1f} ms per launch")
        ctx.set_option(G.KEY_GEMM_SPLITK, 0)
    t1 = run(1)
    ctx.set_option(G.KEY_PROFILE, 1)
    tk = run(1 + k)
    prof = {kk: v for kk, v in ctx.profile_totals().items()}
    ctx.set_option(G.KEY_PROFILE, 0)
    per_step = (tk - t1) / k
    log(f"large window: L=1 {t1:.2f}s, L={1 + k} {tk:.2f}s, {per_step:.3f}s per step")
    per_vec_step = per_step / B
    value = 1.0 / (per_vec_step * wl.n_lanczos * wl.n_orb)
    flop_step = 4.0 * wl.n_r * wl.n_occ * wl.n_emp * wl.poly_degree * B
    # accuracy: mixed vs FP64 on a sample of start vectors, short fractions
    ns = list(np.linspace(0, wl.n_orb - 1, 4).astype(int))
    acc_L = 2
    a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
    s_mx = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    ctx.set_precision("fp64")
    a, b, n2, ol = ctx.lanczos_pairs([m0] * len(ns), ns, [acc_L] * len(ns))
    s_64 = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    ctx.close()
    kern = {kk: round(ms / cnt, 3) for kk, (ms, cnt, _) in prof.items() if cnt}
    gflop = 2.0 * wl.n_r * wl.n_occ * wl.n_emp * B
    print(json.dumps({
        "metric": "Sigma_c spectra/s, mixed, steady-state window extrapolated",
        "unit": "spectra/s", "value": value, "n_gpus": 1, "higher_is_better": True,
        "dtype": "f16", "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.grid), "n_occ": wl.n_occ,
                   "n_emp": wl.n_emp, "pair_dim": wl.n_vc, "orbitals": "FP32",
                   "n_lanczos": wl.n_lanczos, "n_omega": wl.n_omega, "block": B,
                   "window": f"{B} vectors, Lanczos runs of 1 and {1 + k} steps"},
        "seconds_per_lanczos_step": round(per_step, 4),
        "matvec_tflops": round(flop_step / per_step / 1e12, 1),
        "kernel_ms_per_launch": kern,
        "gemm_tflops": {kk: round(gflop / (v * 1e-3) / 1e12, 1) for kk, v in kern.items()
                        if kk.startswith("gemm")},
        "accuracy": {"max_abs_err_ev": float(np.max(np.abs(s_mx - s_64))),
                     "max_abs_sigma_ev": float(np.max(np.abs(s_64))),
                     "sample": f"{len(ns)} start vectors, L={acc_L}, mixed vs FP64 GPU"}}),
          flush=True)


def run_libref(args):
    """The two 16-bit GEMM kernels of one B-vector C-product against the
    vendor BLAS (torch.matmul, hipBLASLt) on the same shapes with plain
    operands: the second GEMM's shape with its A operand already formed, the
    first GEMM's shape with its [B N_v, N_r] product written out (neither
    fused step is included on the library side)."""
    import torch
    import gw_inputs as gi
    import paper_2310_20103_amd as G
    wl = gi.workload(args.workload)
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    B = min(args.block, wl.n_orb)
    box = tuple(n * wl.h for n in wl.grid)
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    m = [int(qp[0])] * B
    n = list(range(B))
    ctx.lanczos_pairs(m, n, [1] * B)
    ctx.set_option(G.KEY_PROFILE, 1)
    ours = {}
    for rep in range(3):
        ctx.lanczos_pairs(m, n, [2] * B)
        for k, (ms, cnt, _) in ctx.profile_totals().items():
            if cnt:
                ours[k] = min(ours.get(k, 1e30), ms / cnt)
    ctx.close()
    log("library kernels timed")
    M, Kc, Nr = B * wl.n_occ, wl.n_emp, wl.n_r
    flop = 2.0 * M * Kc * Nr

    def timed(fn, reps=5):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    lib = {}
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        a = torch.randn(M, Nr, device="cuda", dtype=dt)
        bm = torch.randn(Nr, Kc, device="cuda", dtype=dt)
        lib["gemm2_shape_" + name] = timed(lambda: a @ bm)
        del a, bm
        u = torch.randn(M, Kc, device="cuda", dtype=dt)
        pc = torch.randn(Nr, Kc, device="cuda", dtype=dt)
        out = torch.empty(M, Nr, device="cuda", dtype=dt)
        lib["gemm1_shape_" + name] = timed(lambda: torch.matmul(u, pc.t(), out=out))
        del u, pc, out
        torch.cuda.empty_cache()
        log(f"library {name} timed")
    tf = lambda ms: round(flop / (ms * 1e-3) / 1e12, 1)
    print(json.dumps({
        "metric": "16-bit GEMM ms per launch: fused kernels vs vendor BLAS on the same shapes",
        "config": {"workload": wl.name, "M": M, "N_c": Kc, "N_r": Nr, "block": B},
        "ours_ms": {k: round(v, 4) for k, v in ours.items()},
        "ours_tflops": {k: tf(v) for k, v in ours.items() if k.startswith("gemm")},
        "hipblaslt_ms": {k: round(v, 4) for k, v in lib.items()},
        "hipblaslt_tflops": {k: tf(v) for k, v in lib.items()},
        "note": "ours: gemm1 = FP16 GEMM with the fused row-dot (no C written), gemm2 = FP16 "
                "GEMM forming phi_v*V in staging; library: plain operands, unfused"}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=("headline", "uneven", "sched", "adjoint", "isdf",
                                       "isdf_sweep", "libref", "density", "potential",
                                       "large"),
                    default="headline")
    ap.add_argument("--pairs", type=int, default=256, help="uneven mode: pairs measured")
    ap.add_argument("--adjoint-store", action="store_true",
                    help="adjoint mode: keep the whole forward run instead of recomputing "
                         "it from checkpoints (when it fits)")
    ap.add_argument("--adjoint-workload", default="grid48_v64c256")
    ap.add_argument("--adjoint-lanczos", type=int, default=0, help="adjoint mode: L (0 = the workload's)")
    ap.add_argument("--adjoint-vectors", type=int, default=0,
                    help="adjoint mode: start vectors n in [0, this) (0 = all orbitals)")
    ap.add_argument("--adjoint-omega", type=int, default=0,
                    help="adjoint mode: frequencies (0 = the workload's)")
    ap.add_argument("--large-splits", default="",
                    help="large mode: comma-separated second-GEMM splits to time first")
    ap.add_argument("--uneven-blocks", default="",
                    help="uneven mode: comma-separated block sizes (default: 32,64,128,256 "
                         "with graphs and 128 without)")
    ap.add_argument("--isdf-ratio", type=int, default=4, help="isdf mode: N_mu / N_orb")
    ap.add_argument("--isdf-points", choices=("kmeans", "random", "qrcp"), default="kmeans",
                    help="isdf mode: interpolation points (K-means or the random start)")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--block", type=int, default=0,
                    help="vectors per batch (default 64 in adjoint mode, else 128)")
    ap.add_argument("--workload", default="grid64_v128c512")
    ap.add_argument("--fp64-window", type=int, default=2, help="Lanczos steps of the FP64 window")
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="Lanczos steps of the oracle sample (timed for cpu_baseline and "
                         "compared with the GPU paths)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel eagerly (no HIP graph replay), e.g. under counter "
                         "collection")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if not args.block:
        args.block = 64 if args.mode == "adjoint" else 128
    if args.mode == "sched":
        return run_sched(args)
    if args.mode == "isdf_sweep":
        return run_isdf_sweep(args)
    if args.mode == "density":
        return run_density(args)
    if args.mode == "potential":
        return run_potential(args)
    if args.mode == "uneven":
        return run_uneven(args)
    if args.mode == "adjoint":
        return run_adjoint(args)
    if args.mode == "isdf":
        return run_isdf(args)
    if args.mode == "libref":
        return run_libref(args)
    if args.mode == "large":
        return run_large(args)

    import torch
    import gw_inputs as gi
    import oracle  # the FP64 CPU reference: accuracy and cpu_baseline only
    import paper_2310_20103_amd as G

    assert torch.cuda.is_available(), "needs a GPU"
    if args.calibrate_copy:
        calibration_copy()
    wl = gi.workload(args.workload)
    t = time.perf_counter()
    phi = gi.make_orbitals(wl)
    eps = gi.make_energies(wl)
    qp = gi.frontier_states(eps, wl.n_occ, wl.n_qp_occ, wl.n_qp_emp)
    omega = gi.omega_grid(wl)
    log(f"inputs {time.perf_counter() - t:.1f}s")
    B = min(args.block, wl.n_orb)
    box = tuple(n * wl.h for n in wl.grid)
    t = time.perf_counter()
    ctx = G.Context(phi, eps, wl.n_occ, wl.grid, box, precision="mixed",
                    poly_degree=wl.poly_degree, reorth="full", block=B)
    lo, hi = ctx.interval
    log(f"setup {time.perf_counter() - t:.1f}s, interval [{lo:.4g}, {hi:.4g}] Ha^2")
    if args.no_graphs:
        ctx.set_option(G.KEY_GRAPHS, 0)

    blocks_per_spectrum = (wl.n_orb + B - 1) // B

    def step_args(s):
        m = int(qp[(s // blocks_per_spectrum) % len(qp)])
        nb = (s % blocks_per_spectrum) * B
        return m, nb, min(wl.n_orb, nb + B)

    # buffers and code objects: one Lanczos step over B vectors
    ctx.lanczos_pairs([int(qp[0])] * B, list(range(B)), [1] * B)
    for s in range(args.warmup):
        m, n0, n1 = step_args(s)
        ctx.sigma_c_range([m], n0, n1, omega, wl.eta, wl.n_lanczos)
    ctx.set_option(G.KEY_PROFILE, 1)
    prof = {"gemm1": [0.0, 0, 0], "gemm2": [0.0, 0, 0], "fft": [0.0, 0, 0]}
    n_vec = 0
    n_prod = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        m, n0, n1 = step_args(s)
        ctx.sigma_c_range([m], n0, n1, omega, wl.eta, wl.n_lanczos)
        n_vec += n1 - n0
        n_prod += ctx.query(G.KEY_LAST_C_MATVECS)
        for k, (ms, cnt, vec) in ctx.profile_totals().items():
            prof[k][0] += ms
            prof[k][1] += cnt
            prof[k][2] += vec
        log(f"step {s}: m={m} n=[{n0},{n1}) done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_option(G.KEY_PROFILE, 0)
    spectra = n_vec / wl.n_orb
    value = spectra / elapsed
    flop_vec = 4.0 * wl.n_r * wl.n_occ * wl.n_emp     # both GEMMs, one C-product
    matvec_tflops = flop_vec * n_prod / elapsed / 1e12

    # dominant kernel (largest event time) and its roofline
    dom = max(("gemm1", "gemm2"), key=lambda k: prof[k][0])
    ms, cnt, vec = prof[dom]
    flop_launch = 2.0 * wl.n_r * wl.n_occ * wl.n_emp * (vec / max(cnt, 1))
    achieved = flop_launch / (ms / max(cnt, 1) / 1e3) / 1e12 if cnt else 0.0
    kname = {"gemm1": "gemm1_f16", "gemm2": "gemm2_f16"}[dom]
    traffic = measured_traffic(kname, wl.name, B)
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_16BIT_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_16BIT_TFLOPS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch",
                "algorithmic_flop_per_launch": flop_launch,
                "kernel": kname, "launches": int(cnt),
                "avg_launch_ms": round(ms / max(cnt, 1), 4)}
    kernel_ms = {k: round(v[0], 2) for k, v in prof.items()}

    # plain FP64 GPU path end to end on one block (coupling vectors, Lanczos
    # with full reorthogonalisation, continued fraction, n-sum) at two short
    # lengths, extrapolated linearly in L
    ctx.set_precision("fp64")
    mw = int(qp[0])
    ctx.lanczos_pairs([mw] * B, list(range(B)), [1] * B)
    L1, L2 = args.fp64_window, 3 * args.fp64_window
    times64 = {}
    c64 = 0
    for Lw in (L1, L2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.sigma_c_range([mw], 0, B, omega, wl.eta, Lw)
        torch.cuda.synchronize()
        times64[Lw] = time.perf_counter() - t
        c64 += ctx.query(G.KEY_LAST_C_MATVECS)
        log(f"fp64 block, L = {Lw}: {times64[Lw]:.1f}s")
    slope = (times64[L2] - times64[L1]) / (L2 - L1)
    t_block64 = times64[L2] + (wl.n_lanczos - L2) * slope
    fp64_value = B / wl.n_orb / t_block64
    fp64_tflops = flop_vec * B * wl.poly_degree / slope / 1e12

    # accuracy against the FP64 oracle at full size: Sigma_mm(omega, n) of two
    # start vectors at L = acc_L (the first one also times the oracle)
    acc_L = args.cpu_steps
    ns = [0, wl.n_orb - 1]
    pr = oracle.Problem(phi, eps, wl.n_occ, wl.grid, wl.h, dense=False)
    refs, t_or = [], []
    for n in ns:
        sg, dt = oracle_vector(wl, pr, mw, n, acc_L, lo, hi, omega)
        refs.append(sg)
        t_or.append(dt)
        log(f"oracle vector n={n}: {dt:.1f}s")
    res = {}
    for p in ("fp64", "mixed"):
        ctx.set_precision(p)
        a, b, n2, ol = ctx.lanczos_pairs([mw] * len(ns), ns, [acc_L] * len(ns))
        res[p] = ctx.sigma_from_coeffs(ns, a, b, n2, ol, omega, wl.eta)
    refs = np.array(refs)
    smax = float(np.max(np.abs(refs)))
    ctx.close()
    stress = smooth_stress_error(G, gi)

    line = {
        "metric": METRIC, "value": round(value, 6), "unit": "spectra/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / max(args.steps, 1) * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.grid), "box_bohr": wl.box,
                   "n_occ": wl.n_occ, "n_emp": wl.n_emp, "pair_dim": wl.n_vc,
                   "n_lanczos": wl.n_lanczos, "poly_degree": wl.poly_degree,
                   "n_omega": wl.n_omega, "eta_ev": wl.eta, "block": B, "reorth": "full",
                   "step": f"{B} start vectors of one QP state through the full path"},
        "matvec_tflops": round(matvec_tflops, 2),
        "kernel_event_ms": kernel_ms,
        "fp64_gpu": {"spectra_per_s": fp64_value, "matvec_tflops": round(fp64_tflops, 2),
                     "window": (f"{B} start vectors end to end (sigma_c_range) at L = {L1} "
                                f"and {L2}: {times64[L1]:.2f} s, {times64[L2]:.2f} s; linear "
                                f"in L to {wl.n_lanczos}")},
        "mixed_vs_fp64": round(value / fp64_value, 2),
        "accuracy": {"fp64_vs_oracle_rel": float(np.max(np.abs(res["fp64"] - refs)) / smax),
                     "mixed_vs_oracle_abs_ev": float(np.max(np.abs(res["mixed"] - refs))),
                     "mixed_vs_oracle_rel": float(np.max(np.abs(res["mixed"] - refs)) / smax),
                     "max_abs_sigma_ev": smax,
                     "sample": (f"Sigma_mm(omega, n), m={mw}, n in {ns}, L={acc_L}, "
                                f"{len(omega)} omega, against the oracle's matrix-free FP64 "
                                "route (white-noise orbitals: Sigma is small here)")},
        "accuracy_smooth": stress,
        "roofline": roofline,
    }
    line["cpu_baseline"] = cpu_baseline(wl, float(sum(t_or)), mw, ns, acc_L)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
