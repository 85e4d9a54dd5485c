// Vector-Jacobian product of Sigma_c (gwl_sigma_c_vjp).
//
// Forward: the same path as gwl_sigma_c in FP64 without reorthogonalisation
// (so the recurrence can be recomputed exactly).  When they fit in
// GWL_ADJOINT_STORE_MAX, every step's Chebyshev iterates t_j (t_0 = q_k),
// coupling parts K Delta^1/2 t_j and w_k = p_g(C) q_k are kept from the
// forward; otherwise the forward checkpoints (q_{k-1}, q_k) and the slot state
// every ceil(sqrt(L)) steps, and the backward recomputes, segment by segment
// (last first), the Lanczos vectors from the checkpoint and then, per step,
// the product with its iterates (two more p_g(C) products per step; the same
// kernels in the same order, so both routes agree bitwise).  Backward, per
// block of start vectors: continued-fraction adjoint; then for each step k
// (last first) the reverse Lanczos step gives w_bar_k, and the reverse
// Chebyshev recurrence
// applied to w_bar_k gives D w_bar_k (added to q_bar_k) together with the
// outer products s_j t_{j-1}^T that make up C_bar.  C_bar is pushed into
// Delta_bar directly and into a dense K_bar; the coupling vectors' adjoint
// gives Delta_bar and k_bar.  At the end K_bar and k_bar are contracted with
// the pair potentials V[phi_v phi_c] (plain rocBLAS GEMMs) into the orbital
// gradient, and Delta_bar into the energy gradient.
#include <rocblas/rocblas.h>

#include "context.h"

namespace {

#define GWL_BLAS(call)                                                           \
  do {                                                                           \
    rocblas_status s_ = (call);                                                  \
    if (s_ != rocblas_status_success)                                            \
      throw ::gwl::Error{GWL_EDEVICE, std::string(#call) + ": rocblas status " + \
                                          std::to_string((int)s_)};              \
  } while (0)

struct Blas {
  rocblas_handle h = nullptr;
  ~Blas() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

}  // namespace

extern "C" gwl_status gwl_sigma_c_vjp(gwl_ctx* ctx, const int* qp_states, int n_qp,
                                      const double* omega_ev, int n_omega, double eta_ev,
                                      int n_lanczos, const double* grad_sigma,
                                      double* sigma_out, double* grad_energies,
                                      double* grad_orbitals) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    gwl_ctx& c = *ctx;
    GWL_CHECK(!c.tda && !c.quadrature && !c.isdf_on, GWL_EUNSUPPORTED,
              "the adjoint covers the polynomial method on the grid only (not Tamm-Dancoff, "
              "quadrature or ISDF)");
    GWL_CHECK(n_qp >= 1 && n_omega >= 1, GWL_EINVAL, "need n_qp >= 1 and n_omega >= 1");
    GWL_CHECK(qp_states && omega_ev && grad_sigma && grad_energies && grad_orbitals, GWL_EINVAL,
              "null pointer");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    GWL_CHECK(n_lanczos >= 1 && n_lanczos <= 1024, GWL_EINVAL,
              "n_lanczos must be in [1, 1024] for the adjoint");
    GWL_CHECK(finite_all(omega_ev, n_omega), GWL_EINVAL, "non-finite frequency");
    GWL_CHECK(finite_all(grad_sigma, (size_t)n_qp * n_omega * 2), GWL_EINVAL,
              "non-finite cotangent");
    for (int i = 0; i < n_qp; ++i)
      GWL_CHECK(qp_states[i] >= 0 && qp_states[i] < c.n_orb, GWL_EINVAL, "qp state out of range");
    const long nvc = c.nvc;
    const int g = c.poly_degree;
    const int L = n_lanczos;
    const int P = n_qp * c.n_orb;
    GWL_CHECK((double)nvc * nvc * 8 < 64e9, GWL_EUNSUPPORTED,
              "adjoint holds the dense coupling cotangent: N_vc too large");
    hipStream_t st = c.stream;
    const int saved_prec = c.precision, saved_reorth = c.reorth;
    c.precision = GWL_FP64;
    c.reorth = GWL_REORTH_NONE;
    struct Restore {
      gwl_ctx& c;
      int p, r;
      ~Restore() {
        c.precision = p;
        c.reorth = r;
      }
    } restore{c, saved_prec, saved_reorth};

    const int B = std::max(1, std::min(P, c.block > 0 ? c.block : 64));
    c.ensure_work(B, L, false);
    const int S = c.auto_splitk(B, GWL_FP64);
    const int seg = std::max(1, (int)std::ceil(std::sqrt((double)L)));
    const int nseg = (L + seg - 1) / seg;
    PairGeom pg = c.pair_geom();
    const double lo = c.poly_lo, hi = c.poly_hi;
    const size_t vec = (size_t)B * nvc;

    // pair list (m, n), qp index per pair
    std::vector<int> m(P), n(P), q(P), len(P, L);
    for (int a = 0; a < n_qp; ++a)
      for (int j = 0; j < c.n_orb; ++j) {
        const int p = a * c.n_orb + j;
        m[p] = qp_states[a];
        n[p] = j;
        q[p] = a;
      }
    std::vector<double> en(P), et(P), om(n_omega);
    for (int p = 0; p < P; ++p) {
      en[p] = c.eps_ha[n[p]];
      et[p] = n[p] < c.nv ? 1.0 : -1.0;
    }
    for (int i = 0; i < n_omega; ++i) om[i] = omega_ev[i] / kHartreeEv;

    // buffers
    DevBuf<double> Pb, ckq, ckqp, segq, T, KT, Sv, KS, U, V, wk, wbar, qb0, qb1, qb2, pend, dbar,
        dbar_tot, Kbar, kbar, abar, bbar, nbar, ebar, sig, Gd, e_d, eta_d, om_d, grad_int;
    DevBuf<int> ck_state, qidx_d, slot_pair, mrow_d, nrow_d, flen;
    DevBuf<double> ck_amax, ck_bprev;
    DevBuf<unsigned char> tscr;
    Pb.ensure(vec);
    // kept iterates per step k: t_0..t_g, K~t_0..K~t_{g-1}, w_k; then q_L and q_{-1}
    const size_t per_step = (size_t)(2 * g + 2) * vec;
    bool store = c.adjoint_store &&
                 ((size_t)L * per_step + 2 * vec) * sizeof(double) <= GWL_ADJOINT_STORE_MAX;
    DevBuf<double> It;
    if (store) {
      try {
        It.ensure((size_t)L * per_step + 2 * vec);
      } catch (const Error& e) {
        // not enough free device memory: recompute from checkpoints instead
        if (e.code != GWL_ENOMEM) throw;
        (void)hipGetLastError();
        store = false;
      }
    }
    c.adjoint_stored = store ? 1 : 0;
    if (!store) {
      ckq.ensure((size_t)nseg * vec);
      ckqp.ensure((size_t)nseg * vec);
      ck_state.ensure((size_t)nseg * 2 * B);
      ck_amax.ensure((size_t)nseg * B);
      ck_bprev.ensure((size_t)nseg * B);
      segq.ensure((size_t)(seg + 1) * vec);
      T.ensure((size_t)(g + 1) * vec);
      KT.ensure((size_t)g * vec);
      wk.ensure(vec);
    }
    double* const q_last = store ? It.p + (size_t)L * per_step : nullptr;
    double* const q_m1 = store ? q_last + vec : nullptr;
    Sv.ensure((size_t)(g + 1) * vec);
    KS.ensure((size_t)(g + 1) * vec);
    U.ensure((size_t)g * vec);
    V.ensure((size_t)g * vec);
    wbar.ensure(vec);
    qb0.ensure(vec);
    qb1.ensure(vec);
    qb2.ensure(vec);
    pend.ensure(B);
    dbar.ensure(vec);
    dbar_tot.ensure(nvc);
    Kbar.ensure((size_t)nvc * nvc);
    kbar.ensure((size_t)P * nvc);
    abar.ensure((size_t)P * L);
    bbar.ensure((size_t)P * L);
    nbar.ensure(P);
    ebar.ensure(P);
    sig.ensure((size_t)P * n_omega * 2);
    Gd.ensure((size_t)n_qp * n_omega * 2);
    e_d.ensure(P);
    eta_d.ensure(P);
    om_d.ensure(n_omega);
    qidx_d.ensure(P);
    flen.ensure(P);
    slot_pair.ensure(B);
    tscr.ensure((size_t)B * L * n_omega * 16);
    grad_int.ensure((size_t)(c.gd.nvp + c.gd.ncp) * c.gd.nrp);
    GWL_HIP(hipMemcpy(Gd.p, grad_sigma, sizeof(double) * n_qp * n_omega * 2, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(e_d.p, en.data(), sizeof(double) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(eta_d.p, et.data(), sizeof(double) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(om_d.p, om.data(), sizeof(double) * n_omega, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(qidx_d.p, q.data(), sizeof(int) * P, hipMemcpyHostToDevice));

    Blas blas;
    GWL_BLAS(rocblas_create_handle(&blas.h));
    GWL_BLAS(rocblas_set_stream(blas.h, st));
    const double one = 1.0, zero = 0.0;

    c.coef_a.ensure((size_t)P * L);
    c.coef_b.ensure((size_t)P * L);
    c.norm2.ensure(P);
    c.out_len.ensure(P);
    GWL_HIP(hipMemsetAsync(c.coef_a.p, 0, sizeof(double) * (size_t)P * L, st));
    GWL_HIP(hipMemsetAsync(c.coef_b.p, 0, sizeof(double) * (size_t)P * L, st));
    SlotState ss;
    ss.pair = c.s_pair.p;
    ss.k = c.s_k.p;
    ss.len = c.s_len.p;
    ss.dead = c.s_dead.p;
    ss.amax = c.s_amax.p;
    ss.bprev = c.s_bprev.p;
    ss.coef_a = c.coef_a.p;
    ss.coef_b = c.coef_b.p;
    ss.out_len = c.out_len.p;
    ss.norm2 = c.norm2.p;
    ss.ld = L;

    // one Lanczos step (no reorthogonalisation) of all slots from q, qprev
    auto fwd_step = [&]() {
      c.apply_d_batch(B, c.q.p, c.w.p, GWL_FP64, false);
      lz_alpha(ss, B, c.q.p, c.qprev.p, c.w.p, nvc, st);
      lz_beta(ss, B, c.q.p, c.qprev.p, c.w.p, nullptr, 0, 0, nvc, st);
    };
    // w = p_g(C) t_0 for the vectors t_0 = Ti[0], keeping the iterates
    // t_1..t_g in Ti[1..g] and K~t_j = K Delta^1/2 t_j in KTi[0..g-1]
    // (the same launches as Context::apply_d_batch, plus the K~t_j output)
    auto cheb_iterates = [&](double* Ti, double* KTi, double* w) {
      c.cast(B, Ti, GWL_FP64);
      for (int j = 0; j < g; ++j) {
        c.k_product(B, GWL_FP64, S);
        combine<double, double>(pg, B, S, reinterpret_cast<const double*>(c.ypart.p),
                                Ti + (size_t)j * vec, j > 0 ? Ti + (size_t)(j - 1) * vec : nullptr,
                                Ti + (size_t)(j + 1) * vec, w, j == 0 ? 1 : 2, lo, hi,
                                c.cheb[0], c.cheb[j + 1], j + 1 < g ? c.u64.p : nullptr, st,
                                KTi + (size_t)j * vec);
      }
    };
    // one forward step that keeps its iterates (store route)
    auto fwd_step_store = [&](int k) {
      double* Ti = It.p + (size_t)k * per_step;
      double* KTi = Ti + (size_t)(g + 1) * vec;
      double* Wi = Ti + (size_t)(2 * g + 1) * vec;
      GWL_HIP(hipMemcpyAsync(Ti, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
      cheb_iterates(Ti, KTi, Wi);
      GWL_HIP(hipMemcpyAsync(c.w.p, Wi, vec * 8, hipMemcpyDeviceToDevice, st));
      lz_alpha(ss, B, c.q.p, c.qprev.p, c.w.p, nvc, st);
      lz_beta(ss, B, c.q.p, c.qprev.p, c.w.p, nullptr, 0, 0, nvc, st);
    };
    auto save_state = [&](int sgi) {
      GWL_HIP(hipMemcpyAsync(ckq.p + (size_t)sgi * vec, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(ckqp.p + (size_t)sgi * vec, c.qprev.p, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(ck_state.p + (size_t)sgi * 2 * B, c.s_k.p, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(ck_state.p + (size_t)sgi * 2 * B + B, c.s_dead.p, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(ck_amax.p + (size_t)sgi * B, c.s_amax.p, B * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(ck_bprev.p + (size_t)sgi * B, c.s_bprev.p, B * 8, hipMemcpyDeviceToDevice, st));
    };
    auto load_state = [&](int sgi) {
      GWL_HIP(hipMemcpyAsync(c.q.p, ckq.p + (size_t)sgi * vec, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.qprev.p, ckqp.p + (size_t)sgi * vec, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_k.p, ck_state.p + (size_t)sgi * 2 * B, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_dead.p, ck_state.p + (size_t)sgi * 2 * B + B, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_amax.p, ck_amax.p + (size_t)sgi * B, B * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_bprev.p, ck_bprev.p + (size_t)sgi * B, B * 8, hipMemcpyDeviceToDevice, st));
    };

    for (int p0 = 0; p0 < P; p0 += B) {
      const int nbk = std::min(B, P - p0);
      // slot -> pair map; unused slots carry pair -1
      std::vector<int> hp(B, -1), hl(B, 0), sl(B);
      for (int b = 0; b < nbk; ++b) {
        hp[b] = p0 + b;
        hl[b] = L;
      }
      for (int b = 0; b < B; ++b) sl[b] = b;
      GWL_HIP(hipStreamSynchronize(st));
      GWL_HIP(hipMemcpy(c.s_pair.p, hp.data(), B * 4, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(slot_pair.p, hp.data(), B * 4, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.s_len.p, hl.data(), B * 4, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.s_slots.p, sl.data(), B * 4, hipMemcpyHostToDevice));
      GWL_HIP(hipMemsetAsync(c.q.p, 0, vec * 8, st));
      // ---- forward
      c.coupling_batch(nbk, m.data() + p0, n.data() + p0, c.q.p, nvc);
      GWL_HIP(hipMemcpyAsync(Pb.p, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
      lz_start(ss, B, c.s_slots.p, nbk, c.q.p, c.qprev.p, nullptr, 0, nvc, st);
      if (store) {
        GWL_HIP(hipMemcpyAsync(q_m1, c.qprev.p, vec * 8, hipMemcpyDeviceToDevice, st));
        for (int k = 0; k < L; ++k) fwd_step_store(k);
        GWL_HIP(hipMemcpyAsync(q_last, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
      } else {
        for (int k = 0; k < L; ++k) {
          if (k % seg == 0) save_state(k / seg);
          fwd_step();
        }
      }
      // final lengths (the segment recompute below rewrites out_len step by step)
      GWL_HIP(hipMemcpyAsync(flen.p + p0, c.out_len.p + p0, nbk * 4, hipMemcpyDeviceToDevice, st));
      // ---- continued-fraction adjoint (and the forward Sigma per pair)
      adj_cfrac(nbk, c.coef_a.p + (size_t)p0 * L, c.coef_b.p + (size_t)p0 * L,
                flen.p + p0, c.norm2.p + p0, L, e_d.p + p0, eta_d.p + p0, qidx_d.p + p0,
                om_d.p, n_omega, eta_ev / kHartreeEv, Gd.p, tscr.p, abar.p + (size_t)p0 * L,
                bbar.p + (size_t)p0 * L, nbar.p + p0, ebar.p + p0, sig.p + (size_t)p0 * n_omega * 2,
                st);
      // ---- backward
      double* qbn = qb0.p;  // q_bar_{k+1}
      double* qbc = qb1.p;  // q_bar_k
      double* qbp = qb2.p;  // q_bar_{k-1}
      GWL_HIP(hipMemsetAsync(qbn, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(qbc, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(qbp, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(pend.p, 0, B * 8, st));
      GWL_HIP(hipMemsetAsync(dbar.p, 0, vec * 8, st));
      // backward step k from q_{k+1}, q_k, q_{k-1}, w_k and the iterates of p_g(C) q_k
      auto reverse_step = [&](int k, const double* qn, const double* qk, const double* qpv,
                              const double* Ti, const double* KTi, const double* Wi) {
        // reverse Lanczos step k
        adj_lanczos_step(k, B, slot_pair.p, flen.p, L, c.coef_a.p, c.coef_b.p, abar.p,
                         bbar.p, qn, qk, qpv, Wi, qbn, qbc, qbp, wbar.p, pend.p, nvc, st);
        // reverse Chebyshev recurrence on x = w_bar_k
        adj_scale_copy(Sv.p + (size_t)g * vec, wbar.p, c.cheb[g], (long)vec, st);
        c.cast(B, Sv.p + (size_t)g * vec, GWL_FP64);
        for (int j = g; j >= 1; --j) {
          c.k_product(B, GWL_FP64, S);
          adj_combine(pg, B, S, reinterpret_cast<const double*>(c.ypart.p),
                      Sv.p + (size_t)j * vec, j < g ? Sv.p + (size_t)(j + 1) * vec : nullptr,
                      wbar.p, c.cheb[j - 1], j >= 2 ? 2.0 : 1.0, lo, hi,
                      Sv.p + (size_t)(j - 1) * vec, KS.p + (size_t)j * vec,
                      j - 1 >= 1 ? c.u64.p : nullptr, st);
        }
        // C_bar = (2/(hi-lo)) [sum_{j>=2} 2 s_j t_{j-1}^T + s_1 t_0^T]
        for (int j = 1; j <= g; ++j) {
          const double alpha = (2.0 / (hi - lo)) * (j >= 2 ? 2.0 : 1.0);
          adj_dbar_uv(pg, B, Sv.p + (size_t)j * vec, KS.p + (size_t)j * vec,
                      Ti + (size_t)(j - 1) * vec, KTi + (size_t)(j - 1) * vec, alpha,
                      2.0 * alpha, dbar.p, U.p + (size_t)(j - 1) * vec,
                      V.p + (size_t)(j - 1) * vec, st);
        }
        // K_bar += sum_rows U^T V  (column-major view: Kbar += V_cm U_cm^T)
        GWL_BLAS(rocblas_dgemm(blas.h, rocblas_operation_none, rocblas_operation_transpose,
                               (rocblas_int)nvc, (rocblas_int)nvc, (rocblas_int)(g * B), &one,
                               V.p, (rocblas_int)nvc, U.p, (rocblas_int)nvc, &one, Kbar.p,
                               (rocblas_int)nvc));
        // q_bar_k += D w_bar_k
        adj_axpy(qbc, Sv.p, 1.0, (long)vec, st);
        // rotate: q_bar_{k+1} <- q_bar_k <- q_bar_{k-1} <- 0
        double* t = qbn;
        qbn = qbc;
        qbc = qbp;
        qbp = t;
        GWL_HIP(hipMemsetAsync(qbp, 0, vec * 8, st));
      };
      if (store) {
        for (int k = L - 1; k >= 0; --k) {
          const double* Ti = It.p + (size_t)k * per_step;
          const double* qn = k + 1 < L ? Ti + per_step : q_last;
          const double* qpv = k > 0 ? Ti - per_step : q_m1;
          reverse_step(k, qn, Ti, qpv, Ti, Ti + (size_t)(g + 1) * vec,
                       Ti + (size_t)(2 * g + 1) * vec);
        }
      } else {
        for (int sgi = nseg - 1; sgi >= 0; --sgi) {
          const int k0 = sgi * seg, k1 = std::min(L, k0 + seg);
          load_state(sgi);
          GWL_HIP(hipMemcpyAsync(segq.p, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
          for (int k = k0; k < k1; ++k) {
            fwd_step();
            GWL_HIP(hipMemcpyAsync(segq.p + (size_t)(k - k0 + 1) * vec, c.q.p, vec * 8,
                                   hipMemcpyDeviceToDevice, st));
          }
          const double* qprev0 = ckqp.p + (size_t)sgi * vec;
          for (int k = k1 - 1; k >= k0; --k) {
            const double* qk = segq.p + (size_t)(k - k0) * vec;
            const double* qn = segq.p + (size_t)(k - k0 + 1) * vec;
            const double* qpv = k > k0 ? segq.p + (size_t)(k - k0 - 1) * vec : qprev0;
            // recompute w_k = p_g(C) q_k keeping t_0..t_{g-1} and K Delta^1/2 t_j
            GWL_HIP(hipMemcpyAsync(T.p, qk, vec * 8, hipMemcpyDeviceToDevice, st));
            cheb_iterates(T.p, KT.p, wk.p);
            reverse_step(k, qn, qk, qpv, T.p, KT.p, wk.p);
          }
        }
      }
      // start vector adjoint: q_bar_0 is now in qbn
      adj_start(B, slot_pair.p, c.norm2.p, nbar.p, Pb.p, qbn, c.sdelta.p, dbar.p, kbar.p, nvc,
                st);
      adj_sum_rows(dbar_tot.p, dbar.p, B, nvc, st);
    }

    // ---- energies: Delta_bar -> e_bar, plus the explicit z_n terms
    std::vector<double> dtot(nvc), eb(P);
    GWL_HIP(hipStreamSynchronize(st));
    It.release();  // the kept iterates are done with; the orbital stage needs the room
    GWL_HIP(hipMemcpy(dtot.data(), dbar_tot.p, nvc * 8, hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(eb.data(), ebar.p, P * 8, hipMemcpyDeviceToHost));
    std::vector<double> ge(c.n_orb, 0.0);
    for (int v = 0; v < c.nv; ++v)
      for (int cc = 0; cc < c.nc; ++cc) {
        const double d = dtot[(size_t)v * c.nc + cc];
        ge[v] -= d;
        ge[c.nv + cc] += d;
      }
    for (int p = 0; p < P; ++p) ge[n[p]] += eb[p];
    for (int a = 0; a < c.n_orb; ++a) grad_energies[a] = ge[a] / kHartreeEv;

    // ---- orbitals
    const long ld = c.gd.nrp;
    DevBuf<double> VB, W, Sym, Vnm, Vk;
    VB.ensure((size_t)nvc * ld);
    W.ensure((size_t)nvc * ld);
    Sym.ensure((size_t)nvc * nvc);
    Vnm.ensure((size_t)P * ld);
    Vk.ensure((size_t)P * ld);
    const int chunk = std::min<long>(B, nvc);
    double* rho = reinterpret_cast<double*>(c.rho.p);
    double* fx = reinterpret_cast<double*>(c.fftx.p);
    for (long q0 = 0; q0 < nvc; q0 += chunk) {
      const int cnt = (int)std::min<long>(chunk, nvc - q0);
      adj_pair_density(c.psi_t.p, ld, c.nv, c.nc, c.gd.nvp, q0, cnt, rho, st);
      poisson_launch<double>(c.pg64, rho, ld, 0, 1, VB.p + (size_t)q0 * ld, ld, cnt,
                             reinterpret_cast<cplx<double>*>(fx), st);
    }
    std::vector<int> mr(P), nr_(P);
    for (int p = 0; p < P; ++p) {
      mr[p] = c.orb_row(m[p]);
      nr_[p] = c.orb_row(n[p]);
    }
    mrow_d.ensure(P);
    nrow_d.ensure(P);
    GWL_HIP(hipMemcpy(mrow_d.p, mr.data(), P * 4, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(nrow_d.p, nr_.data(), P * 4, hipMemcpyHostToDevice));
    for (int p0 = 0; p0 < P; p0 += B) {
      const int cnt = std::min(B, P - p0);
      pair_product(c.psi_t.p, ld, (int)c.nr, mrow_d.p + p0, nrow_d.p + p0, cnt, rho, st);
      poisson_launch<double>(c.pg64, rho, ld, 0, 1, Vnm.p + (size_t)p0 * ld, ld, cnt,
                             reinterpret_cast<cplx<double>*>(fx), st);
    }
    adj_symmetrize(Sym.p, Kbar.p, nvc, st);
    // W[(vc)][r] = sum_q Sym[(vc)][q] VB[q][r] + sum_p kbar[p][(vc)] Vnm[p][r]
    GWL_BLAS(rocblas_dgemm(blas.h, rocblas_operation_none, rocblas_operation_none,
                           (rocblas_int)ld, (rocblas_int)nvc, (rocblas_int)nvc, &one, VB.p,
                           (rocblas_int)ld, Sym.p, (rocblas_int)nvc, &zero, W.p, (rocblas_int)ld));
    GWL_BLAS(rocblas_dgemm(blas.h, rocblas_operation_none, rocblas_operation_transpose,
                           (rocblas_int)ld, (rocblas_int)nvc, (rocblas_int)P, &one, Vnm.p,
                           (rocblas_int)ld, kbar.p, (rocblas_int)nvc, &one, W.p, (rocblas_int)ld));
    // Vk[p][r] = sum_q kbar[p][q] VB[q][r]
    GWL_BLAS(rocblas_dgemm(blas.h, rocblas_operation_none, rocblas_operation_none,
                           (rocblas_int)ld, (rocblas_int)P, (rocblas_int)nvc, &one, VB.p,
                           (rocblas_int)ld, kbar.p, (rocblas_int)nvc, &zero, Vk.p, (rocblas_int)ld));
    GWL_HIP(hipMemsetAsync(grad_int.p, 0, grad_int.n * 8, st));
    adj_orb_grad_vc(c.psi_t.p, W.p, ld, (int)c.nr, c.nv, c.nc, c.gd.nvp, c.dv, grad_int.p, st);
    adj_orb_grad_nm(c.psi_t.p, Vk.p, ld, (int)c.nr, mrow_d.p, nrow_d.p, P, c.dv, grad_int.p, st);
    adj_gather_orbitals(grad_int.p, ld, (int)c.nr, c.nv, c.gd.nvp, c.n_orb, grad_orbitals, st);

    if (sigma_out) {
      c.sig_sum.ensure((size_t)n_qp * n_omega * 2);
      sum_groups(sig.p, n_qp, c.n_orb, n_omega, c.sig_sum.p, st);
      GWL_HIP(hipMemcpyAsync(sigma_out, c.sig_sum.p, sizeof(double) * n_qp * n_omega * 2,
                             hipMemcpyDeviceToHost, st));
    }
    GWL_HIP(hipStreamSynchronize(st));
    set_error("");
    return GWL_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GWL_EDEVICE;
  }
}
