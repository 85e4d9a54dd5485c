// Vector-Jacobian product of Sigma_c (gwl_sigma_c_vjp).
//
// Forward: the same path as gwl_sigma_c in FP64 without reorthogonalisation
// (so the recurrence can be recomputed exactly), in segments of S_L steps.
// By default S_L = ceil(sqrt(L)): the forward keeps only (q_{k-1}, q_k) and the
// slot state at each segment start, and the backward recomputes one segment
// at a time (last first), keeping for each of its steps the Chebyshev
// iterates t_0..t_g of p_g(C) q_k, their coupling parts K Delta^1/2 t_j, the
// product w_k and the Hartree potentials V[rho(Delta^1/2 t_j)] that the FFT
// Poisson solve forms inside each C-product.  With GWL_KEY_ADJOINT_STORE the
// whole run is one segment kept by the forward itself when it fits; else the
// forward keeps the last segment's iterates itself (it ends there), so the
// backward recomputes every segment but the last.
//
// Split form (gwl_sigma_c_vjp_forward, then gwl_sigma_c_vjp_backward): the
// forward runs every block of start vectors, returns Sigma and keeps each
// block's checkpoints, start vectors, V[phi_n phi_m] and Lanczos coefficients
// in the context; the backward takes them up for any cotangent without
// running the forward again (an autograd forward and backward then run the
// recurrence once forward and once in the recompute).
//
// Backward, per block of start vectors: continued-fraction adjoint; then for
// each step k (last first) the reverse Lanczos step gives w_bar_k, and the
// reverse Chebyshev recurrence applied to w_bar_k gives D w_bar_k (added to
// q_bar_k) together with the outer products s_j t_{j-1}^T that make up C_bar.
// C_bar goes into Delta_bar at once; its coupling part goes into the orbital
// gradient at once through the factored contraction of adj_zgemm, which pairs
// each pair vector with the potential of its partner (no N_vc x N_vc
// cotangent, no per-pair potentials on the grid).  The start vectors'
// adjoint gives Delta_bar and k_bar, whose orbital terms go the same way
// (k_bar with V[phi_n phi_m], and V[rho(k_bar)] with phi_m and phi_n).
#include "context.h"

using namespace gwl;

namespace {

enum class VjpMode { Full, Forward, Backward };

// What gwl_sigma_c_vjp_forward keeps for the backward calls that follow it:
// the call's arguments, the options it ran with, and per block of start
// vectors the segment checkpoints, the start vectors P_nm and V[phi_n phi_m];
// per pair the Lanczos coefficients and final lengths.
struct VjpSaved {
  std::vector<int> qp;
  std::vector<double> omega;
  int n_begin = 0, n_end = 0, L = 0, B = 0, g = 0, S = 0, kernels = 0;
  double eta_ev = 0, lo = 0, hi = 0;
  long nvc = 0, nrp = 0;
  DevBuf<double> ckq, ckqp, ck_amax, ck_bprev, Pb, Vnm, coef_a, coef_b, norm2;
  DevBuf<int> ck_state, out_len, flen;
};

gwl_status vjp_run(gwl_ctx* ctx, VjpMode mode, const int* qp_states, int n_qp, int n_begin,
                   int n_end, const double* omega_ev, int n_omega, double eta_ev, int n_lanczos,
                   const double* grad_sigma, double* sigma_out, double* grad_energies,
                   void* grad_orbitals) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    gwl_ctx& c = *ctx;
    const bool fwd_only = mode == VjpMode::Forward, bwd_only = mode == VjpMode::Backward;
    const bool persist = mode != VjpMode::Full;  // checkpoints of every block kept
    std::shared_ptr<VjpSaved> sv;
    if (bwd_only) {
      sv = std::static_pointer_cast<VjpSaved>(c.vjp_saved);
      GWL_CHECK(sv != nullptr, GWL_EINVAL,
                "no saved forward: call gwl_sigma_c_vjp_forward on this context first");
      GWL_CHECK(sv->lo == c.poly_lo && sv->hi == c.poly_hi && sv->g == c.poly_degree &&
                    sv->nvc == c.nvc && sv->nrp == c.gd.nrp && sv->kernels == c.fp64_kernel,
                GWL_EINVAL, "the context's options changed since the saved forward");
      qp_states = sv->qp.data();
      n_qp = (int)sv->qp.size();
      n_begin = sv->n_begin;
      n_end = sv->n_end;
      omega_ev = sv->omega.data();
      n_omega = (int)sv->omega.size();
      eta_ev = sv->eta_ev;
      n_lanczos = sv->L;
    }
    GWL_CHECK(0 <= n_begin && n_begin < n_end && n_end <= c.n_orb, GWL_EINVAL,
              "need 0 <= n_begin < n_end <= n_orb");
    GWL_CHECK(!c.tda && !c.quadrature && !c.isdf_on, GWL_EUNSUPPORTED,
              "the adjoint covers the polynomial method on the grid only (not Tamm-Dancoff, "
              "quadrature or ISDF)");
    GWL_CHECK(n_qp >= 1 && n_omega >= 1, GWL_EINVAL, "need n_qp >= 1 and n_omega >= 1");
    GWL_CHECK(qp_states && omega_ev, GWL_EINVAL, "null pointer");
    GWL_CHECK(fwd_only ? sigma_out != nullptr
                       : (grad_sigma && grad_energies && grad_orbitals),
              GWL_EINVAL, "null pointer");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    GWL_CHECK(n_lanczos >= 1 && n_lanczos <= 1024, GWL_EINVAL,
              "n_lanczos must be in [1, 1024] for the adjoint");
    GWL_CHECK(finite_all(omega_ev, n_omega), GWL_EINVAL, "non-finite frequency");
    GWL_CHECK(fwd_only || finite_all(grad_sigma, (size_t)n_qp * n_omega * 2), GWL_EINVAL,
              "non-finite cotangent");
    for (int i = 0; i < n_qp; ++i)
      GWL_CHECK(qp_states[i] >= 0 && qp_states[i] < c.n_orb, GWL_EINVAL, "qp state out of range");
    const long nvc = c.nvc;
    const int g = c.poly_degree;
    const int L = n_lanczos;
    const int nn = n_end - n_begin;
    const int P = n_qp * nn;
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
    const int nblk = (P + B - 1) / B;
    c.ensure_work(B, L, false);
    const int S = c.auto_splitk(B, GWL_FP64);
    // (the recompute must repeat the forward's arithmetic exactly)
    GWL_CHECK(!bwd_only || (B == sv->B && S == sv->S), GWL_EINVAL,
              "the context's options changed since the saved forward");
    PairGeom pg = c.pair_geom();
    const GemmDims& d = c.kd();
    const double lo = c.poly_lo, hi = c.poly_hi;
    const size_t vec = (size_t)B * nvc;
    const size_t fld = (size_t)B * d.nrp;             // B potentials on the padded grid
    const size_t uvp = (size_t)B * d.nvp * d.ncp;     // B padded pair vectors
    const int nct = d.ncp / 64;

    // pair list (m, n), qp index per pair
    std::vector<int> m(P), n(P), q(P);
    for (int a = 0; a < n_qp; ++a)
      for (int j = 0; j < nn; ++j) {
        const int p = a * nn + j;
        m[p] = qp_states[a];
        n[p] = n_begin + j;
        q[p] = a;
      }
    std::vector<double> en(P), et(P), om(n_omega);
    for (int p = 0; p < P; ++p) {
      en[p] = c.eps_ha[n[p]];
      et[p] = n[p] < c.nv ? 1.0 : -1.0;
    }
    for (int i = 0; i < n_omega; ++i) om[i] = omega_ev[i] / kHartreeEv;

    // ---- segment store: per step t_0..t_g, K~t_0..K~t_{g-1}, w_k, V[t_0..t_{g-1}]
    const size_t per_step = (size_t)(2 * g + 2) * vec + (size_t)g * fld;
    int seg = std::max(1, (int)std::ceil(std::sqrt((double)L)));
    DevBuf<double> store;
    bool whole = false;
    if (!persist && c.adjoint_store && seg < L &&
        ((size_t)L * per_step + 2 * vec) * sizeof(double) <= GWL_ADJOINT_STORE_MAX) {
      try {
        store.ensure((size_t)L * per_step + 2 * vec);
        whole = true;
        seg = L;
      } catch (const Error& e) {
        // not enough free device memory: recompute from checkpoints instead
        if (e.code != GWL_ENOMEM) throw;
        (void)hipGetLastError();
      }
    }
    if (seg >= L) whole = !persist, seg = L;
    if (!store.p && !fwd_only) store.ensure((size_t)seg * per_step + 2 * vec);
    c.adjoint_stored = whole ? 1 : 0;
    const int nseg = (L + seg - 1) / seg;
    // Full: the forward of a block ends by keeping its last segment's
    // iterates, so only the earlier segments need checkpoints and a recompute
    const int nck = persist ? nseg : nseg - 1;  // checkpoints per block
    // q after the segment's last step, q_{k0-1} of the segment (no store in a
    // forward-only call)
    double* const sq_end = store.p ? store.p + (size_t)seg * per_step : nullptr;
    double* const sq_prev0 = store.p ? sq_end + vec : nullptr;
    auto step_ptr = [&](int kk) { return store.p + (size_t)kk * per_step; };

    // buffers
    // kept state: in a new VjpSaved (Forward), the saved one (Backward), or a
    // local one for one block at a time (Full)
    std::shared_ptr<VjpSaved> own;
    if (!bwd_only) {
      own = std::make_shared<VjpSaved>();
      sv = own;
      const int nb_keep = persist ? nblk : 1;
      sv->Pb.ensure((size_t)nb_keep * vec);
      sv->Vnm.ensure((size_t)nb_keep * fld);
      if (nck > 0) {
        sv->ckq.ensure((size_t)nb_keep * nck * vec);
        sv->ckqp.ensure((size_t)nb_keep * nck * vec);
        sv->ck_state.ensure((size_t)nb_keep * nck * 2 * B);
        sv->ck_amax.ensure((size_t)nb_keep * nck * B);
        sv->ck_bprev.ensure((size_t)nb_keep * nck * B);
      }
      sv->flen.ensure(P);
      if (persist) {
        sv->coef_a.ensure((size_t)P * L);
        sv->coef_b.ensure((size_t)P * L);
        sv->norm2.ensure(P);
        sv->out_len.ensure(P);
      }
    }
    // block bi's slot in the kept state
    auto kb = [&](int bi) { return persist ? (size_t)bi : (size_t)0; };
    DevBuf<double> Sv, KS, VS, US, UT, wbar, qb0, qb1, qb2, pend, dbar, dbar_tot, kbar, abar,
        bbar, nbar, ebar, sig, Gd, e_d, eta_d, om_d, grad_int, gvpart;
    DevBuf<int> qidx_d, slot_pair, mrow_d, nrow_d;
    DevBuf<unsigned char> tscr;
    if (!fwd_only) {
      Sv.ensure((size_t)(g + 1) * vec);
      KS.ensure((size_t)(g + 1) * vec);
      VS.ensure((size_t)g * fld);
      US.ensure((size_t)g * uvp);
      UT.ensure((size_t)g * uvp);
      wbar.ensure(vec);
      qb0.ensure(vec);
      qb1.ensure(vec);
      qb2.ensure(vec);
      pend.ensure(B);
      dbar.ensure(vec);
      dbar_tot.ensure(nvc);
      kbar.ensure(vec);
      grad_int.ensure((size_t)(d.nvp + d.ncp) * d.nrp);
      gvpart.ensure((size_t)nct * c.nv * d.nrp);
    }
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
    slot_pair.ensure(B);
    mrow_d.ensure(P);
    nrow_d.ensure(P);
    tscr.ensure((size_t)B * L * n_omega * 16);
    std::vector<int> mr(P), nr_(P);
    for (int p = 0; p < P; ++p) {
      mr[p] = c.orb_row(m[p]);
      nr_[p] = c.orb_row(n[p]);
    }
    // (the forward-only call runs the continued-fraction adjoint for Sigma alone,
    // with a zero cotangent)
    if (!fwd_only)
      GWL_HIP(hipMemcpy(Gd.p, grad_sigma, sizeof(double) * n_qp * n_omega * 2,
                        hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(e_d.p, en.data(), sizeof(double) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(eta_d.p, et.data(), sizeof(double) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(om_d.p, om.data(), sizeof(double) * n_omega, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(qidx_d.p, q.data(), sizeof(int) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(mrow_d.p, mr.data(), sizeof(int) * P, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(nrow_d.p, nr_.data(), sizeof(int) * P, hipMemcpyHostToDevice));

    double *coef_a, *coef_b, *norm2;
    int* out_len;
    if (persist) {
      coef_a = sv->coef_a.p;
      coef_b = sv->coef_b.p;
      norm2 = sv->norm2.p;
      out_len = sv->out_len.p;
    } else {
      c.coef_a.ensure((size_t)P * L);
      c.coef_b.ensure((size_t)P * L);
      c.norm2.ensure(P);
      c.out_len.ensure(P);
      coef_a = c.coef_a.p;
      coef_b = c.coef_b.p;
      norm2 = c.norm2.p;
      out_len = c.out_len.p;
    }
    int* const flen = sv->flen.p;
    if (!bwd_only) {
      GWL_HIP(hipMemsetAsync(coef_a, 0, sizeof(double) * (size_t)P * L, st));
      GWL_HIP(hipMemsetAsync(coef_b, 0, sizeof(double) * (size_t)P * L, st));
    }
    SlotState ss;
    ss.pair = c.s_pair.p;
    ss.k = c.s_k.p;
    ss.len = c.s_len.p;
    ss.dead = c.s_dead.p;
    ss.amax = c.s_amax.p;
    ss.bprev = c.s_bprev.p;
    ss.coef_a = coef_a;
    ss.coef_b = coef_b;
    ss.out_len = out_len;
    ss.norm2 = norm2;
    ss.ld = L;

    // one Lanczos step (no reorthogonalisation) of all slots from q, qprev
    auto fwd_step = [&]() {
      c.apply_d_batch(B, c.q.p, c.w.p, GWL_FP64, false);
      lz_alpha(ss, B, c.q.p, c.qprev.p, c.w.p, nvc, st);
      lz_beta(ss, B, c.q.p, c.qprev.p, c.w.p, nullptr, 0, 0, nvc, st);
    };
    // w = p_g(C) t_0 for the vectors t_0 = Ti[0], keeping the iterates
    // t_1..t_g in Ti[1..g], K~t_j = K Delta^1/2 t_j in KTi[0..g-1] and the
    // potentials V[rho(Delta^1/2 t_j)] in VTi[j] (the same launches as
    // Context::apply_d_batch, plus those two outputs)
    auto cheb_iterates = [&](double* Ti, double* KTi, double* w, double* VTi) {
      c.cast(B, Ti, GWL_FP64);
      for (int j = 0; j < g; ++j) {
        c.k_product(B, GWL_FP64, S, VTi + (size_t)j * fld);
        combine<double, double>(pg, B, S, reinterpret_cast<const double*>(c.ypart.p),
                                Ti + (size_t)j * vec, j > 0 ? Ti + (size_t)(j - 1) * vec : nullptr,
                                Ti + (size_t)(j + 1) * vec, w, j == 0 ? 1 : 2, lo, hi,
                                c.cheb[0], c.cheb[j + 1], j + 1 < g ? c.u64.p : nullptr, st,
                                KTi + (size_t)j * vec);
      }
    };
    // steps k0..k1-1 from (qprev, q), keeping each step's iterates in the store
    auto fwd_segment_store = [&](int k0, int k1) {
      GWL_HIP(hipMemcpyAsync(sq_prev0, c.qprev.p, vec * 8, hipMemcpyDeviceToDevice, st));
      for (int k = k0; k < k1; ++k) {
        double* Ti = step_ptr(k - k0);
        double* KTi = Ti + (size_t)(g + 1) * vec;
        double* Wi = Ti + (size_t)(2 * g + 1) * vec;
        double* VTi = Ti + (size_t)(2 * g + 2) * vec;
        GWL_HIP(hipMemcpyAsync(Ti, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
        cheb_iterates(Ti, KTi, Wi, VTi);
        GWL_HIP(hipMemcpyAsync(c.w.p, Wi, vec * 8, hipMemcpyDeviceToDevice, st));
        lz_alpha(ss, B, c.q.p, c.qprev.p, c.w.p, nvc, st);
        lz_beta(ss, B, c.q.p, c.qprev.p, c.w.p, nullptr, 0, 0, nvc, st);
      }
      GWL_HIP(hipMemcpyAsync(sq_end, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
    };
    // checkpoint sgi of block bi: (q, q_prev) and the slot state
    auto save_state = [&](int bi, int sgi) {
      const size_t i = kb(bi) * nck + sgi;
      GWL_HIP(hipMemcpyAsync(sv->ckq.p + i * vec, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(sv->ckqp.p + i * vec, c.qprev.p, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(sv->ck_state.p + i * 2 * B, c.s_k.p, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(sv->ck_state.p + i * 2 * B + B, c.s_dead.p, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(sv->ck_amax.p + i * B, c.s_amax.p, B * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(sv->ck_bprev.p + i * B, c.s_bprev.p, B * 8, hipMemcpyDeviceToDevice, st));
    };
    auto load_state = [&](int bi, int sgi) {
      const size_t i = kb(bi) * nck + sgi;
      GWL_HIP(hipMemcpyAsync(c.q.p, sv->ckq.p + i * vec, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.qprev.p, sv->ckqp.p + i * vec, vec * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_k.p, sv->ck_state.p + i * 2 * B, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_dead.p, sv->ck_state.p + i * 2 * B + B, B * 4, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_amax.p, sv->ck_amax.p + i * B, B * 8, hipMemcpyDeviceToDevice, st));
      GWL_HIP(hipMemcpyAsync(c.s_bprev.p, sv->ck_bprev.p + i * B, B * 8, hipMemcpyDeviceToDevice, st));
    };
    const double* psi_c_rc = c.psi_c_rc64.p;
    const double* psi_v_rv = c.psi_v_rv64.p;
    double* grad_c = grad_int.p + (size_t)d.nvp * d.nrp;

    for (int p0 = 0; p0 < P; p0 += B) {
      const int nbk = std::min(B, P - p0);
      const int bi = p0 / B;
      double* const Pb = sv->Pb.p + kb(bi) * vec;
      double* const Vnm = sv->Vnm.p + kb(bi) * fld;
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
      if (!bwd_only) {
        // ---- forward
        GWL_HIP(hipMemsetAsync(c.q.p, 0, vec * 8, st));
        c.coupling_batch(nbk, m.data() + p0, n.data() + p0, c.q.p, nvc);
        // the coupling build leaves V[phi_n phi_m] of the block in vpot64
        GWL_HIP(hipMemcpyAsync(Vnm, c.vpot64.p, (size_t)nbk * d.nrp * 8, hipMemcpyDeviceToDevice, st));
        GWL_HIP(hipMemcpyAsync(Pb, c.q.p, vec * 8, hipMemcpyDeviceToDevice, st));
        lz_start(ss, B, c.s_slots.p, nbk, c.q.p, c.qprev.p, nullptr, 0, nvc, st);
        for (int k = 0; k < L; ++k) {
          if (k % seg == 0) {
            const int sgi = k / seg;
            if (!persist && sgi == nseg - 1) {  // the last segment: kept, not recomputed
              fwd_segment_store(k, L);
              break;
            }
            save_state(bi, sgi);
          }
          fwd_step();
        }
        // final lengths (the segment recompute below rewrites out_len step by step)
        GWL_HIP(hipMemcpyAsync(flen + p0, out_len + p0, nbk * 4, hipMemcpyDeviceToDevice, st));
      }
      // ---- continued-fraction adjoint (and the forward Sigma per pair)
      adj_cfrac(nbk, coef_a + (size_t)p0 * L, coef_b + (size_t)p0 * L, flen + p0, norm2 + p0, L,
                e_d.p + p0, eta_d.p + p0, qidx_d.p + p0, om_d.p, n_omega, eta_ev / kHartreeEv,
                Gd.p, tscr.p, abar.p + (size_t)p0 * L, bbar.p + (size_t)p0 * L, nbar.p + p0,
                ebar.p + p0, sig.p + (size_t)p0 * n_omega * 2, st);
      if (fwd_only) continue;
      // ---- backward
      double* qbn = qb0.p;  // q_bar_{k+1}
      double* qbc = qb1.p;  // q_bar_k
      double* qbp = qb2.p;  // q_bar_{k-1}
      GWL_HIP(hipMemsetAsync(qbn, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(qbc, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(qbp, 0, vec * 8, st));
      GWL_HIP(hipMemsetAsync(pend.p, 0, B * 8, st));
      GWL_HIP(hipMemsetAsync(dbar.p, 0, vec * 8, st));
      // backward step k from q_{k+1}, q_k, q_{k-1} and the kept iterates of p_g(C) q_k
      auto reverse_step = [&](int k, const double* qn, const double* qk, const double* qpv,
                              const double* Ti, const double* KTi, const double* Wi,
                              const double* VTi) {
        // reverse Lanczos step k
        adj_lanczos_step(k, B, slot_pair.p, flen, L, coef_a, coef_b, abar.p,
                         bbar.p, qn, qk, qpv, Wi, qbn, qbc, qbp, wbar.p, pend.p, nvc, st);
        // reverse Chebyshev recurrence on x = w_bar_k; the product on s_j leaves
        // V[rho(Delta^1/2 s_j)] in VS[j - 1]
        adj_scale_copy(Sv.p + (size_t)g * vec, wbar.p, c.cheb[g], (long)vec, st);
        c.cast(B, Sv.p + (size_t)g * vec, GWL_FP64);
        for (int j = g; j >= 1; --j) {
          c.k_product(B, GWL_FP64, S, VS.p + (size_t)(j - 1) * fld);
          adj_combine(pg, B, S, reinterpret_cast<const double*>(c.ypart.p),
                      Sv.p + (size_t)j * vec, j < g ? Sv.p + (size_t)(j + 1) * vec : nullptr,
                      wbar.p, c.cheb[j - 1], j >= 2 ? 2.0 : 1.0, lo, hi,
                      Sv.p + (size_t)(j - 1) * vec, KS.p + (size_t)j * vec,
                      j - 1 >= 1 ? c.u64.p : nullptr, st);
        }
        // C_bar = (2/(hi-lo)) [sum_{j>=2} 2 s_j t_{j-1}^T + s_1 t_0^T]: its Delta part
        // now, its coupling part as the pair-vector operands of the contraction
        for (int j = 1; j <= g; ++j) {
          const double alpha = (2.0 / (hi - lo)) * (j >= 2 ? 2.0 : 1.0);
          adj_dbar_zops(pg, B, Sv.p + (size_t)j * vec, KS.p + (size_t)j * vec,
                        Ti + (size_t)(j - 1) * vec, KTi + (size_t)(j - 1) * vec, alpha,
                        2.0 * alpha, dbar.p, US.p + (size_t)(j - 1) * uvp,
                        UT.p + (size_t)(j - 1) * uvp, st);
        }
        // orbital gradient of this step's coupling part
        adj_zgemm(d, c.nv, ZSeg{VTi, US.p, g * B}, ZSeg{VS.p, UT.p, g * B}, psi_c_rc, psi_v_rv,
                  c.dv, grad_c, gvpart.p, st);
        // q_bar_k += D w_bar_k
        adj_axpy(qbc, Sv.p, 1.0, (long)vec, st);
        // rotate: q_bar_{k+1} <- q_bar_k <- q_bar_{k-1} <- 0
        double* t = qbn;
        qbn = qbc;
        qbc = qbp;
        qbp = t;
        GWL_HIP(hipMemsetAsync(qbp, 0, vec * 8, st));
      };
      for (int sgi = nseg - 1; sgi >= 0; --sgi) {
        const int k0 = sgi * seg, k1 = std::min(L, k0 + seg);
        if (persist || sgi < nseg - 1) {
          load_state(bi, sgi);
          fwd_segment_store(k0, k1);
        }
        for (int k = k1 - 1; k >= k0; --k) {
          const double* Ti = step_ptr(k - k0);
          const double* qn = k + 1 < k1 ? step_ptr(k + 1 - k0) : sq_end;
          const double* qpv = k > k0 ? step_ptr(k - 1 - k0) : sq_prev0;
          reverse_step(k, qn, Ti, qpv, Ti, Ti + (size_t)(g + 1) * vec,
                       Ti + (size_t)(2 * g + 1) * vec, Ti + (size_t)(2 * g + 2) * vec);
        }
      }
      // start vector adjoint: q_bar_0 is now in qbn; k_bar per slot
      adj_start(B, slot_pair.p, norm2, nbar.p, Pb, qbn, c.sdelta.p, dbar.p, kbar.p, nvc, st);
      adj_sum_rows(dbar_tot.p, dbar.p, B, nvc, st);
      // orbital terms of the coupling integrals (nm|vc) = dV sum_r rho_vc V[phi_n phi_m]:
      // k_bar with V[phi_n phi_m] through the contraction, and the potential of
      // rho(k_bar) with phi_m (for phi_n) and phi_n (for phi_m)
      c.cast(B, kbar.p, GWL_FP64, true);
      adj_zgemm(d, c.nv, ZSeg{Vnm, c.u64.p, nbk}, ZSeg{nullptr, nullptr, 0}, psi_c_rc,
                psi_v_rv, c.dv, grad_c, gvpart.p, st);
      c.potential64(nbk, c.vpot64.p);
      adj_orb_grad_nm(c.psi_t.p, c.vpot64.p, d.nrp, (int)c.nr, mrow_d.p + p0, nrow_d.p + p0, nbk,
                      c.dv, grad_int.p, st);
    }
    if (fwd_only) {
      c.sig_sum.ensure((size_t)n_qp * n_omega * 2);
      sum_groups(sig.p, n_qp, nn, n_omega, c.sig_sum.p, st);
      GWL_HIP(hipMemcpyAsync(sigma_out, c.sig_sum.p, sizeof(double) * n_qp * n_omega * 2,
                             hipMemcpyDeviceToHost, st));
      GWL_HIP(hipStreamSynchronize(st));
      sv->qp.assign(qp_states, qp_states + n_qp);
      sv->omega.assign(omega_ev, omega_ev + n_omega);
      sv->n_begin = n_begin;
      sv->n_end = n_end;
      sv->L = L;
      sv->B = B;
      sv->S = S;
      sv->kernels = c.fp64_kernel;
      sv->g = g;
      sv->eta_ev = eta_ev;
      sv->lo = lo;
      sv->hi = hi;
      sv->nvc = nvc;
      sv->nrp = d.nrp;
      c.vjp_saved = sv;
      set_error("");
      return GWL_OK;
    }
    adj_gv_reduce(gvpart.p, nct, c.nv, d.nrp, grad_int.p, st);

    // ---- energies: Delta_bar -> e_bar, plus the explicit z_n terms
    std::vector<double> dtot(nvc), eb(P);
    GWL_HIP(hipStreamSynchronize(st));
    GWL_HIP(hipMemcpy(dtot.data(), dbar_tot.p, nvc * 8, hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(eb.data(), ebar.p, P * 8, hipMemcpyDeviceToHost));
    std::vector<double> ge(c.n_orb, 0.0);
    for (int v = 0; v < c.nv; ++v)
      for (int cc = 0; cc < c.nc; ++cc) {
        const double dd = dtot[(size_t)v * c.nc + cc];
        ge[v] -= dd;
        ge[c.nv + cc] += dd;
      }
    for (int p = 0; p < P; ++p) ge[n[p]] += eb[p];
    for (int a = 0; a < c.n_orb; ++a) grad_energies[a] = ge[a] / kHartreeEv;

    // ---- orbitals, in the orbitals' own type
    adj_gather_orbitals(grad_int.p, d.nrp, (int)c.nr, c.nv, d.nvp, c.n_orb, grad_orbitals,
                        c.orb_dtype == 4, st);

    if (sigma_out) {
      c.sig_sum.ensure((size_t)n_qp * n_omega * 2);
      sum_groups(sig.p, n_qp, nn, n_omega, c.sig_sum.p, st);
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

}  // namespace

extern "C" gwl_status gwl_sigma_c_vjp(gwl_ctx* ctx, const int* qp_states, int n_qp,
                                      const double* omega_ev, int n_omega, double eta_ev,
                                      int n_lanczos, const double* grad_sigma,
                                      double* sigma_out, double* grad_energies,
                                      void* grad_orbitals) {
  if (!ctx) {
    set_error("null context");
    return GWL_EINVAL;
  }
  return vjp_run(ctx, VjpMode::Full, qp_states, n_qp, 0, ctx->n_orb, omega_ev, n_omega, eta_ev,
                 n_lanczos,
                   grad_sigma, sigma_out, grad_energies, grad_orbitals);
}

extern "C" gwl_status gwl_sigma_c_range_vjp(gwl_ctx* ctx, const int* qp_states, int n_qp,
                                            int n_begin, int n_end, const double* omega_ev,
                                            int n_omega, double eta_ev, int n_lanczos,
                                            const double* grad_sigma, double* sigma_out,
                                            double* grad_energies, void* grad_orbitals) {
  return vjp_run(ctx, VjpMode::Full, qp_states, n_qp, n_begin, n_end, omega_ev, n_omega, eta_ev,
                 n_lanczos,
                   grad_sigma, sigma_out, grad_energies, grad_orbitals);
}

extern "C" gwl_status gwl_sigma_c_vjp_forward(gwl_ctx* ctx, const int* qp_states, int n_qp,
                                              int n_begin, int n_end, const double* omega_ev,
                                              int n_omega, double eta_ev, int n_lanczos,
                                              double* sigma_out) {
  if (ctx) ctx->vjp_saved.reset();  // the previous forward's state goes first
  return vjp_run(ctx, VjpMode::Forward, qp_states, n_qp, n_begin, n_end, omega_ev, n_omega,
                 eta_ev, n_lanczos, nullptr, sigma_out, nullptr, nullptr);
}

extern "C" gwl_status gwl_sigma_c_vjp_backward(gwl_ctx* ctx, const double* grad_sigma,
                                               double* grad_energies, void* grad_orbitals) {
  return vjp_run(ctx, VjpMode::Backward, nullptr, 0, 0, 0, nullptr, 0, 0.0, 0, grad_sigma,
                 nullptr, grad_energies, grad_orbitals);
}
