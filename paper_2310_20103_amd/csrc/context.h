// Context of the Lanczos GW self-energy library: device buffers, options,
// the batched Lanczos scheduler and the product drivers.  Shared by the
// C-ABI entry points (gwl.hip) and the vector-Jacobian product (vjp.hip).
#pragma once
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace gwl {


template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // (Re)allocate to at least cnt elements, zero-filled.  Contents are not kept.
  void ensure(size_t cnt) {
    if (cnt <= n) return;
    release();
    if (cnt == 0) return;
    hipError_t e = hipMalloc((void**)&p, cnt * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{GWL_ENOMEM, "hipMalloc of " + std::to_string(cnt * sizeof(T)) +
                                  " bytes failed: " + hipGetErrorString(e)};
    }
    n = cnt;
    GWL_HIP(hipMemset(p, 0, cnt * sizeof(T)));
    GWL_HIP(hipDeviceSynchronize());
  }
};

// Chebyshev interpolation coefficients of sqrt on [lo, hi] at the g+1
// first-kind Chebyshev points: c_j = (2 - [j=0])/(g+1) sum_k sqrt(x_k) cos(j th_k).
inline std::vector<double> cheb_sqrt(double lo, double hi, int g) {
  std::vector<double> c(g + 1, 0.0);
  for (int j = 0; j <= g; ++j) {
    double s = 0.0;
    for (int k = 0; k <= g; ++k) {
      const double th = kPi * (k + 0.5) / (g + 1);
      const double x = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos(th);
      s += std::sqrt(x) * std::cos(j * th);
    }
    c[j] = 2.0 * s / (g + 1);
  }
  c[0] *= 0.5;
  return c;
}

// Eigenvalues/vectors of a small symmetric matrix by cyclic Jacobi rotations.
inline void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& vec) {
  vec.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) vec[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - s * akq;
          a[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - s * aqk;
          a[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = vec[(size_t)k * n + p], vkq = vec[(size_t)k * n + q];
          vec[(size_t)k * n + p] = c * vkp - s * vkq;
          vec[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

inline bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace gwl

using namespace gwl;


struct gwl_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  int nx = 0, ny = 0, nz = 0;
  double lx = 0, ly = 0, lz = 0;
  long nr = 0;
  int n_orb = 0, nv = 0, nc = 0;
  long nvc = 0;
  GemmDims gd{};
  double dv = 0;

  int precision = GWL_FP64;
  int poly_degree = 7;
  double poly_lo = 0, poly_hi = 0;
  int reorth = GWL_REORTH_FULL;
  int block = 0;
  double kernel_scale = 1.0;
  int splitk = 0;  // 0 = automatic
  int fp64_kernel = 1;  // 0 = plain FMA tiles, 1 = MFMA (both precisions)
  int bf16_tile = 256;  // block tile width of the second 16-bit MFMA GEMM
  bool tile_fixed = false;  // set by the caller: the autotuner keeps it
  int tda = 0;          // 1: Tamm-Dancoff (Lanczos on A = Delta + K from (nm|vc))
  int quadrature = 0;   // 1: Lanczos on C + Gauss quadrature (no polynomial)
  int adjoint_store = 0;     // 1: the adjoint keeps the forward's iterates when they fit
  int orb_dtype = 8;         // 8 = FP64 orbitals were given, 4 = FP32
  int adjoint_stored = -1;   // what the last adjoint call did (-1: no call yet)
  std::shared_ptr<void> vjp_saved;  // state of the last gwl_sigma_c_vjp_forward
  bool poly_hi_auto = false;  // the interval's upper end is estimated (re-done for ISDF)
  double hi_resid = 0.0;      // residual bound of the last estimate's largest Ritz value
  DevBuf<int> ivbad;          // per-run flags of the interval check

  // ISDF of the pair densities: the K product runs on N_mu interpolation
  // points with the Coulomb matrix M / dV in place of the FFT Poisson solve
  int isdf_on = 0, isdf_ready = 0, n_mu = 0;
  GemmDims gdi{};                     // dims with the grid replaced by the points
  DevBuf<double> ipsi_t, ipsi_c_rc64, ipsi_v_rv64, mmat64;  // mmat: [NRp_i][NRp_i]
  DevBuf<f16_t> ipsi_t16;
  DevBuf<f16_t> ipsi_c_rc16, ipsi_v_rv16;
  DevBuf<float> ipsi_v_rv32, mmat32;
  DevBuf<int> ipoints;
  void* blas = nullptr;               // rocblas_handle, created with the ISDF setup
  const GemmDims& kd() const { return isdf_on ? gdi : gd; }
  void set_isdf(int on);
  DevBuf<double> qd, qe, qz;  // quadrature scratch [P][L]
  DevBuf<int> qstat;          // [P]
  bool lanczos_on_c() const { return quadrature && !tda; }
  // FP16 first GEMM of the mixed path: the orbital operands carry orb16_scale
  // and the pair-vector operand u_scale (powers of two chosen from bounds so
  // that no element exceeds 2^14); the combine undoes both
  double orb16_scale = 1.0, u_scale = 1.0, sd_max = 1.0;
  // u_scale for vectors of 2-norm <= norm: |u_i| <= max(Delta^1/2, 1) * norm,
  // and the Chebyshev iterates stay within the same bound
  void set_u_bound(double norm) {
    const double bound = std::max(sd_max, 1.0) * std::max(norm, 1e-300);
    int e = (int)std::floor(std::log2(16384.0 / bound));
    e = std::max(-60, std::min(60, e));
    u_scale = std::ldexp(1.0, e);
  }
  std::vector<double> cheb;
  std::vector<double> eps_ha;

  // operands
  DevBuf<double> psi_t;       // [NVp + NCp][NRp]
  DevBuf<double> psi_c_rc64;  // [NRp][NCp]
  DevBuf<double> psi_v_rv64;  // [NRp][NVp]
  DevBuf<f16_t> psi_t16;      // [NVp + NCp] rows or K panels (orb16_index), FP16, scaled
  int pv16_exp = 0;           // frexp exponent of max |phi_v| in psi_t16
  DevBuf<unsigned> xmax32;    // mixed Poisson solve: bound scratch per field pair
  DevBuf<int> vexp32;         // [cap] scale exponent of each mixed potential
  DevBuf<f16_t> psi_c_rc16;   // [NRp][NCp] FP16, scaled by orb16_scale
  DevBuf<float> psi_v_rv32;   // [NRp][NVp] FP32, scaled (other mixed epilogues)
  DevBuf<f16_t> psi_v_rv16;   // [NRp][NVp] FP16, scaled (MFMA epilogue, N_vp <= 128)
  DevBuf<double> delta1, delta2, sdelta;

  // FFT tables
  DevBuf<cplx<double>> tw64[3];
  DevBuf<cplx<float>> tw32[3];
  DevBuf<double> g2_64[3];
  DevBuf<float> g2_32[3];
  PoissonGeom<double> pg64{};
  PoissonGeom<float> pg32{};

  // work buffers
  int cap = 0;      // slot capacity of the buffers below
  int cap_L = 0;    // basis rows per slot
  DevBuf<double> q, qprev, w, ta, tb;
  // Operand buffers are kept per precision: their zero pads (v >= N_v,
  // c >= N_c, r >= N_r) are written once at allocation and must never hold
  // the other precision's bytes.
  DevBuf<double> u64;          // [cap][NVp][NCp]
  DevBuf<f16_t> u16;           // [cap][NVp][NCp] FP16, scaled by u_scale
  DevBuf<unsigned char> rho;   // [nvt][cap][NRp] x 8 (fully written by the first GEMM)
  DevBuf<double> vpot64;       // [cap][NRp]
  DevBuf<float> vpot32;        // [cap][NRp]
  DevBuf<f16_t> vpot16;        // [cap][NRp] mixed product: scaled FP16 potentials
  DevBuf<unsigned char> fftx;  // [(cap+1)/2][N_r] x 16
  DevBuf<unsigned char> ypart; // [S][cap][NVp][NCp] x 8
  DevBuf<double> basis;        // [cap][cap_L][nvc]
  DevBuf<double> hbuf;         // [cap][cap_L + 1]
  DevBuf<double> rw_n0, rw_part;  // reorthogonalisation scratch [cap], [cap][part_len]
  DevBuf<int> rw_skip;            // [cap]
  DevBuf<int> s_pair, s_k, s_len, s_dead, s_slots, s_m, s_n, s_act;
  // while set, GEMM operand rows map to these slots (see PairGeom::rows)
  const int* cur_rows = nullptr;
  DevBuf<double> s_amax, s_bprev;
  // per-call pair data
  DevBuf<double> coef_a, coef_b, norm2;
  DevBuf<int> out_len;
  DevBuf<double> sig, sig_sum, e_n, eta_n, omega;

  // statistics of the last call
  double last_ms_total = 0;
  long last_c_matvecs = 0;

  // captured graph of one p_g(C) product over the Lanczos slots (q -> w)
  int use_graphs = 1;
  // 1: run_pairs uploads its whole refill schedule once and replays a graph
  // of the whole Lanczos step; 0: the host-driven loop (synchronous refills)
  int sched_tables = 1;
  hipGraphExec_t sgraph = nullptr;  // whole Lanczos step (product + alpha/reorth/beta)
  std::vector<unsigned char> sg_key;
  DevBuf<int> sched_tab;            // refill schedule of the current run_pairs call
  hipGraphExec_t dgraph = nullptr;
  int dg_nb = -1, dg_prec = -1, dg_S = -1, dg_kern = -1, dg_deg = -1;
  double dg_lo = 0, dg_hi = 0, dg_uscale = 0;
  long work_gen = 0, dg_gen = -1;

  // autotuned (block, split) per precision
  struct Tune {
    int B = 0, S = 0, tile = 0;
    double us_per_vec = 0;
  };
  Tune tuned[2];

  // optional per-launch timing with HIP events on the context stream
  int profile = 0;
  std::vector<hipEvent_t> ev_pool;
  struct ProfRec {
    int kind, e0, e1, nvec;
  };
  std::vector<ProfRec> prof_recs;
  double prof_ms[3] = {0, 0, 0};
  long prof_n[3] = {0, 0, 0}, prof_vec[3] = {0, 0, 0};

  void prof_reset() {
    prof_recs.clear();
    for (int i = 0; i < 3; ++i) prof_ms[i] = 0, prof_n[i] = 0, prof_vec[i] = 0;
  }
  int prof_event() {
    const int idx = (int)prof_recs.size() * 2;
    while ((int)ev_pool.size() <= idx) {
      hipEvent_t e;
      GWL_HIP(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return idx;
  }
  int prof_open = -1;
  void prof_begin() {
    if (!profile) return;
    const int e = prof_event();
    GWL_HIP(hipEventRecord(ev_pool[e], stream));
    prof_open = e;
  }
  void prof_end(int kind, int nvec) {
    if (!profile) return;
    const int e0 = prof_open;
    prof_open = -1;
    const int e1 = (int)prof_recs.size() * 2 + 1;
    while ((int)ev_pool.size() <= e1) {
      hipEvent_t e;
      GWL_HIP(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    GWL_HIP(hipEventRecord(ev_pool[e1], stream));
    prof_recs.push_back({kind, e0, e1, nvec});
  }
  // Accumulate recorded intervals; the stream must be idle.
  void prof_flush() {
    for (const auto& r : prof_recs) {
      float ms = 0.f;
      GWL_HIP(hipEventElapsedTime(&ms, ev_pool[r.e0], ev_pool[r.e1]));
      prof_ms[r.kind] += ms;
      prof_n[r.kind] += 1;
      prof_vec[r.kind] += r.nvec;
    }
    prof_recs.clear();
  }

  // a_op: geometry of the Tamm-Dancoff product / coupling vectors
  PairGeom pair_geom(bool a_op = false) const {
    PairGeom g;
    g.rows = cur_rows;
    g.tda = a_op ? 1 : 0;
    g.delta = delta1.p;
    g.nv = nv;
    g.nc = nc;
    g.nvp = gd.nvp;
    g.ncp = gd.ncp;
    g.nvc = nvc;
    g.delta2 = delta2.p;
    g.sdelta = sdelta.p;
    g.dv = dv;
    return g;
  }

  int nvt_max() const {
    return std::max(std::max(gemm1_f64_vtiles(gd), gemm1_f16s_vtiles(gd)),
                    std::max(gemm1_f64m_vtiles(gd), gemm1_f16_vtiles(gd)));
  }

  // Split of the grid sum in the second GEMM: enough blocks to give every
  // CU several (the kernels run one wave per SIMD), each block keeping a
  // K range of at least 2048 grid points.
  int auto_splitk(int nb, int prec) const {
    if (splitk > 0) return splitk;
    if (tuned[prec].B == nb && tuned[prec].S > 0) return tuned[prec].S;
    return heuristic_splitk(nb, prec);
  }
  int heuristic_splitk(int nb, int prec) const {
    const GemmDims& d = kd();
    long blocks;
    if (!fp64_kernel)
      blocks = (long)nb * (d.nvp / 64) * ceil_div(d.ncp, 64);
    else if (prec == GWL_FP64)
      blocks = gemm2_f64m_blocks(d, nb);
    else
      blocks = gemm2_f16_blocks(d, nb, bf16_tile);
    int s = 1;
    // fill the chip (about 1024 blocks) while each split keeps >= 512 grid points
    while (blocks * s < 1024 && s < 32 && (long)d.nrp / (s * 2) >= 512) s *= 2;
    return s;
  }

  void ensure_work(int nb, int Lrows, bool need_basis) {
    const long nvpc = (long)gd.nvp * gd.ncp;
    if (nb > cap) {
      ++work_gen;
      q.ensure((size_t)nb * nvc);
      qprev.ensure((size_t)nb * nvc);
      w.ensure((size_t)nb * nvc);
      ta.ensure((size_t)nb * nvc);
      tb.ensure((size_t)nb * nvc);
      u64.ensure((size_t)nb * nvpc);
      u16.ensure((size_t)alloc_rows_u(nb, gd.nvp) * gd.ncp);
      rho.ensure((size_t)nvt_max() * nb * gd.nrp * 8);
      vpot64.ensure((size_t)nb * gd.nrp);
      vpot32.ensure((size_t)alloc_rows_v(nb, gd.nvp) * gd.nrp);
      vpot16.ensure((size_t)alloc_rows_v(nb, gd.nvp) * gd.nrp);
      xmax32.ensure((size_t)alloc_rows_v(nb, gd.nvp));
      vexp32.ensure((size_t)alloc_rows_v(nb, gd.nvp));
      fftx.ensure((size_t)((nb + 1) / 2) * nr * 16);
      ypart.ensure((size_t)32 * nb * nvpc * 8);
      s_pair.ensure(nb);
      s_k.ensure(nb);
      s_len.ensure(nb);
      s_dead.ensure(nb);
      s_slots.ensure(nb);
      s_act.ensure(nb);
      s_m.ensure(nb);
      s_n.ensure(nb);
      s_amax.ensure(nb);
      s_bprev.ensure(nb);
      rw_n0.ensure(nb);
      rw_part.ensure((size_t)nb * reorth_part_len(nvc));
      rw_skip.ensure(nb);
      cap = nb;
    }
    if (Lrows + 1 > cap_L || nb * (size_t)(Lrows + 1) > hbuf.n) {
      hbuf.ensure((size_t)nb * (Lrows + 2));
      cap_L = std::max(cap_L, Lrows + 1);
    }
    if (need_basis) basis.ensure((size_t)nb * Lrows * nvc);
  }

  int orb_row(int n) const { return n < nv ? n : gd.nvp + (n - nv); }

  // ---------------------------------------------------------------- products
  // The middle step of the K product: FFT Poisson on the grid, or y = (M/dV) rho
  // on the ISDF points (rho partials of the first GEMM summed over v tiles).
  void middle_step(int nb, int prec, int nvt, const void* rho_in, void* v_out);

  // rho <- the first GEMM with its fused row-dot for nb vectors (u already
  // cast): partial densities [nvt][nb][N_rp] in the working precision (FP64,
  // or FP32 carrying the scales u_scale * orb16_scale^2); returns nvt.
  int first_gemm(int nb, int prec) {
    hipStream_t st = stream;
    const bool is = isdf_on;
    const GemmDims& d = kd();
    int nvt;
    prof_begin();
    if (prec == GWL_FP64) {
      const double* crc = is ? ipsi_c_rc64.p : psi_c_rc64.p;
      const double* vrv = is ? ipsi_v_rv64.p : psi_v_rv64.p;
      double* rp = reinterpret_cast<double*>(rho.p);
      if (fp64_kernel) {
        gemm1_f64m(d, nb, crc, vrv, u64.p, rp, st);
        nvt = gemm1_f64m_vtiles(d);
      } else {
        gemm1_f64(d, nb, crc, vrv, u64.p, rp, st);
        nvt = gemm1_f64_vtiles(d);
      }
    } else {
      const f16_t* crc = is ? ipsi_c_rc16.p : psi_c_rc16.p;
      const f16_t* vrv16 = is ? ipsi_v_rv16.p : psi_v_rv16.p;
      const float* vrv32 = is ? ipsi_v_rv32.p : psi_v_rv32.p;
      float* rp = reinterpret_cast<float*>(rho.p);
      if (fp64_kernel) {
        gemm1_f16(d, nb, crc, vrv32, vrv16, u16.p, rp, st);
        nvt = gemm1_f16_vtiles(d);
      } else {
        gemm1_f16s(d, nb, crc, vrv32, u16.p, rp, st);
        nvt = gemm1_f16s_vtiles(d);
      }
    }
    prof_end(0, nb);
    return nvt;
  }

  // ypart <- second GEMM of K applied to u (u already cast for nb vectors).
  // FP64: the Hartree potentials of the nb densities go to vout64 [nb][N_rp]
  // when given (kept by the adjoint), else to vpot64.
  void k_product(int nb, int prec, int S, double* vout64 = nullptr) {
    hipStream_t st = stream;
    const bool is = isdf_on;
    // On N_mu points the 16-bit operand rounding of the second GEMM averages
    // over far fewer terms than on the grid (an emulation gave a 2.5e-3
    // relative error in K x against 4.6e-4 on the grid), so ISDF is FP64 only.
    GWL_CHECK(!is || prec == GWL_FP64, GWL_EUNSUPPORTED, "the ISDF product runs in FP64 only");
    const GemmDims& d = kd();
    if (prec == GWL_FP64) {
      double* rp = reinterpret_cast<double*>(rho.p);
      double* vp = vout64 ? vout64 : vpot64.p;
      double* yp = reinterpret_cast<double*>(ypart.p);
      const double* pt = is ? ipsi_t.p : psi_t.p;
      const int nvt = first_gemm(nb, prec);
      prof_begin();
      if (is)
        middle_step(nb, prec, nvt, rp, vp);
      else
        poisson_launch<double>(pg64, rp, d.nrp, (long)nb * d.nrp, nvt, vp, d.nrp, nb,
                               reinterpret_cast<cplx<double>*>(fftx.p), st);
      prof_end(2, nb);
      const double* pv = pt;
      const double* pc = pt + (size_t)d.nvp * d.nrp;
      prof_begin();
      if (fp64_kernel)
        gemm2_f64m(d, nb, S, pv, pc, vp, yp, st);
      else
        gemm2_f64(d, nb, S, pv, pc, vp, yp, st);
      prof_end(1, nb);
    } else {
      float* rp = reinterpret_cast<float*>(rho.p);
      float* vp = vpot32.p;
      float* yp = reinterpret_cast<float*>(ypart.p);
      const f16_t* pt = is ? ipsi_t16.p : psi_t16.p;
      const int nvt = first_gemm(nb, prec);
      prof_begin();
      if (is)
        middle_step(nb, prec, nvt, rp, vp);
      else
        poisson_launch<float>(pg32, rp, d.nrp, (long)nb * d.nrp, nvt, vp, d.nrp, nb,
                              reinterpret_cast<cplx<float>*>(fftx.p), st, xmax32.p,
                              vexp32.p, pv16_exp, vpot16.p);
      prof_end(2, nb);
      const f16_t* pv = pt;
      const f16_t* pc = pt + orb16_index(d, d.nvp, 0);  // the conduction rows follow
      prof_begin();
      if (fp64_kernel)
        gemm2_f16(d, nb, bf16_tile, S, pv, pc, vpot16.p, yp, st);
      else
        gemm2_f16s(d, nb, S, pv, pc, vpot16.p, yp, st);
      prof_end(1, nb);
    }
  }

  // vout [nb][N_rp] <- Hartree potentials of the densities rho_b(r) =
  // sum_vc phi_v(r) phi_c(r) u_b[v][c] of the FP64 operands already in u64
  // (the first half of the K product, on the grid).
  void potential64(int nb, double* vout) {
    const GemmDims& d = gd;
    double* rp = reinterpret_cast<double*>(rho.p);
    int nvt;
    if (fp64_kernel) {
      gemm1_f64m(d, nb, psi_c_rc64.p, psi_v_rv64.p, u64.p, rp, stream);
      nvt = gemm1_f64m_vtiles(d);
    } else {
      gemm1_f64(d, nb, psi_c_rc64.p, psi_v_rv64.p, u64.p, rp, stream);
      nvt = gemm1_f64_vtiles(d);
    }
    poisson_launch<double>(pg64, rp, d.nrp, (long)nb * d.nrp, nvt, vout, d.nrp, nb,
                           reinterpret_cast<cplx<double>*>(fftx.p), stream);
  }

  void cast(int nb, const double* x, int prec, bool a_op = false) {
    PairGeom g = pair_geom(a_op);
    if (prec == GWL_FP64) {
      cast_u<double>(g, nb, x, nvc, u64.p, stream);
    } else {
      g.uscale = u_scale;
      cast_u<f16_t>(g, nb, x, nvc, u16.p, stream);
    }
  }

  void do_combine(int nb, int S, int prec, const double* x, const double* tp, double* out,
                  double* acc, int mode, double c0, double cj, bool write_u) {
    PairGeom g = pair_geom(mode == 3);
    if (prec == GWL_FP64)
      combine<double, double>(g, nb, S, reinterpret_cast<const double*>(ypart.p), x, tp, out,
                              acc, mode, poly_lo, poly_hi, c0, cj,
                              write_u ? u64.p : nullptr, stream);
    else {
      g.uscale = u_scale;
      // first GEMM: u and both orbital factors scaled; second GEMM: phi_v and
      // phi_c scaled again, and s_b per row (g.vmax)
      g.yscale = 1.0 / (u_scale * orb16_scale * orb16_scale * orb16_scale * orb16_scale);
      g.vexp = vexp32.p;
      combine<float, f16_t>(g, nb, S, reinterpret_cast<const float*>(ypart.p), x, tp, out,
                            acc, mode, poly_lo, poly_hi, c0, cj,
                            write_u ? u16.p : nullptr, stream);
    }
  }

  // out = A x = Delta x + K x (Tamm-Dancoff) for nb vectors; uses u, ypart.
  void apply_a_batch(int nb, const double* x, double* out, int prec) {
    const int S = auto_splitk(nb, prec);
    last_c_matvecs += nb;
    cast(nb, x, prec, true);
    k_product(nb, prec, S);
    do_combine(nb, S, prec, x, nullptr, out, nullptr, 3, 0, 0, false);
  }

  // out = C x for nb vectors (x, out device [nb][nvc]); uses u, ypart.
  void apply_c_batch(int nb, const double* x, double* out, int prec) {
    const int S = auto_splitk(nb, prec);
    last_c_matvecs += nb;
    cast(nb, x, prec);
    k_product(nb, prec, S);
    do_combine(nb, S, prec, x, nullptr, out, nullptr, 0, 0, 0, false);
  }

  // acc = p_g(C) x.  Expects u = cast(Delta^1/2 x) already in place when
  // u_ready, else casts.  x is not modified; uses ta, tb.
  void apply_d_batch(int nb, const double* x, double* acc, int prec, bool u_ready) {
    const int g = poly_degree;
    const int S = auto_splitk(nb, prec);
    if (!u_ready) cast(nb, x, prec);
    // t1 = C~ x, acc = c0 x + c1 t1
    k_product(nb, prec, S);
    double* t_prev = const_cast<double*>(x);
    double* t_cur = ta.p;
    do_combine(nb, S, prec, x, nullptr, t_cur, acc, 1, cheb[0], cheb[1], g >= 2);
    double* spare = tb.p;
    for (int j = 2; j <= g; ++j) {
      k_product(nb, prec, S);
      // t_j = 2 C~ t_{j-1} - t_{j-2}; written over t_{j-2} unless that is x
      double* out = (t_prev == x) ? spare : t_prev;
      do_combine(nb, S, prec, t_cur, t_prev, out, acc, 2, 0.0, cheb[j], j < g);
      t_prev = t_cur;
      t_cur = out;
    }
  }

  // Coupling vectors of cnt (m, n) pairs into rows dst (device [cnt][ldp]).
  void coupling_batch(int cnt, const int* m_host, const int* n_host, double* dst, long ldp) {
    ensure_work(cnt, 1, false);
    std::vector<int> mr(cnt), nrw(cnt);
    for (int i = 0; i < cnt; ++i) {
      mr[i] = orb_row(m_host[i]);
      nrw[i] = orb_row(n_host[i]);
    }
    GWL_HIP(hipStreamSynchronize(stream));
    GWL_HIP(hipMemcpy(s_m.p, mr.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(s_n.p, nrw.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
    coupling_rows(cnt, s_m.p, s_n.p, dst, ldp);
  }

  // Coupling vectors from orbital rows already on the device (mrow, nrow:
  // [cnt] rows of psi_t); queued on the stream, no host synchronisation.
  void coupling_rows(int cnt, const int* mrow, const int* nrow, double* dst, long ldp) {
    double* rp = reinterpret_cast<double*>(rho.p);
    double* vp = vpot64.p;
    double* yp = reinterpret_cast<double*>(ypart.p);
    pair_product(psi_t.p, gd.nrp, (int)nr, mrow, nrow, cnt, rp, stream);
    poisson_launch<double>(pg64, rp, gd.nrp, 0, 1, vp, gd.nrp, cnt,
                           reinterpret_cast<cplx<double>*>(fftx.p), stream);
    const int S = auto_splitk(cnt, GWL_FP64);
    const double* pv = psi_t.p;
    const double* pc = psi_t.p + (size_t)gd.nvp * gd.nrp;
    if (fp64_kernel)
      gemm2_f64m(gd, cnt, S, pv, pc, vp, yp, stream);
    else
      gemm2_f64(gd, cnt, S, pv, pc, vp, yp, stream);
    coupling_finish<double>(pair_geom(tda != 0), cnt, S, yp, dst, ldp, stream);
  }

  // w = p_g(C) q over nb slots; replays a captured graph of the whole product
  // (g x [first GEMM, five FFT passes, second GEMM, combine] + cast) when the
  // shapes and buffers are unchanged.
  void apply_d_step(int nb, int prec) {
    last_c_matvecs += (long)nb * poly_degree;
    const int S = auto_splitk(nb, prec);
    if (cur_rows) {  // a subset of the slots: launched eagerly
      apply_d_batch(nb, q.p, w.p, prec, false);
      return;
    }
    if (!use_graphs || profile || isdf_on) {  // (the ISDF product calls rocBLAS)
      apply_d_batch(nb, q.p, w.p, prec, false);
      return;
    }
    if (!dgraph || dg_nb != nb || dg_prec != prec || dg_S != S || dg_kern != fp64_kernel ||
        dg_gen != work_gen || dg_deg != poly_degree || dg_lo != poly_lo || dg_hi != poly_hi ||
        dg_uscale != u_scale) {
      drop_graph();
      hipGraph_t g = nullptr;
      GWL_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      try {
        apply_d_batch(nb, q.p, w.p, prec, false);
      } catch (...) {
        (void)hipStreamEndCapture(stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      GWL_HIP(hipStreamEndCapture(stream, &g));
      const hipError_t e = hipGraphInstantiate(&dgraph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        dgraph = nullptr;
        throw Error{GWL_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
      }
      dg_nb = nb;
      dg_prec = prec;
      dg_S = S;
      dg_kern = fp64_kernel;
      dg_gen = work_gen;
      dg_deg = poly_degree;
      dg_lo = poly_lo;
      dg_hi = poly_hi;
      dg_uscale = u_scale;
    }
    GWL_HIP(hipGraphLaunch(dgraph, stream));
  }

  void drop_graph() {
    if (dgraph) (void)hipGraphExecDestroy(dgraph);
    dgraph = nullptr;
    if (sgraph) (void)hipGraphExecDestroy(sgraph);
    sgraph = nullptr;
    sg_key.clear();
  }

  // ---------------------------------------------------------------- autotuner
  // Pick the number of Lanczos slots B and the split of the second GEMM by
  // timing one C-product per candidate with HIP events on the context
  // stream; the time per pair vector decides.  Results are kept per context
  // and, when GWL_TUNE_CACHE names a file, shared through it (one line per
  // problem shape: "key B S us_per_vector").
  std::string tune_key(int prec) const {
    return "gfx950:" + std::to_string(nr) + ":" + std::to_string(nv) + ":" +
           std::to_string(nc) + ":" + std::to_string(prec) + ":" + std::to_string(fp64_kernel) + ":" +
           std::to_string(tile_fixed ? bf16_tile : 0) + ":" + std::to_string(isdf_on ? n_mu : 0);
  }

  bool tune_cache_read(int prec, Tune& t) const {
    const char* path = std::getenv("GWL_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char key[256];
    int b = 0, sk = 0, tile = 0;
    double us = 0;
    bool found = false;
    const std::string want = tune_key(prec);
    while (std::fscanf(f, "%255s %d %d %d %lf", key, &b, &sk, &tile, &us) == 5)
      if (want == key && b > 0 && sk > 0 && (tile == 128 || tile == 256)) {
        t.B = b;
        t.S = sk;
        t.tile = tile;
        t.us_per_vec = us;
        found = true;
      }
    std::fclose(f);
    return found;
  }

  void tune_cache_write(int prec, const Tune& t) const {
    const char* path = std::getenv("GWL_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %.3f\n", tune_key(prec).c_str(), t.B, t.S, t.tile,
                 t.us_per_vec);
    std::fclose(f);
  }

  // The mixed product with the MFMA kernels also chooses the second GEMM's
  // block tile (256 or 128 wide) unless the caller fixed it.
  Tune autotune(int prec, int bmax) {
    Tune best = tuned[prec];
    if (best.B > 0) return best;
    const bool pick_tile = prec == GWL_MIXED_F16 && fp64_kernel && !tile_fixed;
    if (tune_cache_read(prec, best)) {
      if (pick_tile) set_tile(best.tile);
      best.tile = bf16_tile;
      tuned[prec] = best;
      return best;
    }
    const int cands[] = {32, 64, 128, 256};
    std::vector<int> tiles = {bf16_tile};
    if (pick_tile) tiles = {256, 128};
    hipEvent_t e0, e1;
    GWL_HIP(hipEventCreate(&e0));
    GWL_HIP(hipEventCreate(&e1));
    best.us_per_vec = 1e300;
    try {
      for (int tile : tiles) {
        bf16_tile = tile;
        for (int B : cands) {
          if (B > bmax && B != cands[0]) break;
          ensure_work(B, 1, false);
          const int s0 = heuristic_splitk(B, prec);
          for (int S : {s0 / 2, s0, s0 * 2}) {
            if (S < 1 || S > 32 || (S > 1 && (long)kd().nrp / S < 1024)) continue;
            cast(B, q.p, prec);
            k_product(B, prec, S);  // warm
            GWL_HIP(hipEventRecord(e0, stream));
            for (int r = 0; r < 2; ++r) k_product(B, prec, S);
            GWL_HIP(hipEventRecord(e1, stream));
            GWL_HIP(hipEventSynchronize(e1));
            float ms = 0;
            GWL_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / 2 / B;
            if (us < best.us_per_vec * 0.97) {
              best.B = B;
              best.S = S;
              best.tile = tile;
              best.us_per_vec = us;
            }
          }
        }
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.B <= 0) {  // nothing timed: fall back to the memory rule and heuristic split
      best.tile = tiles[0];
      bf16_tile = best.tile;
      best.B = std::max(1, std::min(bmax, 128));
      best.S = heuristic_splitk(best.B, prec);
      best.us_per_vec = 0;
    }
    set_tile(best.tile);
    tuned[prec] = best;
    tune_cache_write(prec, best);
    return best;
  }

  // second-GEMM block tile of the mixed product (a captured graph used the old one)
  void set_tile(int tile) {
    if (tile != 128 && tile != 256) return;
    if (bf16_tile != tile) drop_graph();
    bf16_tile = tile;
  }

  // ---------------------------------------------------------------- scheduler
  // Run Lanczos on p_g(C) (or on C itself when on_c) for P start vectors
  // (m_i, n_i) with lengths len_i.  Coefficients land in coef_a/coef_b
  // ([P][ld]), norm2 [P], out_len [P] on the device.
  void run_pairs(int P, const int* m_host, const int* n_host, const int* len_host, int ld,
                 bool on_c = false, const double* start_dev = nullptr) {
    if (sched_tables)
      run_pairs_tables(P, m_host, n_host, len_host, ld, on_c, start_dev);
    else
      run_pairs_host(P, m_host, n_host, len_host, ld, on_c, start_dev);
    if (!on_c && !tda) check_interval(P, ld);
  }

  // Slots B, buffers and the zeroed coefficient arrays of a run_pairs call.
  int prepare_pairs(int P, int ld, bool full) {
    const int prec = precision;
    set_u_bound(1.0);  // Lanczos vectors have unit norm
    int B;
    if (block > 0) {
      B = block;
    } else {
      const int bmem = auto_block(1 << 30, ld);  // memory cap on slots
      B = std::min(autotune(prec, bmem).B, bmem);
    }
    B = std::max(1, std::min(B, P));
    ensure_work(B, ld, full);
    coef_a.ensure((size_t)P * ld);
    coef_b.ensure((size_t)P * ld);
    norm2.ensure(P);
    out_len.ensure(P);
    GWL_HIP(hipMemsetAsync(coef_a.p, 0, sizeof(double) * (size_t)P * ld, stream));
    GWL_HIP(hipMemsetAsync(coef_b.p, 0, sizeof(double) * (size_t)P * ld, stream));
    return B;
  }

  SlotState slot_state(int ld) {
    SlotState ss;
    ss.pair = s_pair.p;
    ss.k = s_k.p;
    ss.len = s_len.p;
    ss.dead = s_dead.p;
    ss.amax = s_amax.p;
    ss.bprev = s_bprev.p;
    ss.coef_a = coef_a.p;
    ss.coef_b = coef_b.p;
    ss.out_len = out_len.p;
    ss.norm2 = norm2.p;
    ss.ld = ld;
    return ss;
  }

  // The product of one Lanczos step over nb slot rows (q -> w).
  void step_product(int nb, int prec, bool on_c, bool eager) {
    if (on_c)
      apply_c_batch(nb, q.p, w.p, prec);
    else if (tda)
      apply_a_batch(nb, q.p, w.p, prec);
    else if (eager) {
      last_c_matvecs += (long)nb * poly_degree;
      apply_d_batch(nb, q.p, w.p, prec, false);
    } else
      apply_d_step(nb, prec);
  }

  // One whole Lanczos step over all B slots -- the product, a_k, the
  // reorthogonalisation against every stored row a slot has (rows beyond a
  // slot's k return at once, so the launch shapes do not change from step
  // to step) and b_{k+1} -- replayed from a captured graph while the shapes
  // and buffers stay the same.
  void lanczos_step_graph(int B, int ld, bool on_c, const SlotState& ss, bool full) {
    const int prec = precision;
    const long bstride = (long)ld * nvc;
    auto body = [&]() {
      step_product(B, prec, on_c, true);
      lz_alpha(ss, B, q.p, qprev.p, w.p, nvc, stream);
      lz_reorth(ss, B, ld - 1, reorth, full ? basis.p : nullptr, bstride, q.p, qprev.p, w.p,
                hbuf.p, ReorthScratch{rw_n0.p, rw_part.p, rw_skip.p}, nvc, stream);
      lz_beta(ss, B, q.p, qprev.p, w.p, full ? basis.p : nullptr, bstride, full ? 1 : 0, nvc,
              stream);
    };
    const long cm = (long)B * (on_c || tda ? 1 : poly_degree);
    if (!use_graphs || profile || isdf_on) {
      body();  // (the ISDF product calls rocBLAS)
      return;
    }
    // everything the captured launches depend on
    struct Key {
      int B, ld, on_c, tda, prec, S, kern, deg, reorth, tile;
      long gen;
      double lo, hi, us;
      const void* p[8];
      SlotState ss;
    } key;
    std::memset(&key, 0, sizeof(key));
    key.B = B;
    key.ld = ld;
    key.on_c = on_c;
    key.tda = tda;
    key.prec = prec;
    key.S = auto_splitk(B, prec);
    key.kern = fp64_kernel;
    key.deg = poly_degree;
    key.reorth = reorth;
    key.tile = bf16_tile;
    key.gen = work_gen;
    key.lo = poly_lo;
    key.hi = poly_hi;
    key.us = u_scale;
    key.p[0] = basis.p;
    key.p[1] = hbuf.p;
    key.p[2] = rw_part.p;
    key.p[3] = coef_a.p;
    key.p[4] = coef_b.p;
    key.p[5] = norm2.p;
    key.p[6] = out_len.p;
    key.p[7] = vexp32.p;
    key.ss = ss;
    const unsigned char* kb = reinterpret_cast<const unsigned char*>(&key);
    std::vector<unsigned char> kv(kb, kb + sizeof(key));
    if (!sgraph || kv != sg_key) {
      if (sgraph) (void)hipGraphExecDestroy(sgraph);
      sgraph = nullptr;
      sg_key.clear();
      hipGraph_t g = nullptr;
      const long saved = last_c_matvecs;
      GWL_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      try {
        body();
      } catch (...) {
        (void)hipStreamEndCapture(stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      GWL_HIP(hipStreamEndCapture(stream, &g));
      last_c_matvecs = saved;
      const hipError_t e = hipGraphInstantiate(&sgraph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        sgraph = nullptr;
        throw Error{GWL_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
      }
      sg_key = kv;
    }
    GWL_HIP(hipGraphLaunch(sgraph, stream));
    last_c_matvecs += cm;
  }

  // Scheduler with the whole refill schedule on the device.  The order of
  // refills is fixed by the lengths (a slot runs its start vector for exactly
  // its length; a breakdown only freezes its coefficients), so the host
  // plays the schedule out first, uploads it once (per refill event: the
  // refilled slots, their orbital rows and the slot table after the event;
  // per change of the busy set: its slot list) and then only queues work:
  // no synchronisation or host-to-device copy inside the loop.  Steps with
  // neither a refill nor a change of the busy set replay one graph of the
  // whole step.
  void run_pairs_tables(int P, const int* m_host, const int* n_host, const int* len_host,
                        int ld, bool on_c, const double* start_dev) {
    const int prec = precision;
    const bool full = (reorth == GWL_REORTH_FULL);
    const int B = prepare_pairs(P, ld, full);
    const SlotState ss = slot_state(ld);
    const long bstride = (long)ld * nvc;
    // ---- play the schedule out on the host
    struct Ev {
      long step;
      int cnt;
      bool contiguous;
      long o_slots, o_m, o_n, o_pair, o_len;  // offsets into tab
    };
    struct Act {
      long step;
      int nact;
      long o_rows;  // -1: all B slots
    };
    std::vector<int> tab;
    std::vector<Ev> evs;
    std::vector<Act> acts;
    long nsteps = 0;
    {
      std::vector<int> order(P);
      for (int i = 0; i < P; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int b) { return len_host[a] > len_host[b]; });
      std::vector<int> hp(B, -1), hk(B, 0), hl(B, 0), act, prev_act;
      int next = 0;
      for (long step = 0;; ++step) {
        std::vector<int> slots, mr, nr_;
        for (int b = 0; b < B && next < P; ++b)
          if (hp[b] < 0 || hk[b] >= hl[b]) {
            const int pi = order[next++];
            hp[b] = pi;
            hk[b] = 0;
            hl[b] = len_host[pi];
            slots.push_back(b);
            mr.push_back(orb_row(m_host[pi]));
            nr_.push_back(orb_row(n_host[pi]));
          }
        if (!slots.empty()) {
          for (int b = 0; b < B; ++b)
            if (hp[b] >= 0 && hk[b] >= hl[b]) hp[b] = -1;
          Ev e;
          e.step = step;
          e.cnt = (int)slots.size();
          e.contiguous = true;
          for (int i = 0; i < e.cnt; ++i) e.contiguous &= (slots[i] == slots[0] + i);
          auto put = [&](const std::vector<int>& v) {
            const long o = (long)tab.size();
            tab.insert(tab.end(), v.begin(), v.end());
            return o;
          };
          e.o_slots = put(slots);
          e.o_m = put(mr);
          e.o_n = put(nr_);
          e.o_pair = put(hp);
          e.o_len = put(hl);
          evs.push_back(e);
        }
        act.clear();
        for (int b = 0; b < B; ++b)
          if (hp[b] >= 0 && hk[b] < hl[b]) act.push_back(b);
        if (act.empty()) {
          nsteps = step;
          break;
        }
        if (act != prev_act) {
          Act a;
          a.step = step;
          a.nact = (int)act.size();
          a.o_rows = -1;
          if (a.nact < B) {
            a.o_rows = (long)tab.size();
            tab.insert(tab.end(), act.begin(), act.end());
          }
          acts.push_back(a);
          prev_act = act;
        }
        for (int b = 0; b < B; ++b)
          if (hp[b] >= 0 && hk[b] < hl[b]) ++hk[b];
      }
    }
    // ---- upload it once
    sched_tab.ensure(std::max<size_t>(tab.size(), 1));
    GWL_HIP(hipMemcpyAsync(sched_tab.p, tab.data(), tab.size() * sizeof(int),
                           hipMemcpyHostToDevice, stream));
    GWL_HIP(hipStreamSynchronize(stream));  // tab may go once the copy is done
    const int* T = sched_tab.p;
    // ---- run
    size_t ie = 0, ia = 0;
    int nact = B;
    const int* rows = nullptr;
    for (long step = 0; step < nsteps; ++step) {
      if (ie < evs.size() && evs[ie].step == step) {
        const Ev& e = evs[ie++];
        GWL_HIP(hipMemcpyAsync(s_pair.p, T + e.o_pair, B * sizeof(int), hipMemcpyDeviceToDevice,
                               stream));
        GWL_HIP(hipMemcpyAsync(s_len.p, T + e.o_len, B * sizeof(int), hipMemcpyDeviceToDevice,
                               stream));
        std::vector<int> hs;  // host copy of the slot list, for the row copies below
        if (start_dev || !e.contiguous) hs.assign(tab.begin() + e.o_slots, tab.begin() + e.o_slots + e.cnt);
        if (start_dev) {
          const int* hpair = tab.data() + e.o_pair;
          for (int i = 0; i < e.cnt; ++i)
            GWL_HIP(hipMemcpyAsync(q.p + (size_t)hs[i] * nvc,
                                   start_dev + (size_t)hpair[hs[i]] * nvc, nvc * sizeof(double),
                                   hipMemcpyDeviceToDevice, stream));
        } else if (e.contiguous) {
          coupling_rows(e.cnt, T + e.o_m, T + e.o_n, q.p + (size_t)tab[e.o_slots] * nvc, nvc);
        } else {
          coupling_rows(e.cnt, T + e.o_m, T + e.o_n, w.p, nvc);
          for (int i = 0; i < e.cnt; ++i)
            GWL_HIP(hipMemcpyAsync(q.p + (size_t)hs[i] * nvc, w.p + (size_t)i * nvc,
                                   nvc * sizeof(double), hipMemcpyDeviceToDevice, stream));
        }
        lz_start(ss, B, T + e.o_slots, e.cnt, q.p, qprev.p, full ? basis.p : nullptr, bstride,
                 nvc, stream);
      }
      if (ia < acts.size() && acts[ia].step == step) {
        nact = acts[ia].nact;
        rows = acts[ia].o_rows >= 0 ? T + acts[ia].o_rows : nullptr;
        ++ia;
      }
      if (!rows) {
        lanczos_step_graph(B, ld, on_c, ss, full);
      } else {
        cur_rows = rows;
        try {
          step_product(nact, prec, on_c, true);
        } catch (...) {
          cur_rows = nullptr;
          throw;
        }
        cur_rows = nullptr;
        lz_alpha(ss, B, q.p, qprev.p, w.p, nvc, stream);
        lz_reorth(ss, B, ld - 1, reorth, full ? basis.p : nullptr, bstride, q.p, qprev.p, w.p,
                  hbuf.p, ReorthScratch{rw_n0.p, rw_part.p, rw_skip.p}, nvc, stream);
        lz_beta(ss, B, q.p, qprev.p, w.p, full ? basis.p : nullptr, bstride, full ? 1 : 0,
                nvc, stream);
      }
      if (profile && prof_recs.size() > 4096) {
        GWL_HIP(hipStreamSynchronize(stream));
        prof_flush();
      }
    }
    GWL_HIP(hipStreamSynchronize(stream));
    prof_flush();
  }

  // The host-driven scheduler: refills decided and uploaded step by step
  // (a host synchronisation and copies per refill); the product of a step is
  // a replayed graph, the vector kernels are launched eagerly.
  void run_pairs_host(int P, const int* m_host, const int* n_host, const int* len_host, int ld,
                      bool on_c, const double* start_dev) {
    const int prec = precision;
    const bool full = (reorth == GWL_REORTH_FULL);
    const int B = prepare_pairs(P, ld, full);
    const SlotState ss = slot_state(ld);
    const long bstride = (long)ld * nvc;
    std::vector<int> hp(B, -1), hk(B, 0), hl(B, 0);
    GWL_HIP(hipMemcpyAsync(s_pair.p, hp.data(), B * sizeof(int), hipMemcpyHostToDevice, stream));
    GWL_HIP(hipStreamSynchronize(stream));
    // longest runs first, so that the slots still busy when the queue
    // runs dry hold the shortest ones
    std::vector<int> order(P);
    for (int i = 0; i < P; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return len_host[a] > len_host[b]; });
    int next = 0;
    std::vector<int> slots, ms, ns, act, act_dev;
    while (true) {
      // refill
      slots.clear();
      ms.clear();
      ns.clear();
      for (int b = 0; b < B && next < P; ++b) {
        if (hp[b] < 0 || hk[b] >= hl[b]) {
          const int pi = order[next];
          hp[b] = pi;
          hk[b] = 0;
          hl[b] = len_host[pi];
          slots.push_back(b);
          ms.push_back(m_host[pi]);
          ns.push_back(n_host[pi]);
          ++next;
        }
      }
      if (!slots.empty()) {
        const int cnt = (int)slots.size();
        GWL_HIP(hipStreamSynchronize(stream));
        prof_flush();
        // mark slots that are done as empty
        for (int b = 0; b < B; ++b)
          if (hp[b] >= 0 && hk[b] >= hl[b]) hp[b] = -1;
        GWL_HIP(hipMemcpy(s_pair.p, hp.data(), B * sizeof(int), hipMemcpyHostToDevice));
        GWL_HIP(hipMemcpy(s_len.p, hl.data(), B * sizeof(int), hipMemcpyHostToDevice));
        GWL_HIP(hipMemcpy(s_slots.p, slots.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
        if (start_dev) {
          for (int i = 0; i < cnt; ++i)
            GWL_HIP(hipMemcpyAsync(q.p + (size_t)slots[i] * nvc,
                                   start_dev + (size_t)hp[slots[i]] * nvc, nvc * sizeof(double),
                                   hipMemcpyDeviceToDevice, stream));
        } else {
          // coupling vectors straight into q rows (contiguous run of slots
          // when all refill at once; otherwise one row at a time via w)
          bool contiguous = true;
          for (int i = 0; i < cnt; ++i) contiguous &= (slots[i] == slots[0] + i);
          if (contiguous) {
            coupling_batch(cnt, ms.data(), ns.data(), q.p + (size_t)slots[0] * nvc, nvc);
          } else {
            coupling_batch(cnt, ms.data(), ns.data(), w.p, nvc);
            for (int i = 0; i < cnt; ++i)
              GWL_HIP(hipMemcpyAsync(q.p + (size_t)slots[i] * nvc, w.p + (size_t)i * nvc,
                                     nvc * sizeof(double), hipMemcpyDeviceToDevice, stream));
          }
        }
        lz_start(ss, B, s_slots.p, cnt, q.p, qprev.p, full ? basis.p : nullptr, bstride, nvc,
                 stream);
      }
      int kmax = 0;
      act.clear();
      for (int b = 0; b < B; ++b)
        if (hp[b] >= 0 && hk[b] < hl[b]) {
          act.push_back(b);
          kmax = std::max(kmax, hk[b]);
        }
      if (act.empty()) break;
      // one Lanczos step for every slot; once slots fall idle (queue empty)
      // the product runs over the busy ones only
      const int nact = (int)act.size();
      if (nact < B && act != act_dev) {
        GWL_HIP(hipStreamSynchronize(stream));
        GWL_HIP(hipMemcpy(s_act.p, act.data(), nact * sizeof(int), hipMemcpyHostToDevice));
        act_dev = act;
      }
      if (nact < B) cur_rows = s_act.p;
      try {
        if (on_c)
          apply_c_batch(nact, q.p, w.p, prec);
        else if (tda)
          apply_a_batch(nact, q.p, w.p, prec);
        else
          apply_d_step(nact, prec);
      } catch (...) {
        cur_rows = nullptr;
        throw;
      }
      cur_rows = nullptr;
      lz_alpha(ss, B, q.p, qprev.p, w.p, nvc, stream);
      lz_reorth(ss, B, kmax, reorth, full ? basis.p : nullptr, bstride, q.p, qprev.p, w.p,
                hbuf.p, ReorthScratch{rw_n0.p, rw_part.p, rw_skip.p}, nvc, stream);
      lz_beta(ss, B, q.p, qprev.p, w.p, full ? basis.p : nullptr, bstride, full ? 1 : 0, nvc,
              stream);
      for (int b = 0; b < B; ++b)
        if (hp[b] >= 0 && hk[b] < hl[b]) ++hk[b];
      // bound the number of outstanding timing events
      if (profile && prof_recs.size() > 4096) {
        GWL_HIP(hipStreamSynchronize(stream));
        prof_flush();
      }
    }
    GWL_HIP(hipStreamSynchronize(stream));
    prof_flush();
  }

  int auto_block(int P, int L) const {
    // memory per slot: basis (FULL) + work vectors; keep the basis under 64 GB
    const double per_slot = (reorth == GWL_REORTH_FULL ? (double)L * nvc * 8 : 0.0) +
                            8.0 * nvc * 8 + 4.0 * gd.nrp * 8;
    int B = (int)std::min<double>(256.0, 64e9 / std::max(per_slot, 1.0));
    if (nvc <= 4096) B = 256;
    B = std::max(1, std::min(B, P));
    return B;
  }

  // Upper end of the spectrum of C: Lanczos on C from a fixed pseudo-random
  // start, largest Ritz value theta of the steps x steps tridiagonal plus its
  // residual bound |b_steps u_last| (one more step supplies b_steps; the
  // residual is 0 when the recurrence ends in an invariant subspace), 1 %
  // margin.  A Ritz residual locates an eigenvalue near theta, it does not
  // bound the spectrum; the Sturm check after every Lanczos run on p_g(C)
  // catches an estimate that fell short.
  double estimate_hi() {
    const int steps = (int)std::min<long>(40, nvc);
    const int len = steps < nvc ? steps + 1 : steps;
    std::vector<double> x0(nvc);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (long i = 0; i < nvc; ++i) {
      st ^= st << 13;
      st ^= st >> 7;
      st ^= st << 17;
      x0[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
    }
    DevBuf<double> start;
    start.ensure(nvc);
    GWL_HIP(hipMemcpy(start.p, x0.data(), nvc * sizeof(double), hipMemcpyHostToDevice));
    const int saved_reorth = reorth, saved_block = block, saved_prec = precision;
    const int saved_tda = tda;
    reorth = GWL_REORTH_FULL;
    block = 1;
    precision = GWL_FP64;
    tda = 0;
    int m0 = 0, n0 = 0, lreq = len;
    run_pairs(1, &m0, &n0, &lreq, len, true, start.p);
    reorth = saved_reorth;
    block = saved_block;
    precision = saved_prec;
    tda = saved_tda;
    std::vector<double> a(len), b(len);
    int lout = 0;
    GWL_HIP(hipMemcpy(a.data(), coef_a.p, len * sizeof(double), hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(b.data(), coef_b.p, len * sizeof(double), hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(&lout, out_len.p, sizeof(int), hipMemcpyDeviceToHost));
    GWL_CHECK(lout >= 1 && finite_all(a.data(), lout) && finite_all(b.data(), lout),
              GWL_ENUMERIC, "spectrum estimate failed");
    const int L = std::min(lout, steps);
    std::vector<double> t((size_t)L * L, 0.0), vec;
    for (int i = 0; i < L; ++i) {
      t[(size_t)i * L + i] = a[i];
      if (i + 1 < L) t[(size_t)i * L + i + 1] = t[(size_t)(i + 1) * L + i] = b[i];
    }
    jacobi_eig(L, t, vec);
    int imax = 0;
    for (int i = 1; i < L; ++i)
      if (t[(size_t)i * L + i] > t[(size_t)imax * L + imax]) imax = i;
    const double theta = t[(size_t)imax * L + imax];
    hi_resid = (lout > steps) ? std::fabs(b[steps - 1] * vec[(size_t)(L - 1) * L + imax]) : 0.0;
    return (theta + hi_resid) * 1.01;
  }

  // Range [pmin, pmax] of p_g over [lo, hi]: the polynomial sampled at 8193
  // points x = cos(theta), theta uniform (dense near both ends), by Clenshaw.
  void poly_range(double& pmin, double& pmax) const {
    const int ns = 8193;
    pmin = 1e300;
    pmax = -1e300;
    for (int i = 0; i < ns; ++i) {
      const double x = std::cos(kPi * i / (ns - 1));
      double b1 = 0.0, b2 = 0.0;
      for (int j = (int)cheb.size() - 1; j >= 1; --j) {
        const double b0 = cheb[j] + 2.0 * x * b1 - b2;
        b2 = b1;
        b1 = b0;
      }
      const double p = cheb[0] + x * b1 - b2;
      pmin = std::min(pmin, p);
      pmax = std::max(pmax, p);
    }
  }

  // After Lanczos runs on p_g(C) (coefficients of P pairs in coef_a/coef_b,
  // lengths out_len, leading dimension ld): fail with GWL_ENUMERIC when some
  // run's tridiagonal has an eigenvalue outside [pmin - tol, pmax + tol],
  // tol = 0.5 % of max |p_g| -- the spectrum of C left [lo, hi] and p_g
  // extrapolated there.
  void check_interval(int P, int ld) {
    double pmin, pmax;
    poly_range(pmin, pmax);
    const double tol = 5e-3 * std::max(std::fabs(pmin), std::fabs(pmax));
    ivbad.ensure(P);
    lz_interval_check(P, coef_a.p, coef_b.p, out_len.p, ld, pmin - tol, pmax + tol, ivbad.p,
                      stream);
    std::vector<int> bad(P);
    GWL_HIP(hipMemcpyAsync(bad.data(), ivbad.p, P * sizeof(int), hipMemcpyDeviceToHost, stream));
    GWL_HIP(hipStreamSynchronize(stream));
    int nbad = 0;
    for (int v : bad) nbad += v != 0;
    GWL_CHECK(nbad == 0, GWL_ENUMERIC,
              "the spectrum of C leaves the Chebyshev interval [" + std::to_string(poly_lo) +
                  ", " + std::to_string(poly_hi) + "] hartree^2 (" + std::to_string(nbad) +
                  " of " + std::to_string(P) + " runs): p_g(C) is no square root there");
  }
};
