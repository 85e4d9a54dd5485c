// Host runtime and C ABI of the Lanczos GW self-energy library (see gwl.h).
//
// One context per orbital set.  Setup packs the orbitals into the GEMM
// layouts (FP64 always; BF16/FP32 copies for the mixed mode), builds Delta,
// the FFT tables and the Chebyshev coefficients of p_g ~ sqrt.  The
// self-energy runs a slot scheduler: B Lanczos slots advance together, one
// p_g(C) product (g factored C-products) per step, and a slot whose run has
// reached its length is refilled with the next (m, n) start vector, whose
// coupling vector is built on the spot.  All coefficients stay on the device
// until the continued fraction has produced Sigma.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace gwl {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

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
std::vector<double> cheb_sqrt(double lo, double hi, int g) {
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
void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& vec) {
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

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

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
  std::vector<double> cheb;
  std::vector<double> eps_ha;

  // operands
  DevBuf<double> psi_t;       // [NVp + NCp][NRp]
  DevBuf<double> psi_c_rc64;  // [NRp][NCp]
  DevBuf<double> psi_v_rv64;  // [NRp][NVp]
  DevBuf<bf16_t> psi_t16;     // [NVp + NCp][NRp]
  DevBuf<bf16_t> psi_c_rc16;  // [NRp][NCp]
  DevBuf<float> psi_v_rv32;   // [NRp][NVp] (plain BF16 kernel epilogue)
  DevBuf<bf16_t> psi_v_rv16;  // [NRp][NVp] (MFMA BF16 kernel epilogue)
  DevBuf<double> delta2, sdelta;

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
  DevBuf<bf16_t> u16;          // [cap][NVp][NCp]
  DevBuf<unsigned char> rho;   // [nvt][cap][NRp] x 8 (fully written by the first GEMM)
  DevBuf<double> vpot64;       // [cap][NRp]
  DevBuf<float> vpot32;        // [cap][NRp]
  DevBuf<unsigned char> fftx;  // [(cap+1)/2][N_r] x 16
  DevBuf<unsigned char> ypart; // [S][cap][NVp][NCp] x 8
  DevBuf<double> basis;        // [cap][cap_L][nvc]
  DevBuf<double> hbuf;         // [cap][cap_L + 1]
  DevBuf<int> s_pair, s_k, s_len, s_dead, s_slots, s_m, s_n;
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
  hipGraphExec_t dgraph = nullptr;
  int dg_nb = -1, dg_prec = -1, dg_S = -1, dg_kern = -1, dg_deg = -1;
  double dg_lo = 0, dg_hi = 0;
  long work_gen = 0, dg_gen = -1;

  // autotuned (block, split) per precision
  struct Tune {
    int B = 0, S = 0;
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

  PairGeom pair_geom() const {
    PairGeom g;
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
    return std::max(std::max(gemm1_f64_vtiles(gd), gemm1_bf16s_vtiles(gd)),
                    std::max(gemm1_f64m_vtiles(gd), gemm1_bf16_vtiles(gd)));
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
    long blocks;
    if (!fp64_kernel)
      blocks = (long)nb * (gd.nvp / 64) * ceil_div(gd.ncp, 64);
    else if (prec == GWL_FP64)
      blocks = gemm2_f64m_blocks(gd, nb);
    else
      blocks = gemm2_bf16_blocks(gd, nb);
    int s = 1;
    while (blocks * s < 1024 && s < 32 && (long)gd.nrp / (s * 2) >= 2048) s *= 2;
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
      u16.ensure((size_t)nb * nvpc);
      rho.ensure((size_t)nvt_max() * nb * gd.nrp * 8);
      vpot64.ensure((size_t)nb * gd.nrp);
      vpot32.ensure((size_t)nb * gd.nrp);
      fftx.ensure((size_t)((nb + 1) / 2) * nr * 16);
      ypart.ensure((size_t)32 * nb * nvpc * 8);
      s_pair.ensure(nb);
      s_k.ensure(nb);
      s_len.ensure(nb);
      s_dead.ensure(nb);
      s_slots.ensure(nb);
      s_m.ensure(nb);
      s_n.ensure(nb);
      s_amax.ensure(nb);
      s_bprev.ensure(nb);
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
  // ypart <- second GEMM of K applied to u (u already cast for nb vectors).
  void k_product(int nb, int prec, int S) {
    hipStream_t st = stream;
    if (prec == GWL_FP64) {
      const double* uu = u64.p;
      double* rp = reinterpret_cast<double*>(rho.p);
      double* vp = vpot64.p;
      double* yp = reinterpret_cast<double*>(ypart.p);
      int nvt;
      prof_begin();
      if (fp64_kernel) {
        gemm1_f64m(gd, nb, psi_c_rc64.p, psi_v_rv64.p, uu, rp, st);
        nvt = gemm1_f64m_vtiles(gd);
      } else {
        gemm1_f64(gd, nb, psi_c_rc64.p, psi_v_rv64.p, uu, rp, st);
        nvt = gemm1_f64_vtiles(gd);
      }
      prof_end(0, nb);
      prof_begin();
      poisson_launch<double>(pg64, rp, gd.nrp, (long)nb * gd.nrp, nvt, vp, gd.nrp, nb,
                             reinterpret_cast<cplx<double>*>(fftx.p), st);
      prof_end(2, nb);
      const double* pv = psi_t.p;
      const double* pc = psi_t.p + (size_t)gd.nvp * gd.nrp;
      prof_begin();
      if (fp64_kernel)
        gemm2_f64m(gd, nb, S, pv, pc, vp, yp, st);
      else
        gemm2_f64(gd, nb, S, pv, pc, vp, yp, st);
      prof_end(1, nb);
    } else {
      const bf16_t* uu = u16.p;
      float* rp = reinterpret_cast<float*>(rho.p);
      float* vp = vpot32.p;
      float* yp = reinterpret_cast<float*>(ypart.p);
      int nvt;
      prof_begin();
      if (fp64_kernel) {
        gemm1_bf16(gd, nb, psi_c_rc16.p, psi_v_rv16.p, uu, rp, st);
        nvt = gemm1_bf16_vtiles(gd);
      } else {
        gemm1_bf16s(gd, nb, psi_c_rc16.p, psi_v_rv32.p, uu, rp, st);
        nvt = gemm1_bf16s_vtiles(gd);
      }
      prof_end(0, nb);
      prof_begin();
      poisson_launch<float>(pg32, rp, gd.nrp, (long)nb * gd.nrp, nvt, vp, gd.nrp, nb,
                            reinterpret_cast<cplx<float>*>(fftx.p), st);
      prof_end(2, nb);
      const bf16_t* pv = psi_t16.p;
      const bf16_t* pc = psi_t16.p + (size_t)gd.nvp * gd.nrp;
      prof_begin();
      if (fp64_kernel)
        gemm2_bf16(gd, nb, S, pv, pc, vp, yp, st);
      else
        gemm2_bf16s(gd, nb, S, pv, pc, vp, yp, st);
      prof_end(1, nb);
    }
  }

  void cast(int nb, const double* x, int prec) {
    PairGeom g = pair_geom();
    if (prec == GWL_FP64)
      cast_u<double>(g, nb, x, nvc, u64.p, stream);
    else
      cast_u<bf16_t>(g, nb, x, nvc, u16.p, stream);
  }

  void do_combine(int nb, int S, int prec, const double* x, const double* tp, double* out,
                  double* acc, int mode, double c0, double cj, bool write_u) {
    PairGeom g = pair_geom();
    if (prec == GWL_FP64)
      combine<double, double>(g, nb, S, reinterpret_cast<const double*>(ypart.p), x, tp, out,
                              acc, mode, poly_lo, poly_hi, c0, cj,
                              write_u ? u64.p : nullptr, stream);
    else
      combine<float, bf16_t>(g, nb, S, reinterpret_cast<const float*>(ypart.p), x, tp, out,
                             acc, mode, poly_lo, poly_hi, c0, cj,
                             write_u ? u16.p : nullptr, stream);
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
    double* rp = reinterpret_cast<double*>(rho.p);
    double* vp = vpot64.p;
    double* yp = reinterpret_cast<double*>(ypart.p);
    pair_product(psi_t.p, gd.nrp, (int)nr, s_m.p, s_n.p, cnt, rp, stream);
    poisson_launch<double>(pg64, rp, gd.nrp, 0, 1, vp, gd.nrp, cnt,
                           reinterpret_cast<cplx<double>*>(fftx.p), stream);
    const int S = auto_splitk(cnt, GWL_FP64);
    const double* pv = psi_t.p;
    const double* pc = psi_t.p + (size_t)gd.nvp * gd.nrp;
    if (fp64_kernel)
      gemm2_f64m(gd, cnt, S, pv, pc, vp, yp, stream);
    else
      gemm2_f64(gd, cnt, S, pv, pc, vp, yp, stream);
    coupling_finish<double>(pair_geom(), cnt, S, yp, dst, ldp, stream);
  }

  // w = p_g(C) q over nb slots; replays a captured graph of the whole product
  // (g x [first GEMM, five FFT passes, second GEMM, combine] + cast) when the
  // shapes and buffers are unchanged.
  void apply_d_step(int nb, int prec) {
    last_c_matvecs += (long)nb * poly_degree;
    const int S = auto_splitk(nb, prec);
    if (!use_graphs || profile) {
      apply_d_batch(nb, q.p, w.p, prec, false);
      return;
    }
    if (!dgraph || dg_nb != nb || dg_prec != prec || dg_S != S || dg_kern != fp64_kernel ||
        dg_gen != work_gen || dg_deg != poly_degree || dg_lo != poly_lo || dg_hi != poly_hi) {
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
    }
    GWL_HIP(hipGraphLaunch(dgraph, stream));
  }

  void drop_graph() {
    if (dgraph) (void)hipGraphExecDestroy(dgraph);
    dgraph = nullptr;
  }

  // ---------------------------------------------------------------- autotuner
  // Pick the number of Lanczos slots B and the split of the second GEMM by
  // timing one C-product per candidate with HIP events on the context
  // stream; the time per pair vector decides.  Results are kept per context
  // and, when GWL_TUNE_CACHE names a file, shared through it (one line per
  // problem shape: "key B S us_per_vector").
  std::string tune_key(int prec) const {
    return "gfx950:" + std::to_string(nr) + ":" + std::to_string(nv) + ":" +
           std::to_string(nc) + ":" + std::to_string(prec) + ":" + std::to_string(fp64_kernel);
  }

  bool tune_cache_read(int prec, Tune& t) const {
    const char* path = std::getenv("GWL_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char key[256];
    int b = 0, sk = 0;
    double us = 0;
    bool found = false;
    const std::string want = tune_key(prec);
    while (std::fscanf(f, "%255s %d %d %lf", key, &b, &sk, &us) == 4)
      if (want == key && b > 0 && sk > 0) {
        t.B = b;
        t.S = sk;
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
    std::fprintf(f, "%s %d %d %.3f\n", tune_key(prec).c_str(), t.B, t.S, t.us_per_vec);
    std::fclose(f);
  }

  Tune autotune(int prec, int bmax) {
    Tune best = tuned[prec];
    if (best.B > 0) return best;
    if (tune_cache_read(prec, best)) {
      tuned[prec] = best;
      return best;
    }
    const int cands[] = {32, 64, 128, 256};
    hipEvent_t e0, e1;
    GWL_HIP(hipEventCreate(&e0));
    GWL_HIP(hipEventCreate(&e1));
    best.us_per_vec = 1e300;
    try {
      for (int B : cands) {
        if (B > bmax && B != cands[0]) break;
        ensure_work(B, 1, false);
        const int s0 = heuristic_splitk(B, prec);
        for (int S : {s0 / 2, s0, s0 * 2}) {
          if (S < 1 || S > 32 || (S > 1 && (long)gd.nrp / S < 1024)) continue;
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
            best.us_per_vec = us;
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
      best.B = std::max(1, std::min(bmax, 128));
      best.S = heuristic_splitk(best.B, prec);
      best.us_per_vec = 0;
    }
    tuned[prec] = best;
    tune_cache_write(prec, best);
    return best;
  }

  // ---------------------------------------------------------------- scheduler
  // Run Lanczos on p_g(C) (or on C itself when on_c) for P start vectors
  // (m_i, n_i) with lengths len_i.  Coefficients land in coef_a/coef_b
  // ([P][ld]), norm2 [P], out_len [P] on the device.
  void run_pairs(int P, const int* m_host, const int* n_host, const int* len_host, int ld,
                 bool on_c = false, const double* start_dev = nullptr) {
    const int prec = precision;
    int B;
    if (block > 0) {
      B = block;
    } else {
      const int bmem = auto_block(1 << 30, ld);  // memory cap on slots
      B = std::min(autotune(prec, bmem).B, bmem);
    }
    B = std::max(1, std::min(B, P));
    const bool full = (reorth == GWL_REORTH_FULL);
    ensure_work(B, ld, full);
    coef_a.ensure((size_t)P * ld);
    coef_b.ensure((size_t)P * ld);
    norm2.ensure(P);
    out_len.ensure(P);
    GWL_HIP(hipMemsetAsync(coef_a.p, 0, sizeof(double) * (size_t)P * ld, stream));
    GWL_HIP(hipMemsetAsync(coef_b.p, 0, sizeof(double) * (size_t)P * ld, stream));
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
    const long bstride = (long)ld * nvc;
    std::vector<int> hp(B, -1), hk(B, 0), hl(B, 0);
    GWL_HIP(hipMemcpyAsync(s_pair.p, hp.data(), B * sizeof(int), hipMemcpyHostToDevice, stream));
    GWL_HIP(hipStreamSynchronize(stream));
    int next = 0;
    std::vector<int> slots, ms, ns;
    while (true) {
      // refill
      slots.clear();
      ms.clear();
      ns.clear();
      for (int b = 0; b < B && next < P; ++b) {
        if (hp[b] < 0 || hk[b] >= hl[b]) {
          hp[b] = next;
          hk[b] = 0;
          hl[b] = len_host[next];
          slots.push_back(b);
          ms.push_back(m_host[next]);
          ns.push_back(n_host[next]);
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
      bool any = false;
      int kmax = 0;
      for (int b = 0; b < B; ++b)
        if (hp[b] >= 0 && hk[b] < hl[b]) {
          any = true;
          kmax = std::max(kmax, hk[b]);
        }
      if (!any) break;
      // one Lanczos step for every slot
      if (on_c)
        apply_c_batch(B, q.p, w.p, prec);
      else
        apply_d_step(B, prec);
      lz_alpha(ss, B, q.p, qprev.p, w.p, nvc, stream);
      lz_reorth(ss, B, kmax, reorth, full ? basis.p : nullptr, bstride, q.p, qprev.p, w.p,
                hbuf.p, nvc, stream);
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
  // start, largest Ritz value plus its residual bound, 1% margin.
  double estimate_hi() {
    const int steps = (int)std::min<long>(40, nvc);
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
    reorth = GWL_REORTH_FULL;
    block = 1;
    precision = GWL_FP64;
    int m0 = 0, n0 = 0, len = steps;
    run_pairs(1, &m0, &n0, &len, steps, true, start.p);
    reorth = saved_reorth;
    block = saved_block;
    precision = saved_prec;
    std::vector<double> a(steps), b(steps);
    int L = 0;
    GWL_HIP(hipMemcpy(a.data(), coef_a.p, steps * sizeof(double), hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(b.data(), coef_b.p, steps * sizeof(double), hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(&L, out_len.p, sizeof(int), hipMemcpyDeviceToHost));
    GWL_CHECK(L >= 1 && finite_all(a.data(), L), GWL_ENUMERIC, "spectrum estimate failed");
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
    const double resid = (L < steps) ? 0.0 : std::fabs(b[L - 1] * vec[(size_t)(L - 1) * L + imax]);
    return (theta + resid) * 1.01;
  }
};

namespace {

template <typename F>
gwl_status guarded(F&& f) {
  try {
    f();
    set_error("");
    return GWL_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GWL_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GWL_EDEVICE;
  }
}

template <typename T>
void upload_tables(int n, double len, DevBuf<cplx<T>>& tw, DevBuf<T>& g2) {
  std::vector<cplx<T>> h(n);
  std::vector<T> gg(n);
  for (int k = 0; k < n; ++k) {
    const double a = -2.0 * kPi * k / n;
    h[k] = {(T)std::cos(a), (T)std::sin(a)};
    const int f = std::min(k, n - k);
    const double g = 2.0 * kPi * f / len;
    gg[k] = (T)(g * g);
  }
  tw.ensure(n);
  g2.ensure(n);
  GWL_HIP(hipMemcpy(tw.p, h.data(), n * sizeof(cplx<T>), hipMemcpyHostToDevice));
  GWL_HIP(hipMemcpy(g2.p, gg.data(), n * sizeof(T), hipMemcpyHostToDevice));
}

void check_ctx(gwl_ctx* c) { GWL_CHECK(c != nullptr, GWL_EINVAL, "null context"); }

}  // namespace

extern "C" {

void gwl_default_options(gwl_options* o) {
  if (!o) return;
  o->precision = GWL_FP64;
  o->poly_degree = 7;
  o->poly_lo = 0.0;
  o->poly_hi = 0.0;
  o->reorth = GWL_REORTH_FULL;
  o->block = 0;
  o->kernel_scale = 1.0;
  o->stream = nullptr;
}

const char* gwl_last_error(void) { return g_last_error.c_str(); }

gwl_status gwl_setup(const void* orbitals, int orb_dtype, int orb_on_device, int n_orb,
                     int n_occ, const double* energies_ev, const gwl_grid* grid,
                     const gwl_options* opts, gwl_ctx** out) {
  return guarded([&] {
    GWL_CHECK(orbitals && energies_ev && grid && out, GWL_EINVAL, "null pointer argument");
    GWL_CHECK(orb_dtype == 8 || orb_dtype == 4, GWL_EINVAL, "orb_dtype must be 8 or 4");
    GWL_CHECK(n_orb >= 2 && n_occ >= 1 && n_occ < n_orb, GWL_EINVAL,
              "need 1 <= n_occ < n_orb");
    GWL_CHECK(grid->nx >= 2 && grid->ny >= 2 && grid->nz >= 2 && grid->nx <= 256 &&
                  grid->ny <= 256 && grid->nz <= 256,
              GWL_EUNSUPPORTED, "grid edges must be in [2, 256]");
    GWL_CHECK(grid->lx > 0 && grid->ly > 0 && grid->lz > 0 && std::isfinite(grid->lx) &&
                  std::isfinite(grid->ly) && std::isfinite(grid->lz),
              GWL_EINVAL, "box edges must be positive");
    gwl_options o;
    gwl_default_options(&o);
    if (opts) o = *opts;
    GWL_CHECK(o.precision == GWL_FP64 || o.precision == GWL_MIXED_BF16, GWL_EINVAL,
              "unknown precision");
    GWL_CHECK(o.poly_degree >= 1 && o.poly_degree <= 30, GWL_EINVAL,
              "poly_degree must be in [1, 30]");
    GWL_CHECK(o.reorth >= 0 && o.reorth <= 2, GWL_EINVAL, "unknown reorth mode");
    GWL_CHECK(o.block >= 0, GWL_EINVAL, "block must be >= 0");
    GWL_CHECK(std::isfinite(o.kernel_scale) && o.kernel_scale >= 0, GWL_EINVAL,
              "kernel_scale must be finite and >= 0");
    GWL_CHECK(finite_all(energies_ev, n_orb), GWL_EINVAL, "non-finite energy");
    double emax_occ = -1e300, emin_emp = 1e300;
    for (int i = 0; i < n_occ; ++i) emax_occ = std::max(emax_occ, energies_ev[i]);
    for (int i = n_occ; i < n_orb; ++i) emin_emp = std::min(emin_emp, energies_ev[i]);
    GWL_CHECK(emin_emp > emax_occ, GWL_EINVAL,
              "every empty energy must exceed every occupied one (Delta > 0)");

    auto ctx = std::make_unique<gwl_ctx>();
    gwl_ctx& c = *ctx;
    GWL_HIP(hipGetDevice(&c.device));
    if (o.stream) {
      c.stream = (hipStream_t)o.stream;
    } else {
      GWL_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
      c.own_stream = true;
    }
    c.nx = grid->nx;
    c.ny = grid->ny;
    c.nz = grid->nz;
    c.lx = grid->lx;
    c.ly = grid->ly;
    c.lz = grid->lz;
    c.nr = (long)c.nx * c.ny * c.nz;
    c.n_orb = n_orb;
    c.nv = n_occ;
    c.nc = n_orb - n_occ;
    c.nvc = (long)c.nv * c.nc;
    c.dv = (c.lx / c.nx) * (c.ly / c.ny) * (c.lz / c.nz);
    c.gd.nr = (int)c.nr;
    c.gd.nrp = (int)round_up(c.nr, kPadR);
    c.gd.nv = c.nv;
    c.gd.nvp = pad_nv(c.nv);
    c.gd.nc = c.nc;
    c.gd.ncp = (int)round_up(c.nc, kPadC);
    c.precision = o.precision;
    c.poly_degree = o.poly_degree;
    c.reorth = o.reorth;
    c.block = o.block;
    c.kernel_scale = o.kernel_scale;
    for (int a = 0; a < 3; ++a) {
      const int n = a == 0 ? c.nx : (a == 1 ? c.ny : c.nz);
      GWL_CHECK(make_plan(n).ok, GWL_EUNSUPPORTED,
                "grid edge " + std::to_string(n) + " does not factor into 2, 3, 4, 8");
    }

    // energies, Delta
    c.eps_ha.resize(n_orb);
    for (int i = 0; i < n_orb; ++i) c.eps_ha[i] = energies_ev[i] / kHartreeEv;
    std::vector<double> d2(c.nvc), sd(c.nvc);
    double dmin = 1e300;
    for (int v = 0; v < c.nv; ++v)
      for (int cc = 0; cc < c.nc; ++cc) {
        const double d = c.eps_ha[c.nv + cc] - c.eps_ha[v];
        d2[(size_t)v * c.nc + cc] = d * d;
        sd[(size_t)v * c.nc + cc] = std::sqrt(d);
        dmin = std::min(dmin, d);
      }
    c.delta2.ensure(c.nvc);
    c.sdelta.ensure(c.nvc);
    GWL_HIP(hipMemcpy(c.delta2.p, d2.data(), c.nvc * 8, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(c.sdelta.p, sd.data(), c.nvc * 8, hipMemcpyHostToDevice));

    // orbitals -> FP64 host staging in the padded transposed layout
    const long nrp = c.gd.nrp;
    const int nvp = c.gd.nvp, ncp = c.gd.ncp;
    std::vector<double> host((size_t)(nvp + ncp) * nrp, 0.0);
    {
      std::vector<unsigned char> raw;
      const unsigned char* src = static_cast<const unsigned char*>(orbitals);
      const size_t bytes = (size_t)n_orb * c.nr * orb_dtype;
      if (orb_on_device) {
        raw.resize(bytes);
        GWL_HIP(hipMemcpy(raw.data(), orbitals, bytes, hipMemcpyDeviceToHost));
        src = raw.data();
      }
      for (int n = 0; n < n_orb; ++n) {
        double* dst = host.data() + (size_t)c.orb_row(n) * nrp;
        if (orb_dtype == 8) {
          const double* s = reinterpret_cast<const double*>(src) + (size_t)n * c.nr;
          for (long r = 0; r < c.nr; ++r) dst[r] = s[r];
        } else {
          const float* s = reinterpret_cast<const float*>(src) + (size_t)n * c.nr;
          for (long r = 0; r < c.nr; ++r) dst[r] = s[r];
        }
      }
      GWL_CHECK(finite_all(host.data(), host.size()), GWL_EINVAL, "non-finite orbital value");
    }
    c.psi_t.ensure(host.size());
    GWL_HIP(hipMemcpy(c.psi_t.p, host.data(), host.size() * 8, hipMemcpyHostToDevice));
    {
      std::vector<double> crc((size_t)nrp * ncp, 0.0), vrv((size_t)nrp * nvp, 0.0);
      for (int cc = 0; cc < ncp; ++cc) {
        const double* s = host.data() + (size_t)(nvp + cc) * nrp;
        for (long r = 0; r < nrp; ++r) crc[(size_t)r * ncp + cc] = s[r];
      }
      for (int v = 0; v < nvp; ++v) {
        const double* s = host.data() + (size_t)v * nrp;
        for (long r = 0; r < nrp; ++r) vrv[(size_t)r * nvp + v] = s[r];
      }
      c.psi_c_rc64.ensure(crc.size());
      c.psi_v_rv64.ensure(vrv.size());
      GWL_HIP(hipMemcpy(c.psi_c_rc64.p, crc.data(), crc.size() * 8, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.psi_v_rv64.p, vrv.data(), vrv.size() * 8, hipMemcpyHostToDevice));
      // mixed-precision copies
      std::vector<bf16_t> t16(host.size()), c16(crc.size());
      for (size_t i = 0; i < host.size(); ++i) t16[i] = f32_to_bf16((float)host[i]);
      for (size_t i = 0; i < crc.size(); ++i) c16[i] = f32_to_bf16((float)crc[i]);
      std::vector<float> v32(vrv.size());
      std::vector<bf16_t> v16(vrv.size());
      for (size_t i = 0; i < vrv.size(); ++i) {
        v32[i] = (float)vrv[i];
        v16[i] = f32_to_bf16(v32[i]);
      }
      c.psi_t16.ensure(t16.size());
      c.psi_c_rc16.ensure(c16.size());
      c.psi_v_rv32.ensure(v32.size());
      c.psi_v_rv16.ensure(v16.size());
      GWL_HIP(hipMemcpy(c.psi_v_rv16.p, v16.data(), v16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.psi_t16.p, t16.data(), t16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.psi_c_rc16.p, c16.data(), c16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.psi_v_rv32.p, v32.data(), v32.size() * 4, hipMemcpyHostToDevice));
    }

    // FFT tables
    const double lens[3] = {c.lx, c.ly, c.lz};
    const int ns[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a) {
      upload_tables<double>(ns[a], lens[a], c.tw64[a], c.g2_64[a]);
      upload_tables<float>(ns[a], lens[a], c.tw32[a], c.g2_32[a]);
    }
    auto fill_geom = [&](auto& pg, auto& tw, auto& g2) {
      pg.nx = c.nx;
      pg.ny = c.ny;
      pg.nz = c.nz;
      pg.px = make_plan(c.nx);
      pg.py = make_plan(c.ny);
      pg.pz = make_plan(c.nz);
      pg.twx = tw[0].p;
      pg.twy = tw[1].p;
      pg.twz = tw[2].p;
      pg.g2x = g2[0].p;
      pg.g2y = g2[1].p;
      pg.g2z = g2[2].p;
    };
    fill_geom(c.pg64, c.tw64, c.g2_64);
    fill_geom(c.pg32, c.tw32, c.g2_32);
    c.pg64.vscale = c.kernel_scale * 4.0 * kPi / (double)c.nr;
    c.pg32.vscale = (float)(c.kernel_scale * 4.0 * kPi / (double)c.nr);

    // Chebyshev interval and coefficients
    c.poly_lo = o.poly_lo > 0 ? o.poly_lo : dmin * dmin;
    if (o.poly_hi > 0) {
      c.poly_hi = o.poly_hi;
    } else {
      c.poly_hi = 1.0;  // placeholder for the estimate's own C-products
      c.cheb = cheb_sqrt(c.poly_lo, c.poly_hi, c.poly_degree);
      c.poly_hi = std::max(c.estimate_hi(), c.poly_lo * (1.0 + 1e-6));
    }
    GWL_CHECK(c.poly_hi > c.poly_lo, GWL_EINVAL, "poly_hi must exceed poly_lo");
    c.cheb = cheb_sqrt(c.poly_lo, c.poly_hi, c.poly_degree);
    GWL_HIP(hipStreamSynchronize(c.stream));
    *out = ctx.release();
  });
}

void gwl_destroy(gwl_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  ctx->drop_graph();
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

gwl_status gwl_set_option(gwl_ctx* ctx, int key, double value) {
  return guarded([&] {
    check_ctx(ctx);
    switch (key) {
      case GWL_KEY_PRECISION:
        GWL_CHECK(value == GWL_FP64 || value == GWL_MIXED_BF16, GWL_EINVAL, "bad precision");
        ctx->precision = (int)value;
        break;
      case GWL_KEY_REORTH:
        GWL_CHECK(value >= 0 && value <= 2, GWL_EINVAL, "bad reorth");
        ctx->reorth = (int)value;
        break;
      case GWL_KEY_BLOCK:
        GWL_CHECK(value >= 0 && value <= 4096, GWL_EINVAL, "bad block");
        ctx->block = (int)value;
        break;
      case GWL_KEY_GEMM_SPLITK:
        GWL_CHECK(value >= 0 && value <= 32, GWL_EINVAL, "split must be in [0, 32]");
        ctx->splitk = (int)value;
        break;
      case GWL_KEY_KERNELS:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "kernels must be 0 or 1");
        ctx->fp64_kernel = (int)value;
        break;
      case GWL_KEY_PROFILE:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "profile must be 0 or 1");
        ctx->profile = (int)value;
        break;
      case GWL_KEY_GRAPHS:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "graphs must be 0 or 1");
        ctx->use_graphs = (int)value;
        if (!ctx->use_graphs) ctx->drop_graph();
        break;
      default:
        throw Error{GWL_EINVAL, "unknown or read-only option key"};
    }
  });
}

gwl_status gwl_query(gwl_ctx* ctx, int key, double* out) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(out != nullptr, GWL_EINVAL, "null output");
    switch (key) {
      case GWL_KEY_PRECISION: *out = ctx->precision; break;
      case GWL_KEY_REORTH: *out = ctx->reorth; break;
      case GWL_KEY_BLOCK: *out = ctx->block; break;
      case GWL_KEY_POLY_LO: *out = ctx->poly_lo; break;
      case GWL_KEY_POLY_HI: *out = ctx->poly_hi; break;
      case GWL_KEY_POLY_DEGREE: *out = ctx->poly_degree; break;
      case GWL_KEY_N_VC: *out = (double)ctx->nvc; break;
      case GWL_KEY_LAST_MS_TOTAL: *out = ctx->last_ms_total; break;
      case GWL_KEY_LAST_C_MATVECS: *out = (double)ctx->last_c_matvecs; break;
      case GWL_KEY_GEMM_SPLITK: *out = ctx->splitk; break;
      case GWL_KEY_KERNELS: *out = ctx->fp64_kernel; break;
      case GWL_KEY_PROFILE: *out = ctx->profile; break;
      case GWL_KEY_GRAPHS: *out = ctx->use_graphs; break;
      case GWL_KEY_TUNED_BLOCK: *out = ctx->tuned[ctx->precision].B; break;
      case GWL_KEY_TUNED_SPLITK: *out = ctx->tuned[ctx->precision].S; break;
      case GWL_KEY_PROF_MS_GEMM1: *out = ctx->prof_ms[0]; break;
      case GWL_KEY_PROF_N_GEMM1: *out = (double)ctx->prof_n[0]; break;
      case GWL_KEY_PROF_VEC_GEMM1: *out = (double)ctx->prof_vec[0]; break;
      case GWL_KEY_PROF_MS_GEMM2: *out = ctx->prof_ms[1]; break;
      case GWL_KEY_PROF_N_GEMM2: *out = (double)ctx->prof_n[1]; break;
      case GWL_KEY_PROF_VEC_GEMM2: *out = (double)ctx->prof_vec[1]; break;
      case GWL_KEY_PROF_MS_FFT: *out = ctx->prof_ms[2]; break;
      case GWL_KEY_PROF_N_FFT: *out = (double)ctx->prof_n[2]; break;
      case GWL_KEY_PROF_VEC_FFT: *out = (double)ctx->prof_vec[2]; break;
      default: throw Error{GWL_EINVAL, "unknown option key"};
    }
  });
}

gwl_status gwl_poisson(gwl_ctx* ctx, const void* rho, void* v, int n_fields, int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_fields >= 0, GWL_EINVAL, "n_fields < 0");
    if (n_fields == 0) return;
    GWL_CHECK(rho && v, GWL_EINVAL, "null pointer");
    GWL_CHECK(precision == GWL_FP64 || precision == GWL_MIXED_BF16, GWL_EINVAL,
              "bad precision");
    const int chunk = std::max(2, std::min(n_fields + (n_fields & 1), 64));
    ctx->ensure_work(chunk, 1, false);
    for (int f0 = 0; f0 < n_fields; f0 += chunk) {
      const int nf = std::min(chunk, n_fields - f0);
      if (precision == GWL_FP64)
        poisson_launch<double>(ctx->pg64, static_cast<const double*>(rho) + (size_t)f0 * ctx->nr,
                               ctx->nr, 0, 1, static_cast<double*>(v) + (size_t)f0 * ctx->nr,
                               ctx->nr, nf, reinterpret_cast<cplx<double>*>(ctx->fftx.p),
                               ctx->stream);
      else
        poisson_launch<float>(ctx->pg32, static_cast<const float*>(rho) + (size_t)f0 * ctx->nr,
                              ctx->nr, 0, 1, static_cast<float*>(v) + (size_t)f0 * ctx->nr,
                              ctx->nr, nf, reinterpret_cast<cplx<float>*>(ctx->fftx.p),
                              ctx->stream);
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
  });
}

gwl_status gwl_apply_c(gwl_ctx* ctx, const double* x, double* y, int n_vec, int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_vec >= 0, GWL_EINVAL, "n_vec < 0");
    if (n_vec == 0) return;
    GWL_CHECK(x && y, GWL_EINVAL, "null pointer");
    GWL_CHECK(precision == GWL_FP64 || precision == GWL_MIXED_BF16, GWL_EINVAL,
              "bad precision");
    ctx->prof_reset();
    const int chunk = std::min(n_vec, 64);
    ctx->ensure_work(chunk, 1, false);
    for (int i0 = 0; i0 < n_vec; i0 += chunk) {
      const int nb = std::min(chunk, n_vec - i0);
      ctx->apply_c_batch(nb, x + (size_t)i0 * ctx->nvc, y + (size_t)i0 * ctx->nvc, precision);
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof_flush();
  });
}

gwl_status gwl_apply_d(gwl_ctx* ctx, const double* x, double* y, int n_vec, int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_vec >= 0, GWL_EINVAL, "n_vec < 0");
    if (n_vec == 0) return;
    GWL_CHECK(x && y, GWL_EINVAL, "null pointer");
    GWL_CHECK(precision == GWL_FP64 || precision == GWL_MIXED_BF16, GWL_EINVAL,
              "bad precision");
    ctx->prof_reset();
    const int chunk = std::min(n_vec, 64);
    ctx->ensure_work(chunk, 1, false);
    for (int i0 = 0; i0 < n_vec; i0 += chunk) {
      const int nb = std::min(chunk, n_vec - i0);
      ctx->last_c_matvecs += (long)nb * ctx->poly_degree;
      ctx->apply_d_batch(nb, x + (size_t)i0 * ctx->nvc, y + (size_t)i0 * ctx->nvc, precision,
                         false);
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof_flush();
  });
}

gwl_status gwl_coupling(gwl_ctx* ctx, const int* m_idx, const int* n_idx, int count, double* p) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(count >= 0, GWL_EINVAL, "count < 0");
    if (count == 0) return;
    GWL_CHECK(m_idx && n_idx && p, GWL_EINVAL, "null pointer");
    for (int i = 0; i < count; ++i)
      GWL_CHECK(m_idx[i] >= 0 && m_idx[i] < ctx->n_orb && n_idx[i] >= 0 &&
                    n_idx[i] < ctx->n_orb,
                GWL_EINVAL, "orbital index out of range");
    const int chunk = std::min(count, 64);
    for (int i0 = 0; i0 < count; i0 += chunk) {
      const int cnt = std::min(chunk, count - i0);
      ctx->coupling_batch(cnt, m_idx + i0, n_idx + i0, p + (size_t)i0 * ctx->nvc, ctx->nvc);
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
  });
}

gwl_status gwl_lanczos_pairs(gwl_ctx* ctx, const int* m_idx, const int* n_idx, const int* lengths,
                             int n_pairs, double* alpha, double* beta, double* p_norm2,
                             int* out_len_h, int ld) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_pairs >= 0, GWL_EINVAL, "n_pairs < 0");
    if (n_pairs == 0) return;
    GWL_CHECK(m_idx && n_idx && lengths && alpha && beta && p_norm2, GWL_EINVAL,
              "null pointer");
    int lmax = 0;
    for (int i = 0; i < n_pairs; ++i) {
      GWL_CHECK(m_idx[i] >= 0 && m_idx[i] < ctx->n_orb && n_idx[i] >= 0 &&
                    n_idx[i] < ctx->n_orb,
                GWL_EINVAL, "orbital index out of range");
      GWL_CHECK(lengths[i] >= 1 && lengths[i] <= 4000, GWL_EINVAL,
                "lengths must be in [1, 4000]");
      lmax = std::max(lmax, lengths[i]);
    }
    GWL_CHECK(ld >= lmax, GWL_EINVAL, "ld < max(lengths)");
    auto t0 = std::chrono::steady_clock::now();
    ctx->last_c_matvecs = 0;
    ctx->prof_reset();
    ctx->run_pairs(n_pairs, m_idx, n_idx, lengths, lmax);
    std::vector<double> a((size_t)n_pairs * lmax), b((size_t)n_pairs * lmax), n2(n_pairs);
    std::vector<int> ol(n_pairs);
    GWL_HIP(hipMemcpy(a.data(), ctx->coef_a.p, a.size() * 8, hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(b.data(), ctx->coef_b.p, b.size() * 8, hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(n2.data(), ctx->norm2.p, n2.size() * 8, hipMemcpyDeviceToHost));
    GWL_HIP(hipMemcpy(ol.data(), ctx->out_len.p, ol.size() * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < n_pairs; ++i) {
      for (int k = 0; k < ld; ++k) {
        alpha[(size_t)i * ld + k] = k < ol[i] ? a[(size_t)i * lmax + k] : 0.0;
        beta[(size_t)i * ld + k] = k + 1 < ol[i] ? b[(size_t)i * lmax + k] : 0.0;
      }
      p_norm2[i] = n2[i];
      if (out_len_h) out_len_h[i] = ol[i];
      GWL_CHECK(std::isfinite(n2[i]) && finite_all(alpha + (size_t)i * ld, ol[i]) &&
                    finite_all(beta + (size_t)i * ld, ol[i]),
                GWL_ENUMERIC, "non-finite Lanczos coefficient");
    }
    ctx->last_ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

}  // extern "C"

namespace {

// Continued fraction over P pairs already on the device (coef_a/b, norm2,
// out_len of the context), then per-group sums when per > 0.
void sigma_device(gwl_ctx* ctx, int P, const int* n_host, int ld, const double* omega_ev,
                  int n_omega, double eta_ev) {
  std::vector<double> en(P), et(P), om(n_omega);
  for (int i = 0; i < P; ++i) {
    en[i] = ctx->eps_ha[n_host[i]];
    et[i] = n_host[i] < ctx->nv ? 1.0 : -1.0;
  }
  for (int i = 0; i < n_omega; ++i) om[i] = omega_ev[i] / kHartreeEv;
  ctx->e_n.ensure(P);
  ctx->eta_n.ensure(P);
  ctx->omega.ensure(n_omega);
  ctx->sig.ensure((size_t)P * n_omega * 2);
  GWL_HIP(hipMemcpy(ctx->e_n.p, en.data(), P * 8, hipMemcpyHostToDevice));
  GWL_HIP(hipMemcpy(ctx->eta_n.p, et.data(), P * 8, hipMemcpyHostToDevice));
  GWL_HIP(hipMemcpy(ctx->omega.p, om.data(), n_omega * 8, hipMemcpyHostToDevice));
  cfrac_sigma(P, ctx->coef_a.p, ctx->coef_b.p, ctx->out_len.p, ctx->norm2.p, ld, ctx->e_n.p,
              ctx->eta_n.p, ctx->omega.p, n_omega, eta_ev / kHartreeEv, ctx->sig.p,
              ctx->stream);
}

}  // namespace

extern "C" {

gwl_status gwl_sigma_c_range(gwl_ctx* ctx, const int* qp_states, int n_qp, int n_begin,
                             int n_end, const double* omega_ev, int n_omega, double eta_ev,
                             int n_lanczos, double* sigma_out) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_qp >= 0 && n_omega >= 0, GWL_EINVAL, "negative count");
    GWL_CHECK(n_begin >= 0 && n_begin < n_end && n_end <= ctx->n_orb, GWL_EINVAL,
              "need 0 <= n_begin < n_end <= n_orb");
    if (n_qp == 0 || n_omega == 0) return;
    GWL_CHECK(qp_states && omega_ev && sigma_out, GWL_EINVAL, "null pointer");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    GWL_CHECK(n_lanczos >= 1 && n_lanczos <= 4000, GWL_EINVAL,
              "n_lanczos must be in [1, 4000]");
    GWL_CHECK(finite_all(omega_ev, n_omega), GWL_EINVAL, "non-finite frequency");
    for (int i = 0; i < n_qp; ++i)
      GWL_CHECK(qp_states[i] >= 0 && qp_states[i] < ctx->n_orb, GWL_EINVAL,
                "qp state out of range");
    auto t0 = std::chrono::steady_clock::now();
    ctx->last_c_matvecs = 0;
    ctx->prof_reset();
    const int per = n_end - n_begin;
    const int P = n_qp * per;
    std::vector<int> m(P), n(P), len(P, n_lanczos);
    for (int q = 0; q < n_qp; ++q)
      for (int j = 0; j < per; ++j) {
        m[(size_t)q * per + j] = qp_states[q];
        n[(size_t)q * per + j] = n_begin + j;
      }
    ctx->run_pairs(P, m.data(), n.data(), len.data(), n_lanczos);
    sigma_device(ctx, P, n.data(), n_lanczos, omega_ev, n_omega, eta_ev);
    ctx->sig_sum.ensure((size_t)n_qp * n_omega * 2);
    sum_groups(ctx->sig.p, n_qp, per, n_omega, ctx->sig_sum.p, ctx->stream);
    GWL_HIP(hipMemcpyAsync(sigma_out, ctx->sig_sum.p, sizeof(double) * n_qp * n_omega * 2,
                           hipMemcpyDeviceToHost, ctx->stream));
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    GWL_CHECK(finite_all(sigma_out, (size_t)n_qp * n_omega * 2), GWL_ENUMERIC,
              "non-finite self-energy");
    ctx->last_ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
}

gwl_status gwl_sigma_c(gwl_ctx* ctx, const int* qp_states, int n_qp, const double* omega_ev,
                       int n_omega, double eta_ev, int n_lanczos, double* sigma_out) {
  if (ctx == nullptr) {
    set_error("null context");
    return GWL_EINVAL;
  }
  return gwl_sigma_c_range(ctx, qp_states, n_qp, 0, ctx->n_orb, omega_ev, n_omega, eta_ev,
                           n_lanczos, sigma_out);
}

gwl_status gwl_sigma_from_coeffs(gwl_ctx* ctx, const int* n_idx, int n_pairs, const double* alpha,
                                 const double* beta, const double* p_norm2, const int* lens,
                                 int ld, const double* omega_ev, int n_omega, double eta_ev,
                                 double* sigma_out) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_pairs >= 0 && n_omega >= 0, GWL_EINVAL, "negative count");
    if (n_pairs == 0 || n_omega == 0) return;
    GWL_CHECK(n_idx && alpha && beta && p_norm2 && lens && omega_ev && sigma_out, GWL_EINVAL,
              "null pointer");
    GWL_CHECK(ld >= 1 && ld <= 4000, GWL_EINVAL, "ld must be in [1, 4000]");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    for (int i = 0; i < n_pairs; ++i) {
      GWL_CHECK(n_idx[i] >= 0 && n_idx[i] < ctx->n_orb, GWL_EINVAL, "orbital out of range");
      GWL_CHECK(lens[i] >= 0 && lens[i] <= ld, GWL_EINVAL, "length out of range");
    }
    ctx->coef_a.ensure((size_t)n_pairs * ld);
    ctx->coef_b.ensure((size_t)n_pairs * ld);
    ctx->norm2.ensure(n_pairs);
    ctx->out_len.ensure(n_pairs);
    GWL_HIP(hipMemcpy(ctx->coef_a.p, alpha, sizeof(double) * n_pairs * ld, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(ctx->coef_b.p, beta, sizeof(double) * n_pairs * ld, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(ctx->norm2.p, p_norm2, sizeof(double) * n_pairs, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(ctx->out_len.p, lens, sizeof(int) * n_pairs, hipMemcpyHostToDevice));
    sigma_device(ctx, n_pairs, n_idx, ld, omega_ev, n_omega, eta_ev);
    GWL_HIP(hipMemcpyAsync(sigma_out, ctx->sig.p, sizeof(double) * n_pairs * n_omega * 2,
                           hipMemcpyDeviceToHost, ctx->stream));
    GWL_HIP(hipStreamSynchronize(ctx->stream));
  });
}

}  // extern "C"
