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

#include <limits>

#include <rocblas/rocblas.h>

#include "context.h"

namespace gwl {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace gwl

using namespace gwl;


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

// The two built precisions; the split-BF16 and FP32 members of gwl_precision
// are named by the ABI but not built.
void check_precision(int p) {
  GWL_CHECK(p != GWL_MIXED_BF16X3 && p != GWL_MIXED_FP32, GWL_EUNSUPPORTED,
            "precision not built: use GWL_FP64 or GWL_MIXED_F16");
  GWL_CHECK(p == GWL_FP64 || p == GWL_MIXED_F16, GWL_EINVAL, "unknown precision");
}

}  // namespace

namespace {

// Largest 2-norm among n_vec device vectors of length N_vc (sets the FP16
// operand scale for caller-given vectors).
double max_row_norm(gwl_ctx* ctx, const double* x, int n_vec) {
  DevBuf<double> nrm;
  nrm.ensure(n_vec);
  row_norm2(x, ctx->nvc, n_vec, nrm.p, ctx->stream);
  std::vector<double> h(n_vec);
  GWL_HIP(hipMemcpyAsync(h.data(), nrm.p, n_vec * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  GWL_HIP(hipStreamSynchronize(ctx->stream));
  double m = 0.0;
  for (double v : h) {
    GWL_CHECK(std::isfinite(v), GWL_EINVAL, "non-finite input vector");
    m = std::max(m, v);
  }
  return m;
}

// Potentials of the caller into the padded [nb][N_rp] rows of the FP64 product
// (pads zero).
__global__ void pot_pad_kernel(const double* __restrict__ v, long nr, long nrp,
                               double* __restrict__ out) {
  const int b = blockIdx.y;
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < nrp; r += (long)gridDim.x * blockDim.x)
    out[b * nrp + r] = r < nr ? v[b * nr + r] : 0.0;
}

// Mixed product: the power of two of each potential (from its largest |V|, as
// the Poisson solve chooses it) and the FP16 rows V 2^e (pads zero).  One
// block per potential for the maximum (fixed order).
__global__ void pot16_exp_kernel(const double* __restrict__ v, long nr, int pexp,
                                 int* __restrict__ vexp) {
  __shared__ float sh[256];
  const int b = blockIdx.x;
  float m = 0.0f;
  for (long r = threadIdx.x; r < nr; r += blockDim.x) m = fmaxf(m, (float)fabs(v[b * nr + r]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) vexp[b] = f16_operand_exp(sh[0], pexp);
}
__global__ void pot16_kernel(const double* __restrict__ v, long nr, long nrp,
                             const int* __restrict__ vexp, f16_t* __restrict__ out) {
  const int b = blockIdx.y;
  const float sc = ldexpf(1.0f, vexp[b]);
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < nrp; r += (long)gridDim.x * blockDim.x)
    out[b * nrp + r] = f32_to_f16(r < nr ? (float)v[b * nr + r] * sc : 0.0f);
}

// y[b][vc] = scale 2^-vexp[b] sum_s ypart[s][b][v][c] (vexp optional).
template <typename Y>
__global__ void potprod_finish_kernel(int nv, int nc, int nvp, int ncp, int nb, int splitk,
                                      const Y* __restrict__ ypart, const int* __restrict__ vexp,
                                      double scale, double* __restrict__ y) {
  const int b = blockIdx.y;
  const long nvc = (long)nv * nc, stride_s = (long)nb * nvp * ncp;
  const double sc = vexp ? ldexp(scale, -vexp[b]) : scale;
  const Y* yb = ypart + (long)b * nvp * ncp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nvc; e += (long)gridDim.x * blockDim.x) {
    const int v = (int)(e / nc), c = (int)(e - (long)v * nc);
    double t = 0.0;
    for (int s = 0; s < splitk; ++s) t += (double)yb[s * stride_s + (long)v * ncp + c];
    y[b * nvc + e] = sc * t;
  }
}

// out[b][r] = inv_scale * sum_t part[t][b][r] for r < N_r (partial densities
// of the first GEMM's v tiles, in its working precision).
template <typename T>
__global__ void density_out_kernel(const T* __restrict__ part, int nvt, long tstride, long nrp,
                                   long nr, double inv_scale, double* __restrict__ out) {
  const int b = blockIdx.y;
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < nr; r += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < nvt; ++t) s += (double)part[t * tstride + b * nrp + r];
    out[b * nr + r] = inv_scale * s;
  }
}

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
    GWL_CHECK((long)n_occ * (n_orb - n_occ) < (1L << 31), GWL_EUNSUPPORTED,
              "the pair dimension N_v N_c must be below 2^31");
    GWL_CHECK(grid->nx >= 2 && grid->ny >= 2 && grid->nz >= 2 && grid->nx <= 256 &&
                  grid->ny <= 256 && grid->nz <= 256,
              GWL_EUNSUPPORTED, "grid edges must be in [2, 256]");
    GWL_CHECK(grid->lx > 0 && grid->ly > 0 && grid->lz > 0 && std::isfinite(grid->lx) &&
                  std::isfinite(grid->ly) && std::isfinite(grid->lz),
              GWL_EINVAL, "box edges must be positive");
    gwl_options o;
    gwl_default_options(&o);
    if (opts) o = *opts;
    check_precision(o.precision);
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
    poisson_prepare_device();
    noalloc_bind_current_device();
    if (o.stream) {
      c.stream = (hipStream_t)o.stream;
    } else {
      GWL_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
      c.own_stream = true;
    }
    // a setup that fails after this point destroys the stream it created
    struct StreamGuard {
      std::unique_ptr<gwl_ctx>& ctx;
      ~StreamGuard() {
        if (ctx && ctx->own_stream) {
          (void)hipStreamSynchronize(ctx->stream);
          (void)hipStreamDestroy(ctx->stream);
        }
      }
    } stream_guard{ctx};
    c.nx = grid->nx;
    c.ny = grid->ny;
    c.nz = grid->nz;
    c.lx = grid->lx;
    c.ly = grid->ly;
    c.lz = grid->lz;
    c.nr = (long)c.nx * c.ny * c.nz;
    c.n_orb = n_orb;
    c.orb_dtype = orb_dtype;
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
    std::vector<double> d1(c.nvc), d2(c.nvc), sd(c.nvc);
    double dmin = 1e300;
    for (int v = 0; v < c.nv; ++v)
      for (int cc = 0; cc < c.nc; ++cc) {
        const double d = c.eps_ha[c.nv + cc] - c.eps_ha[v];
        d1[(size_t)v * c.nc + cc] = d;
        d2[(size_t)v * c.nc + cc] = d * d;
        sd[(size_t)v * c.nc + cc] = std::sqrt(d);
        dmin = std::min(dmin, d);
      }
    c.sd_max = 0.0;
    for (double v : sd) c.sd_max = std::max(c.sd_max, v);
    c.delta1.ensure(c.nvc);
    c.delta2.ensure(c.nvc);
    c.sdelta.ensure(c.nvc);
    GWL_HIP(hipMemcpy(c.delta1.p, d1.data(), c.nvc * 8, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(c.delta2.p, d2.data(), c.nvc * 8, hipMemcpyHostToDevice));
    GWL_HIP(hipMemcpy(c.sdelta.p, sd.data(), c.nvc * 8, hipMemcpyHostToDevice));

    // orbitals -> the kernels' layouts, packed on the GPU from one upload
    const long nrp = c.gd.nrp;
    const int nvp = c.gd.nvp, ncp = c.gd.ncp;
    {
      DevBuf<unsigned char> raw;
      const void* src = orbitals;
      if (!orb_on_device) {
        const size_t bytes = (size_t)n_orb * c.nr * orb_dtype;
        raw.ensure(bytes);
        GWL_HIP(hipMemcpy(raw.p, orbitals, bytes, hipMemcpyHostToDevice));
        src = raw.p;
      }
      DevBuf<unsigned long long> flags;  // [0] non-finite seen, [1] max |phi|, [2] max |f16 phi_v|
      flags.ensure(3);
      c.psi_t.ensure((size_t)(nvp + ncp) * nrp);
      c.psi_c_rc64.ensure((size_t)nrp * ncp);
      c.psi_v_rv64.ensure((size_t)nrp * nvp);
      pack_orbitals64(c.gd, src, orb_dtype, n_orb, c.nr, c.psi_t.p, c.psi_c_rc64.p,
                      c.psi_v_rv64.p, reinterpret_cast<int*>(flags.p), flags.p + 1, c.stream);
      unsigned long long h[3];
      GWL_HIP(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
      GWL_HIP(hipStreamSynchronize(c.stream));
      raw.release();
      GWL_CHECK((unsigned)h[0] == 0, GWL_EINVAL, "non-finite orbital value");
      // mixed-precision copies in FP16 (both GEMMs' orbital operands and the
      // first GEMM's row-dot weights), scaled by a power of two that puts the
      // largest orbital value near 2^11
      double omax;
      std::memcpy(&omax, &h[1], 8);
      {
        int e = omax > 0.0 ? (int)std::floor(std::log2(2048.0 / omax)) : 0;
        e = std::max(-60, std::min(60, e));
        c.orb16_scale = std::ldexp(1.0, e);
      }
      // the second GEMM's orbitals in rows or K panels (orb16_index)
      c.psi_t16.ensure((size_t)panel_rows(c.gd) * nrp);
      c.psi_c_rc16.ensure((size_t)nrp * ncp);
      c.psi_v_rv32.ensure((size_t)nrp * nvp);
      c.psi_v_rv16.ensure((size_t)nrp * nvp);
      pack_orbitals16(c.gd, c.psi_t.p, c.psi_c_rc64.p, c.psi_v_rv64.p, c.orb16_scale,
                      c.psi_t16.p, c.psi_c_rc16.p, c.psi_v_rv32.p, c.psi_v_rv16.p, flags.p + 2,
                      c.stream);
      GWL_HIP(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
      GWL_HIP(hipStreamSynchronize(c.stream));
      float pvmax;
      const unsigned pvb = (unsigned)h[2];
      std::memcpy(&pvmax, &pvb, 4);
      c.pv16_exp = 0;
      if (pvmax > 0.0f) (void)std::frexp(pvmax, &c.pv16_exp);
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
    c.poly_hi_auto = !(o.poly_hi > 0);
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
  if (ctx->blas) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(ctx->blas));
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

gwl_status gwl_set_option(gwl_ctx* ctx, int key, double value) {
  return guarded([&] {
    check_ctx(ctx);
    switch (key) {
      case GWL_KEY_PRECISION:
        check_precision((int)value);
        GWL_CHECK(value == (int)value, GWL_EINVAL, "bad precision");
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
      case GWL_KEY_TDA:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "tda must be 0 or 1");
        ctx->tda = (int)value;
        break;
      case GWL_KEY_QUADRATURE:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "quadrature must be 0 or 1");
        ctx->quadrature = (int)value;
        break;
      case GWL_KEY_ADJOINT_STORE:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "adjoint_store must be 0 or 1");
        ctx->adjoint_store = (int)value;
        break;
      case GWL_KEY_ISDF:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "isdf must be 0 or 1");
        ctx->set_isdf((int)value);
        break;
      case GWL_KEY_BF16_TILE:
        GWL_CHECK(value == 128 || value == 256, GWL_EINVAL, "BF16 tile must be 128 or 256");
        if (ctx->bf16_tile != (int)value || !ctx->tile_fixed) {
          ctx->bf16_tile = (int)value;
          ctx->tile_fixed = true;
          ctx->tuned[GWL_MIXED_F16] = gwl_ctx::Tune{};
          ctx->drop_graph();
        }
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
      case GWL_KEY_SCHEDULER:
        GWL_CHECK(value == 0 || value == 1, GWL_EINVAL, "scheduler must be 0 or 1");
        ctx->sched_tables = (int)value;
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
      case GWL_KEY_BF16_TILE: *out = ctx->bf16_tile; break;
      case GWL_KEY_TDA: *out = ctx->tda; break;
      case GWL_KEY_QUADRATURE: *out = ctx->quadrature; break;
      case GWL_KEY_ADJOINT_STORE: *out = ctx->adjoint_store; break;
      case GWL_KEY_ADJOINT_STORED: *out = ctx->adjoint_stored; break;
      case GWL_KEY_HI_RESIDUAL: *out = ctx->hi_resid; break;
      case GWL_KEY_ISDF: *out = ctx->isdf_on; break;
      case GWL_KEY_ISDF_NMU: *out = ctx->isdf_ready ? ctx->n_mu : 0; break;
      case GWL_KEY_PROFILE: *out = ctx->profile; break;
      case GWL_KEY_GRAPHS: *out = ctx->use_graphs; break;
      case GWL_KEY_SCHEDULER: *out = ctx->sched_tables; break;
      case GWL_KEY_TUNED_BLOCK: *out = ctx->tuned[ctx->precision].B; break;
      case GWL_KEY_TUNED_SPLITK: *out = ctx->tuned[ctx->precision].S; break;
      case GWL_KEY_TUNED_TILE: *out = ctx->tuned[ctx->precision].tile; break;
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
    check_precision(precision);
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
    check_precision(precision);
    ctx->prof_reset();
    const int chunk = std::min(n_vec, 64);
    ctx->ensure_work(chunk, 1, false);
    if (precision != GWL_FP64) ctx->set_u_bound(max_row_norm(ctx, x, n_vec));
    for (int i0 = 0; i0 < n_vec; i0 += chunk) {
      const int nb = std::min(chunk, n_vec - i0);
      ctx->apply_c_batch(nb, x + (size_t)i0 * ctx->nvc, y + (size_t)i0 * ctx->nvc, precision);
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof_flush();
  });
}

gwl_status gwl_pair_density(gwl_ctx* ctx, const double* x, double* rho, int n_vec,
                            int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_vec >= 0, GWL_EINVAL, "n_vec < 0");
    if (n_vec == 0) return;
    GWL_CHECK(x && rho, GWL_EINVAL, "null pointer");
    check_precision(precision);
    GWL_CHECK(!ctx->isdf_on, GWL_EUNSUPPORTED,
              "pair densities live on the grid: switch the ISDF product off");
    ctx->prof_reset();
    const int chunk = std::min(n_vec, 128);
    ctx->ensure_work(chunk, 1, false);
    if (precision != GWL_FP64) ctx->set_u_bound(max_row_norm(ctx, x, n_vec));
    const GemmDims& d = ctx->gd;
    for (int i0 = 0; i0 < n_vec; i0 += chunk) {
      const int nb = std::min(chunk, n_vec - i0);
      ctx->cast(nb, x + (size_t)i0 * ctx->nvc, precision);
      const int nvt = ctx->first_gemm(nb, precision);
      dim3 grid((unsigned)std::min<long>(1024, (ctx->nr + 255) / 256), (unsigned)nb);
      double* out = rho + (size_t)i0 * ctx->nr;
      if (precision == GWL_FP64) {
        density_out_kernel<double><<<grid, 256, 0, ctx->stream>>>(
            reinterpret_cast<const double*>(ctx->rho.p), nvt, (long)nb * d.nrp, d.nrp, ctx->nr,
            1.0, out);
      } else {
        const double os = ctx->orb16_scale;
        density_out_kernel<float><<<grid, 256, 0, ctx->stream>>>(
            reinterpret_cast<const float*>(ctx->rho.p), nvt, (long)nb * d.nrp, d.nrp, ctx->nr,
            1.0 / (ctx->u_scale * os * os), out);
      }
      GWL_HIP(hipGetLastError());
    }
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof_flush();
  });
}

gwl_status gwl_potential_product(gwl_ctx* ctx, const double* v, double* y, int n_vec,
                                 int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_vec >= 0, GWL_EINVAL, "n_vec < 0");
    if (n_vec == 0) return;
    GWL_CHECK(v && y, GWL_EINVAL, "null pointer");
    check_precision(precision);
    GWL_CHECK(!ctx->isdf_on, GWL_EUNSUPPORTED,
              "potentials live on the grid: switch the ISDF product off");
    gwl_ctx& c = *ctx;
    c.prof_reset();
    const int chunk = std::min(n_vec, 128);
    c.ensure_work(chunk, 1, false);
    const GemmDims& d = c.gd;
    hipStream_t st = c.stream;
    for (int i0 = 0; i0 < n_vec; i0 += chunk) {
      const int nb = std::min(chunk, n_vec - i0);
      const double* vb = v + (size_t)i0 * c.nr;
      double* yb = y + (size_t)i0 * c.nvc;
      const int S = c.auto_splitk(nb, precision);
      dim3 gr((unsigned)std::min<long>(1024, (d.nrp + 255) / 256), (unsigned)nb);
      dim3 gy((unsigned)std::min<long>(1024, (c.nvc + 255) / 256), (unsigned)nb);
      c.prof_begin();
      if (precision == GWL_FP64) {
        pot_pad_kernel<<<gr, 256, 0, st>>>(vb, c.nr, d.nrp, c.vpot64.p);
        const double* pv = c.psi_t.p;
        const double* pc = c.psi_t.p + (size_t)d.nvp * d.nrp;
        double* yp = reinterpret_cast<double*>(c.ypart.p);
        if (c.fp64_kernel)
          gemm2_f64m(d, nb, S, pv, pc, c.vpot64.p, yp, st);
        else
          gemm2_f64(d, nb, S, pv, pc, c.vpot64.p, yp, st);
        potprod_finish_kernel<double><<<gy, 256, 0, st>>>(c.nv, c.nc, d.nvp, d.ncp, nb, S, yp,
                                                          nullptr, c.dv, yb);
      } else {
        pot16_exp_kernel<<<nb, 256, 0, st>>>(vb, c.nr, c.pv16_exp, c.vexp32.p);
        pot16_kernel<<<gr, 256, 0, st>>>(vb, c.nr, d.nrp, c.vexp32.p, c.vpot16.p);
        const f16_t* pt = c.psi_t16.p;
        const f16_t* pc = pt + orb16_index(d, d.nvp, 0);
        float* yp = reinterpret_cast<float*>(c.ypart.p);
        if (c.fp64_kernel)
          gemm2_f16(d, nb, c.bf16_tile, S, pt, pc, c.vpot16.p, yp, st);
        else
          gemm2_f16s(d, nb, S, pt, pc, c.vpot16.p, yp, st);
        const double os = c.orb16_scale;
        potprod_finish_kernel<float><<<gy, 256, 0, st>>>(c.nv, c.nc, d.nvp, d.ncp, nb, S, yp,
                                                         c.vexp32.p, c.dv / (os * os), yb);
      }
      c.prof_end(1, nb);
      GWL_HIP(hipGetLastError());
    }
    GWL_HIP(hipStreamSynchronize(st));
    c.prof_flush();
  });
}

gwl_status gwl_apply_d(gwl_ctx* ctx, const double* x, double* y, int n_vec, int precision) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_vec >= 0, GWL_EINVAL, "n_vec < 0");
    if (n_vec == 0) return;
    GWL_CHECK(x && y, GWL_EINVAL, "null pointer");
    check_precision(precision);
    ctx->prof_reset();
    const int chunk = std::min(n_vec, 64);
    ctx->ensure_work(chunk, 1, false);
    if (precision != GWL_FP64) ctx->set_u_bound(max_row_norm(ctx, x, n_vec));
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

gwl_status gwl_sigma_x(gwl_ctx* ctx, const int* qp_states, int n_qp, double* sigma_x_out) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_qp >= 0, GWL_EINVAL, "n_qp < 0");
    if (n_qp == 0) return;
    GWL_CHECK(qp_states && sigma_x_out, GWL_EINVAL, "null pointer");
    for (int i = 0; i < n_qp; ++i)
      GWL_CHECK(qp_states[i] >= 0 && qp_states[i] < ctx->n_orb, GWL_EINVAL,
                "qp state out of range");
    gwl_ctx& c = *ctx;
    const int nv = c.nv;
    const int chunk = std::min(nv, 64);
    c.ensure_work(chunk, 1, false);
    DevBuf<double> e;
    e.ensure((size_t)nv);
    std::vector<int> mr(chunk), vr(chunk);
    std::vector<double> he(nv);
    double* rp = reinterpret_cast<double*>(c.rho.p);
    for (int q = 0; q < n_qp; ++q) {
      for (int v0 = 0; v0 < nv; v0 += chunk) {
        const int cnt = std::min(chunk, nv - v0);
        for (int i = 0; i < cnt; ++i) {
          mr[i] = c.orb_row(qp_states[q]);
          vr[i] = c.orb_row(v0 + i);
        }
        GWL_HIP(hipStreamSynchronize(c.stream));
        GWL_HIP(hipMemcpy(c.s_m.p, mr.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
        GWL_HIP(hipMemcpy(c.s_n.p, vr.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
        pair_product(c.psi_t.p, c.gd.nrp, (int)c.nr, c.s_m.p, c.s_n.p, cnt, rp, c.stream);
        poisson_launch<double>(c.pg64, rp, c.gd.nrp, 0, 1, c.vpot64.p, c.gd.nrp, cnt,
                               reinterpret_cast<cplx<double>*>(c.fftx.p), c.stream);
        pair_energy(rp, c.vpot64.p, c.gd.nrp, (int)c.nr, c.dv, cnt, e.p + v0, c.stream);
      }
      GWL_HIP(hipMemcpyAsync(he.data(), e.p, nv * sizeof(double), hipMemcpyDeviceToHost,
                             c.stream));
      GWL_HIP(hipStreamSynchronize(c.stream));
      double sx = 0.0;
      for (int v = 0; v < nv; ++v) sx -= he[v];
      sigma_x_out[q] = sx * kHartreeEv;
    }
    GWL_CHECK(finite_all(sigma_x_out, n_qp), GWL_ENUMERIC, "non-finite exchange self-energy");
  });
}

gwl_status gwl_qp_solve(const double* omega_ev, int n_omega, const double* sigma_c,
                        double eps_ev, double sigma_x_ev, double vxc_ev, double* e_qp,
                        double* z) {
  return guarded([&] {
    GWL_CHECK(omega_ev && sigma_c && e_qp && z, GWL_EINVAL, "null pointer");
    GWL_CHECK(n_omega >= 2, GWL_EINVAL, "need at least two frequencies");
    for (int i = 0; i + 1 < n_omega; ++i)
      GWL_CHECK(omega_ev[i + 1] > omega_ev[i], GWL_EINVAL, "frequencies must increase");
    *e_qp = std::numeric_limits<double>::quiet_NaN();
    *z = std::numeric_limits<double>::quiet_NaN();
    // f(w) = e + Sigma^x + Re Sigma^c(w) - v_xc - w; roots by sign change and
    // linear interpolation, the one nearest e wins
    auto f = [&](int i) { return eps_ev + sigma_x_ev + sigma_c[2 * i] - vxc_ev - omega_ev[i]; };
    int best_seg = -1;
    double best = 0.0;
    for (int i = 0; i + 1 < n_omega; ++i) {
      const double f0 = f(i), f1 = f(i + 1);
      double root;
      if (f0 == 0.0)
        root = omega_ev[i];
      else if ((f0 < 0.0) != (f1 < 0.0) && f1 != 0.0)
        root = omega_ev[i] - f0 * (omega_ev[i + 1] - omega_ev[i]) / (f1 - f0);
      else
        continue;
      if (best_seg < 0 || std::fabs(root - eps_ev) < std::fabs(best - eps_ev)) {
        best = root;
        best_seg = i;
      }
    }
    GWL_CHECK(best_seg >= 0, GWL_ENUMERIC, "the quasiparticle equation has no root on the grid");
    const double slope = (sigma_c[2 * (best_seg + 1)] - sigma_c[2 * best_seg]) /
                         (omega_ev[best_seg + 1] - omega_ev[best_seg]);
    *e_qp = best;
    *z = 1.0 / (1.0 - slope);
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
    GWL_CHECK(!ctx->lanczos_on_c() || ctx->precision == GWL_FP64, GWL_EUNSUPPORTED,
              "the quadrature variant runs in FP64 only");
    ctx->run_pairs(n_pairs, m_idx, n_idx, lengths, lmax, ctx->lanczos_on_c());
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
  if (ctx->lanczos_on_c()) {
    ctx->qd.ensure((size_t)P * ld);
    ctx->qe.ensure((size_t)P * ld);
    ctx->qz.ensure((size_t)P * ld);
    ctx->qstat.ensure(P);
    quad_sigma(P, ctx->coef_a.p, ctx->coef_b.p, ctx->out_len.p, ctx->norm2.p, ld, ctx->e_n.p,
               ctx->eta_n.p, ctx->omega.p, n_omega, eta_ev / kHartreeEv, ctx->qd.p, ctx->qe.p,
               ctx->qz.p, ctx->qstat.p, ctx->sig.p, ctx->stream);
    std::vector<int> st(P);
    GWL_HIP(hipMemcpyAsync(st.data(), ctx->qstat.p, P * sizeof(int), hipMemcpyDeviceToHost,
                           ctx->stream));
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < P; ++i)
      GWL_CHECK(st[i] == 0, GWL_ENUMERIC, "tridiagonal eigenvalue iteration did not converge");
  } else {
    cfrac_sigma(P, ctx->coef_a.p, ctx->coef_b.p, ctx->out_len.p, ctx->norm2.p, ld, ctx->e_n.p,
                ctx->eta_n.p, ctx->omega.p, n_omega, eta_ev / kHartreeEv, ctx->tda, ctx->sig.p,
                ctx->stream);
  }
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
    GWL_CHECK(!ctx->lanczos_on_c() || ctx->precision == GWL_FP64, GWL_EUNSUPPORTED,
              "the quadrature variant runs in FP64 only");
    ctx->run_pairs(P, m.data(), n.data(), len.data(), n_lanczos, ctx->lanczos_on_c());
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

gwl_status gwl_sigma_c_offdiag(gwl_ctx* ctx, int m, int m2, const double* omega_ev, int n_omega,
                               double eta_ev, int n_lanczos, double* sigma_out) {
  return guarded([&] {
    check_ctx(ctx);
    GWL_CHECK(n_omega >= 0, GWL_EINVAL, "negative count");
    if (n_omega == 0) return;
    GWL_CHECK(omega_ev && sigma_out, GWL_EINVAL, "null pointer");
    GWL_CHECK(m >= 0 && m < ctx->n_orb && m2 >= 0 && m2 < ctx->n_orb, GWL_EINVAL,
              "qp state out of range");
    GWL_CHECK(std::isfinite(eta_ev) && eta_ev > 0, GWL_EINVAL, "eta must be > 0");
    GWL_CHECK(n_lanczos >= 1 && n_lanczos <= 4000, GWL_EINVAL,
              "n_lanczos must be in [1, 4000]");
    GWL_CHECK(finite_all(omega_ev, n_omega), GWL_EINVAL, "non-finite frequency");
    GWL_CHECK(!ctx->lanczos_on_c() || ctx->precision == GWL_FP64, GWL_EUNSUPPORTED,
              "the quadrature variant runs in FP64 only");
    auto t0 = std::chrono::steady_clock::now();
    ctx->last_c_matvecs = 0;
    ctx->prof_reset();
    const int no = ctx->n_orb;
    const long nvc = ctx->nvc;
    // start vectors: rows 2n, 2n + 1 = P_nm + P_nm2, P_nm - P_nm2
    DevBuf<double> start, pa, pb;
    start.ensure((size_t)2 * no * nvc);
    const int chunk = std::min(no, 64);
    pa.ensure((size_t)chunk * nvc);
    pb.ensure((size_t)chunk * nvc);
    std::vector<int> mv(chunk, m), m2v(chunk, m2), nv(chunk);
    for (int n0 = 0; n0 < no; n0 += chunk) {
      const int cnt = std::min(chunk, no - n0);
      for (int i = 0; i < cnt; ++i) nv[i] = n0 + i;
      ctx->coupling_batch(cnt, mv.data(), nv.data(), pa.p, nvc);
      ctx->coupling_batch(cnt, m2v.data(), nv.data(), pb.p, nvc);
      polar_rows(pa.p, pb.p, nvc, cnt, start.p + (size_t)2 * n0 * nvc, ctx->stream);
    }
    const int P = 2 * no;
    std::vector<int> pm(P, m), pn(P), len(P, n_lanczos);
    for (int i = 0; i < P; ++i) pn[i] = i / 2;
    ctx->run_pairs(P, pm.data(), pn.data(), len.data(), n_lanczos, ctx->lanczos_on_c(),
                   start.p);
    sigma_device(ctx, P, pn.data(), n_lanczos, omega_ev, n_omega, eta_ev);
    ctx->sig_sum.ensure((size_t)n_omega * 2);
    sum_polar(ctx->sig.p, no, n_omega, ctx->sig_sum.p, ctx->stream);
    GWL_HIP(hipMemcpyAsync(sigma_out, ctx->sig_sum.p, sizeof(double) * n_omega * 2,
                           hipMemcpyDeviceToHost, ctx->stream));
    GWL_HIP(hipStreamSynchronize(ctx->stream));
    GWL_CHECK(finite_all(sigma_out, (size_t)n_omega * 2), GWL_ENUMERIC,
              "non-finite self-energy");
    ctx->last_ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  });
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
