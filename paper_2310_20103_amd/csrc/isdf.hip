// Interpolative separable density fitting (ISDF) of the pair densities
// (Eqs. 15-17): phi_v phi_c(r) ~ sum_mu zeta_mu(r) C^mu_vc with C^mu_vc =
// phi_v(r_mu) phi_c(r_mu) at caller-given interpolation points, the auxiliary
// functions zeta the least-squares fit zeta = Z C^T (C C^T)^-1, and the
// two-centre integrals M = dV zeta^T V[zeta].  Then K u = C^T M C u, which is
// the library's K product with the grid replaced by the points (the first and
// second GEMMs run on N_mu sampled orbital values) and the FFT Poisson solve
// replaced by the dense product y = (M / dV) rho.  Only the (vc|v'c')
// integrals of K are fitted; the coupling integrals (nm|vc) stay on the grid.
//
// Setup (FP64): Z C^T = (Phi_v Phi_v(pts)^T) o (Phi_c Phi_c(pts)^T) by two
// rocBLAS GEMMs and a Hadamard product (the pair densities are never formed),
// C C^T = its rows at the points, Cholesky (rocSOLVER) and two triangular
// solves for zeta, the FFT Poisson solve of every zeta_mu, and one more GEMM
// for M.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <vector>

#include "context.h"

namespace gwl {
namespace {

#define GWL_BLAS(call)                                                                   \
  do {                                                                                   \
    rocblas_status s_ = (call);                                                          \
    if (s_ != rocblas_status_success)                                                    \
      throw ::gwl::Error{GWL_EDEVICE, std::string(#call) + ": rocblas status " +         \
                                          std::to_string((int)s_)};                      \
  } while (0)

constexpr int NT = 256;

// dst[row][i] = src[row][pts[i]] for i < n_mu, 0 for n_mu <= i < ld_dst.
__global__ void gather_cols_kernel(const double* __restrict__ src, long ld_src,
                                   const int* __restrict__ pts, int n_mu,
                                   double* __restrict__ dst, long ld_dst) {
  const int row = blockIdx.y;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < ld_dst;
       i += (long)gridDim.x * blockDim.x)
    dst[(long)row * ld_dst + i] = i < n_mu ? src[(long)row * ld_src + pts[i]] : 0.0;
}

// dst[i][:] = src[pts[i]][:] (rows of width w), zero rows for n_mu <= i < rows.
__global__ void gather_rows_kernel(const double* __restrict__ src, int w,
                                   const int* __restrict__ pts, int n_mu,
                                   double* __restrict__ dst) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < w; j += gridDim.x * blockDim.x)
    dst[(long)i * w + j] = i < n_mu ? src[(long)pts[i] * w + j] : 0.0;
}

__global__ void hadamard_kernel(double* __restrict__ a, const double* __restrict__ b, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    a[i] *= b[i];
}

// padded symmetric copy: out[i][j] = (m[i][j] + m[j][i]) / 2 for i, j < n, 0 else
__global__ void sym_pad_kernel(const double* __restrict__ m, int n, int ldo,
                               double* __restrict__ out64, float* __restrict__ out32) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ldo; j += gridDim.x * blockDim.x) {
    double v = 0.0;
    if (i < n && j < n) v = 0.5 * (m[(long)i * n + j] + m[(long)j * n + i]);
    out64[(long)i * ldo + j] = v;
    out32[(long)i * ldo + j] = (float)v;
  }
}

int blocks_for(long n) { return (int)std::min<long>(1024, (n + NT - 1) / NT); }

}  // namespace
}  // namespace gwl

using namespace gwl;

// y[b] = (M / dV) sum_vt rho[vt][b] on the points (FP64 or FP32 GEMMs).
void gwl_ctx::middle_step(int nb, int prec, int nvt, const void* rho_in, void* v_out) {
  rocblas_handle h = static_cast<rocblas_handle>(blas);
  GWL_BLAS(rocblas_set_stream(h, stream));
  const int n = (int)gdi.nrp;
  for (int t = 0; t < nvt; ++t) {
    if (prec == GWL_FP64) {
      const double one = 1.0, beta = t == 0 ? 0.0 : 1.0;
      const double* r = static_cast<const double*>(rho_in) + (size_t)t * nb * n;
      GWL_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, nb, n, &one,
                             mmat64.p, n, r, n, &beta, static_cast<double*>(v_out), n));
    } else {
      const float one = 1.0f, beta = t == 0 ? 0.0f : 1.0f;
      const float* r = static_cast<const float*>(rho_in) + (size_t)t * nb * n;
      GWL_BLAS(rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_none, n, nb, n, &one,
                             mmat32.p, n, r, n, &beta, static_cast<float*>(v_out), n));
    }
  }
}

// Switch the K product between the grid and the ISDF points.  The tuned
// block/split choices and the captured graph belong to the other product;
// an estimated interval is estimated again for the new operator.
void gwl_ctx::set_isdf(int on) {
  GWL_CHECK(!on || isdf_ready, GWL_ESTATE, "ISDF is not set up (call gwl_isdf_setup)");
  if (isdf_on == on) return;
  isdf_on = on;
  drop_graph();
  tuned[0] = Tune{};
  tuned[1] = Tune{};
  if (poly_hi_auto) {
    poly_hi = 1.0;
    cheb = cheb_sqrt(poly_lo, poly_hi, poly_degree);
    poly_hi = std::max(estimate_hi(), poly_lo * (1.0 + 1e-6));
    cheb = cheb_sqrt(poly_lo, poly_hi, poly_degree);
  }
}

extern "C" gwl_status gwl_isdf_setup(gwl_ctx* ctx, const int* points, int n_mu) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    gwl_ctx& c = *ctx;
    GWL_CHECK(points != nullptr, GWL_EINVAL, "null pointer");
    GWL_CHECK(n_mu >= 1 && n_mu <= c.nr, GWL_EINVAL, "need 1 <= n_mu <= N_r");
    std::vector<int> pts(points, points + n_mu);
    for (int i = 0; i < n_mu; ++i) {
      GWL_CHECK(pts[i] >= 0 && pts[i] < c.nr, GWL_EINVAL, "point index out of range");
      GWL_CHECK(i == 0 || pts[i] > pts[i - 1], GWL_EINVAL,
                "points must be strictly increasing grid indices");
    }
    hipStream_t st = c.stream;
    if (!c.blas) {
      rocblas_handle h = nullptr;
      GWL_BLAS(rocblas_create_handle(&h));
      c.blas = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(c.blas);
    GWL_BLAS(rocblas_set_stream(h, st));
    c.isdf_on = 0;
    c.isdf_ready = 0;
    c.drop_graph();

    const long nrp = c.gd.nrp;
    const int nvp = c.gd.nvp, ncp = c.gd.ncp;
    GemmDims di = c.gd;
    di.nr = n_mu;
    di.nrp = (int)round_up(n_mu, kPadR);
    const long nrpi = di.nrp;
    c.ipoints.ensure(n_mu);
    GWL_HIP(hipMemcpy(c.ipoints.p, pts.data(), n_mu * sizeof(int), hipMemcpyHostToDevice));

    // sampled orbital layouts (FP64)
    c.ipsi_t.ensure((size_t)(nvp + ncp) * nrpi);
    gather_cols_kernel<<<dim3(blocks_for(nrpi), nvp + ncp), NT, 0, st>>>(
        c.psi_t.p, nrp, c.ipoints.p, n_mu, c.ipsi_t.p, nrpi);
    GWL_HIP(hipGetLastError());
    c.ipsi_c_rc64.ensure((size_t)nrpi * ncp);
    c.ipsi_v_rv64.ensure((size_t)nrpi * nvp);
    gather_rows_kernel<<<dim3(blocks_for(ncp), (unsigned)nrpi), NT, 0, st>>>(
        c.psi_c_rc64.p, ncp, c.ipoints.p, n_mu, c.ipsi_c_rc64.p);
    GWL_HIP(hipGetLastError());
    gather_rows_kernel<<<dim3(blocks_for(nvp), (unsigned)nrpi), NT, 0, st>>>(
        c.psi_v_rv64.p, nvp, c.ipoints.p, n_mu, c.ipsi_v_rv64.p);
    GWL_HIP(hipGetLastError());

    // Z C^T = (Phi_v^T Phi_v(pts)) o (Phi_c^T Phi_c(pts)): column-major [NRp][n_mu]
    DevBuf<double> zc, pc, g, vz;
    zc.ensure((size_t)nrp * n_mu);
    pc.ensure((size_t)nrp * n_mu);
    const double one = 1.0, zero = 0.0;
    GWL_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (int)nrp,
                           n_mu, c.nv, &one, c.psi_t.p, (int)nrp, c.ipsi_t.p, (int)nrpi, &zero,
                           zc.p, (int)nrp));
    GWL_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (int)nrp,
                           n_mu, c.nc, &one, c.psi_t.p + (size_t)nvp * nrp, (int)nrp,
                           c.ipsi_t.p + (size_t)nvp * nrpi, (int)nrpi, &zero, pc.p, (int)nrp));
    hadamard_kernel<<<blocks_for(nrp * n_mu), NT, 0, st>>>(zc.p, pc.p, nrp * (long)n_mu);
    GWL_HIP(hipGetLastError());
    // C C^T = rows of Z C^T at the points (gather along the leading dimension)
    g.ensure((size_t)n_mu * n_mu);
    gather_cols_kernel<<<dim3(blocks_for(n_mu), n_mu), NT, 0, st>>>(zc.p, nrp, c.ipoints.p,
                                                                    n_mu, g.p, n_mu);
    GWL_HIP(hipGetLastError());
    // zeta = (Z C^T) (C C^T)^-1: Cholesky C C^T = L L^T, then two right solves
    DevBuf<int> info;
    info.ensure(1);
    GWL_BLAS(rocsolver_dpotrf(h, rocblas_fill_lower, n_mu, g.p, n_mu, info.p));
    int hinfo = 0;
    GWL_HIP(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
    GWL_HIP(hipStreamSynchronize(st));
    GWL_CHECK(hinfo == 0, GWL_ENUMERIC,
              "C C^T is not positive definite at these points (choose other points)");
    GWL_BLAS(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                           rocblas_diagonal_non_unit, (int)nrp, n_mu, &one, g.p, n_mu, zc.p,
                           (int)nrp));
    GWL_BLAS(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                           rocblas_diagonal_non_unit, (int)nrp, n_mu, &one, g.p, n_mu, zc.p,
                           (int)nrp));
    // V[zeta_mu] for every column (fields of length NRp, chunks of the work capacity)
    vz.ensure((size_t)nrp * n_mu);
    const int chunk = std::max(1, std::min(n_mu, 64));
    c.ensure_work(chunk, 1, false);
    for (int f0 = 0; f0 < n_mu; f0 += chunk) {
      const int cnt = std::min(chunk, n_mu - f0);
      poisson_launch<double>(c.pg64, zc.p + (size_t)f0 * nrp, nrp, 0, 1,
                             vz.p + (size_t)f0 * nrp, nrp, cnt,
                             reinterpret_cast<cplx<double>*>(c.fftx.p), st);
    }
    // M / dV = zeta^T V[zeta] (the combine multiplies by dV)
    DevBuf<double> m;
    m.ensure((size_t)n_mu * n_mu);
    GWL_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n_mu, n_mu,
                           (int)nrp, &one, zc.p, (int)nrp, vz.p, (int)nrp, &zero, m.p, n_mu));
    c.mmat64.ensure((size_t)nrpi * nrpi);
    c.mmat32.ensure((size_t)nrpi * nrpi);
    sym_pad_kernel<<<dim3(blocks_for(nrpi), (unsigned)nrpi), NT, 0, st>>>(
        m.p, n_mu, (int)nrpi, c.mmat64.p, c.mmat32.p);
    GWL_HIP(hipGetLastError());

    // mixed-precision sampled copies (same scale as the grid copies)
    {
      std::vector<double> t((size_t)(nvp + ncp) * nrpi), crc((size_t)nrpi * ncp),
          vrv((size_t)nrpi * nvp);
      GWL_HIP(hipMemcpyAsync(t.data(), c.ipsi_t.p, t.size() * 8, hipMemcpyDeviceToHost, st));
      GWL_HIP(hipMemcpyAsync(crc.data(), c.ipsi_c_rc64.p, crc.size() * 8, hipMemcpyDeviceToHost,
                             st));
      GWL_HIP(hipMemcpyAsync(vrv.data(), c.ipsi_v_rv64.p, vrv.size() * 8, hipMemcpyDeviceToHost,
                             st));
      GWL_HIP(hipStreamSynchronize(st));
      const double os = c.orb16_scale;
      // the second GEMM's sampled orbitals, in rows or K panels (orb16_index)
      std::vector<f16_t> t16((size_t)panel_rows(di) * nrpi, f16_t{0});
      std::vector<f16_t> c16(crc.size()), v16(vrv.size());
      std::vector<float> v32(vrv.size());
      for (size_t i = 0; i < t.size(); ++i) {
        const long row = (long)(i / nrpi), r = (long)(i % nrpi);
        t16[(size_t)orb16_index(di, row, r)] = f32_to_f16((float)(os * t[i]));
      }
      for (size_t i = 0; i < crc.size(); ++i) c16[i] = f32_to_f16((float)(os * crc[i]));
      for (size_t i = 0; i < vrv.size(); ++i) {
        v32[i] = (float)(os * vrv[i]);
        v16[i] = f32_to_f16(v32[i]);
      }
      c.ipsi_t16.ensure(t16.size());
      c.ipsi_c_rc16.ensure(c16.size());
      c.ipsi_v_rv16.ensure(v16.size());
      c.ipsi_v_rv32.ensure(v32.size());
      GWL_HIP(hipMemcpy(c.ipsi_t16.p, t16.data(), t16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.ipsi_c_rc16.p, c16.data(), c16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.ipsi_v_rv16.p, v16.data(), v16.size() * 2, hipMemcpyHostToDevice));
      GWL_HIP(hipMemcpy(c.ipsi_v_rv32.p, v32.data(), v32.size() * 4, hipMemcpyHostToDevice));
    }
    c.gdi = di;
    c.n_mu = n_mu;
    c.isdf_ready = 1;
    c.set_isdf(1);
    GWL_HIP(hipStreamSynchronize(st));
    return GWL_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GWL_ENOMEM;
  }
}
