// ISDF interpolation points by column-pivoted QR of a sketch of the pair
// densities (gwl_isdf_qrcp).
//
// The pair-density matrix Z[(vc), r] = phi_v(r) phi_c(r) (the matrix ISDF
// interpolates, Eqs. 15-17) has N_v N_c rows; it is sketched with caller-given
// random factors Gv [N_v][p], Gc [N_c][p]:
//   S[r][k] = (sum_v Gv[v][k] phi_v(r)) (sum_c Gc[c][k] phi_c(r)),
// whose column space (over r) follows Z's.  Column-pivoted Gram-Schmidt on S
// then takes, n_mu times, the grid point with the largest residual norm
// (ties to the lower index), normalises its column and projects it out of
// every other column.  Everything stays on the device; the pivot of a step
// goes from the arg-max kernel to the update kernel through device memory,
// so the loop has no host round trip.  Reductions run in a fixed order, so
// the points are reproducible bit for bit.
#include "context.h"

namespace gwl {
namespace {

constexpr int QT = 256;
constexpr int QK = 8;  // sketch columns per block of the sketch kernel

// S[r][k] for 256 grid points and QK columns per block; the factors' columns
// are staged in LDS.
__global__ void __launch_bounds__(QT)
qr_sketch_kernel(const double* __restrict__ psi_t, long ld, long nr, int nv, int nvp, int nc,
                 const double* __restrict__ gv, const double* __restrict__ gc, int p,
                 double* __restrict__ S) {
  extern __shared__ double gsh[];  // [nv + nc][QK]
  const int k0 = blockIdx.y * QK;
  const int nk = min(QK, p - k0);
  for (int i = threadIdx.x; i < (nv + nc) * QK; i += QT) {
    const int o = i / QK, kk = i - o * QK;
    double g = 0.0;
    if (kk < nk) g = o < nv ? gv[(long)o * p + k0 + kk] : gc[(long)(o - nv) * p + k0 + kk];
    gsh[i] = g;
  }
  __syncthreads();
  const long r = (long)blockIdx.x * QT + threadIdx.x;
  if (r >= nr) return;
  double av[QK], ac[QK];
#pragma unroll
  for (int kk = 0; kk < QK; ++kk) av[kk] = ac[kk] = 0.0;
  for (int v = 0; v < nv; ++v) {
    const double x = psi_t[(long)v * ld + r];
#pragma unroll
    for (int kk = 0; kk < QK; ++kk) av[kk] += x * gsh[v * QK + kk];
  }
  for (int c = 0; c < nc; ++c) {
    const double x = psi_t[(long)(nvp + c) * ld + r];
#pragma unroll
    for (int kk = 0; kk < QK; ++kk) ac[kk] += x * gsh[(nv + c) * QK + kk];
  }
  for (int kk = 0; kk < nk; ++kk) S[r * p + k0 + kk] = av[kk] * ac[kk];
}

__device__ inline double wave_sum_q(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// nrm[r] = |S[r]|^2, one wave per row, lanes over k in a fixed order.
__global__ void __launch_bounds__(QT)
qr_norms_kernel(const double* __restrict__ S, long nr, int p, double* __restrict__ nrm) {
  const long r = (long)blockIdx.x * (QT / 64) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (r >= nr) return;
  double s = 0.0;
  for (int k = l; k < p; k += 64) s += S[r * p + k] * S[r * p + k];
  s = wave_sum_q(s);
  if (l == 0) nrm[r] = s;
}

// (value, index) maximum with ties to the lower index
__device__ inline void better(double& bv, long& bi, double v, long i) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

// Per-block maximum of nrm over the rows not taken yet.
__global__ void __launch_bounds__(QT)
qr_argmax_part_kernel(const double* __restrict__ nrm, const int* __restrict__ taken, long nr,
                      double* __restrict__ pv, long* __restrict__ pi) {
  __shared__ double sv[QT];
  __shared__ long si[QT];
  double bv = -1.0;
  long bi = nr;
  for (long r = (long)blockIdx.x * QT + threadIdx.x; r < nr; r += (long)gridDim.x * QT)
    if (!taken[r]) better(bv, bi, nrm[r], r);
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = QT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double v = sv[threadIdx.x];
      long i = si[threadIdx.x];
      better(v, i, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = v;
      si[threadIdx.x] = i;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

// Final maximum over the block partials; records the pivot of this step,
// marks it taken and forms q = S[j] / |S[j]| (q = 0 when the residual is zero).
__global__ void __launch_bounds__(QT)
qr_pivot_kernel(const double* __restrict__ pv, const long* __restrict__ pi, int nparts,
                const double* __restrict__ S, int p, int step, int* __restrict__ taken,
                int* __restrict__ piv, long* __restrict__ jcur, double* __restrict__ q) {
  __shared__ double sv[QT];
  __shared__ long si[QT];
  double bv = -1.0;
  long bi = 0x7fffffffffffffffL;
  for (int i = threadIdx.x; i < nparts; i += QT) better(bv, bi, pv[i], pi[i]);
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = QT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double v = sv[threadIdx.x];
      long i = si[threadIdx.x];
      better(v, i, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = v;
      si[threadIdx.x] = i;
    }
    __syncthreads();
  }
  const long j = si[0];
  const double n2 = sv[0];
  const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  for (int k = threadIdx.x; k < p; k += QT) q[k] = S[j * p + k] * inv;
  if (threadIdx.x == 0) {
    piv[step] = (int)j;
    taken[j] = 1;
    *jcur = j;
  }
}

// Project q out of every row not taken: S[r] -= (q . S[r]) q; nrm[r] = |S[r]|^2.
__global__ void __launch_bounds__(QT)
qr_update_kernel(double* __restrict__ S, long nr, int p, const double* __restrict__ q,
                 const int* __restrict__ taken, double* __restrict__ nrm) {
  extern __shared__ double qs[];
  for (int k = threadIdx.x; k < p; k += QT) qs[k] = q[k];
  __syncthreads();
  const long r = (long)blockIdx.x * (QT / 64) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (r >= nr || taken[r]) return;
  double* row = S + r * p;
  double c = 0.0;
  for (int k = l; k < p; k += 64) c += qs[k] * row[k];
  c = wave_sum_q(c);
  double s = 0.0;
  for (int k = l; k < p; k += 64) {
    const double x = row[k] - c * qs[k];
    row[k] = x;
    s += x * x;
  }
  s = wave_sum_q(s);
  if (l == 0) nrm[r] = s;
}

}  // namespace
}  // namespace gwl

using namespace gwl;

extern "C" gwl_status gwl_isdf_qrcp(gwl_ctx* ctx, const double* gv, const double* gc, int p,
                                    int n_mu, int* points_out) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    gwl_ctx& c = *ctx;
    GWL_CHECK(gv && gc && points_out, GWL_EINVAL, "null pointer");
    GWL_CHECK(p >= 1 && n_mu >= 1 && n_mu <= p && (long)n_mu <= c.nr, GWL_EINVAL,
              "need 1 <= n_mu <= p and n_mu <= N_r");
    GWL_CHECK(finite_all(gv, (size_t)c.nv * p) && finite_all(gc, (size_t)c.nc * p), GWL_EINVAL,
              "non-finite sketch factor");
    const long nr = c.nr;
    GWL_CHECK((double)nr * p * 8 <= 64e9, GWL_EUNSUPPORTED, "sketch larger than 64 GB");
    GWL_CHECK((size_t)(c.nv + c.nc) * QK * 8 <= 64 * 1024 && (size_t)p * 8 <= 64 * 1024,
              GWL_EUNSUPPORTED, "too many orbitals or sketch columns for the LDS staging");
    hipStream_t st = c.stream;
    DevBuf<double> dgv, dgc, S, nrm, q, pv;
    DevBuf<long> pi, jcur;
    DevBuf<int> taken, piv;
    dgv.ensure((size_t)c.nv * p);
    dgc.ensure((size_t)c.nc * p);
    S.ensure((size_t)nr * p);
    nrm.ensure(nr);
    q.ensure(p);
    taken.ensure(nr);
    piv.ensure(n_mu);
    jcur.ensure(1);
    const int nparts = (int)std::min<long>(1024, (nr + QT - 1) / QT);
    pv.ensure(nparts);
    pi.ensure(nparts);
    GWL_HIP(hipMemcpyAsync(dgv.p, gv, sizeof(double) * c.nv * p, hipMemcpyHostToDevice, st));
    GWL_HIP(hipMemcpyAsync(dgc.p, gc, sizeof(double) * c.nc * p, hipMemcpyHostToDevice, st));
    dim3 gs((unsigned)((nr + QT - 1) / QT), (unsigned)((p + QK - 1) / QK));
    qr_sketch_kernel<<<gs, QT, (size_t)(c.nv + c.nc) * QK * 8, st>>>(
        c.psi_t.p, c.gd.nrp, nr, c.nv, c.gd.nvp, c.nc, dgv.p, dgc.p, p, S.p);
    GWL_HIP(hipGetLastError());
    const unsigned rows_blocks = (unsigned)((nr + QT / 64 - 1) / (QT / 64));
    qr_norms_kernel<<<rows_blocks, QT, 0, st>>>(S.p, nr, p, nrm.p);
    GWL_HIP(hipGetLastError());
    for (int step = 0; step < n_mu; ++step) {
      qr_argmax_part_kernel<<<nparts, QT, 0, st>>>(nrm.p, taken.p, nr, pv.p, pi.p);
      qr_pivot_kernel<<<1, QT, 0, st>>>(pv.p, pi.p, nparts, S.p, p, step, taken.p, piv.p, jcur.p,
                                        q.p);
      qr_update_kernel<<<rows_blocks, QT, (size_t)p * 8, st>>>(S.p, nr, p, q.p, taken.p, nrm.p);
    }
    GWL_HIP(hipGetLastError());
    std::vector<int> hp(n_mu);
    GWL_HIP(hipMemcpyAsync(hp.data(), piv.p, sizeof(int) * n_mu, hipMemcpyDeviceToHost, st));
    GWL_HIP(hipStreamSynchronize(st));
    std::sort(hp.begin(), hp.end());
    for (int i = 0; i < n_mu; ++i) {
      GWL_CHECK(hp[i] >= 0 && hp[i] < nr && (i == 0 || hp[i] > hp[i - 1]), GWL_ENUMERIC,
                "pivoted QR produced an invalid point set");
      points_out[i] = hp[i];
    }
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
