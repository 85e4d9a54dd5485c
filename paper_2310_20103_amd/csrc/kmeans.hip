// Interpolation points for ISDF by weighted K-means (centroidal Voronoi
// tessellation of the grid).  The paper names ISDF without its point
// selection; this follows the weighted K-means reading:
//
//   w(r) = (sum_v phi_v(r)^2)(sum_c phi_c(r)^2), each sum in orbital order,
//   quantised to W(r) = floor(w / max w * 2^30 + 1/2) so that the cluster sums
//   below are exact integers, independent of summation order;
//   assignment: nearest centroid under the periodic minimum-image distance in
//   bohr, ties to the lower centroid index;
//   update: centroid = its nearest grid point + (sum W D) / (sum W), D the
//   integer displacement of a member from that grid point wrapped into
//   [-n/2, n/2) per axis; clusters without weight keep their centroid;
//   stop when an assignment repeats the previous one or after max_iter
//   updates; each non-empty cluster contributes its member nearest the
//   centroid (ties to the lower grid index).
//
// Every floating-point step is a single IEEE operation in a fixed order
// (floating-point contraction is off in this file, so no multiply-add is
// fused), so the points are reproducible bit for bit.  FP64 throughout; one thread per grid
// point, centroids staged through LDS.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"

#pragma clang fp contract(off)

namespace gwl {
namespace {

constexpr int KT = 256;
constexpr int KCH = 1024;                 // centroids per LDS chunk
constexpr double KQ = 1073741824.0;       // 2^30

__device__ inline unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

__global__ void __launch_bounds__(KT)
km_weight_kernel(const double* __restrict__ psi_t, long nrp, long nr, int nv, int nvp, int nc,
                 double* __restrict__ w, unsigned long long* __restrict__ wmax) {
  __shared__ unsigned long long red[KT / 64];
  const long r = blockIdx.x * (long)KT + threadIdx.x;
  double x = 0.0;
  if (r < nr) {
    double a = 0.0, b = 0.0;
    for (int v = 0; v < nv; ++v) {
      const double p = psi_t[(long)v * nrp + r];
      a = a + p * p;
    }
    for (int c = 0; c < nc; ++c) {
      const double p = psi_t[(long)(nvp + c) * nrp + r];
      b = b + p * p;
    }
    x = a * b;
    w[r] = x;
  }
  // w >= 0, so its bit pattern orders like its value
  unsigned long long m = dbits(x);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(m, o, 64);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < KT / 64; ++i) m = red[i] > m ? red[i] : m;
    atomicMax(wmax, m);
  }
}

__global__ void km_quant_kernel(const double* __restrict__ w, long nr,
                                const unsigned long long* __restrict__ wmax,
                                long long* __restrict__ W) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const double m = __longlong_as_double((long long)*wmax);
  W[r] = (long long)floor(w[r] / m * KQ + 0.5);
}

// periodic minimum image of d (grid units) on an axis of n points, in bohr
__device__ inline double mimg(double d, double n, double h) {
  const double f = floor(d / n + 0.5);
  return (d - n * f) * h;
}

__global__ void __launch_bounds__(KT)
km_assign_kernel(long nr, int nx, int ny, int nz, double hx, double hy, double hz,
                 const double* __restrict__ cent, int K, int* __restrict__ lab,
                 double* __restrict__ best, int* __restrict__ changed, int first) {
  __shared__ double cs[KCH * 3];
  const long r = blockIdx.x * (long)KT + threadIdx.x;
  const bool ok = r < nr;
  const long yz = (long)ny * nz;
  const double x = ok ? (double)(r / yz) : 0.0;
  const double y = ok ? (double)((r % yz) / nz) : 0.0;
  const double z = ok ? (double)(r % nz) : 0.0;
  const double fx = nx, fy = ny, fz = nz;
  double bd = INFINITY;
  int bk = 0;
  for (int k0 = 0; k0 < K; k0 += KCH) {
    const int cnt = min(KCH, K - k0);
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * 3; i += KT) cs[i] = cent[(long)k0 * 3 + i];
    __syncthreads();
    if (ok) {
      for (int k = 0; k < cnt; ++k) {
        const double px = mimg(x - cs[3 * k], fx, hx);
        const double py = mimg(y - cs[3 * k + 1], fy, hy);
        const double pz = mimg(z - cs[3 * k + 2], fz, hz);
        const double d2 = px * px + py * py + pz * pz;
        if (d2 < bd) {
          bd = d2;
          bk = k0 + k;
        }
      }
    }
  }
  bool ch = false;
  if (ok) {
    ch = first || lab[r] != bk;
    lab[r] = bk;
    best[r] = bd;
  }
  const unsigned long long any = __ballot(ch);
  if (any && (threadIdx.x & 63) == 0) atomicOr(changed, 1);
}

// wrapped integer displacement of coordinate q from the grid point nearest c
__device__ inline long long wrap_disp(long q, double c, int n) {
  const long long rc = (long long)floor(c + 0.5);
  long long m = (q - rc + n / 2) % n;
  if (m < 0) m += n;
  return m - n / 2;
}

__global__ void km_accum_kernel(long nr, int nx, int ny, int nz, const int* __restrict__ lab,
                                const long long* __restrict__ W,
                                const double* __restrict__ cent,
                                unsigned long long* __restrict__ s0,
                                unsigned long long* __restrict__ s1) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r >= nr) return;
  const long long w = W[r];
  if (w == 0) return;
  const int k = lab[r];
  const long yz = (long)ny * nz;
  const long q[3] = {r / yz, (r % yz) / nz, r % nz};
  const int n[3] = {nx, ny, nz};
  atomicAdd(&s0[k], (unsigned long long)w);
  for (int a = 0; a < 3; ++a)
    atomicAdd(&s1[3 * k + a], (unsigned long long)(w * wrap_disp(q[a], cent[3 * k + a], n[a])));
}

__global__ void km_update_kernel(int K, int nx, int ny, int nz,
                                 const unsigned long long* __restrict__ s0,
                                 const unsigned long long* __restrict__ s1,
                                 double* __restrict__ cent) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const long long S0 = (long long)s0[k];
  if (S0 <= 0) return;
  const int n[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    const double rc = floor(cent[3 * k + a] + 0.5);
    const double na = rc + (double)(long long)s1[3 * k + a] / (double)S0;
    const double fn = n[a];
    cent[3 * k + a] = na - fn * floor(na / fn);
  }
}

__global__ void km_pick_dist_kernel(long nr, const int* __restrict__ lab,
                                    const double* __restrict__ best,
                                    unsigned long long* __restrict__ mind) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r < nr) atomicMin(&mind[lab[r]], dbits(best[r]));
}

__global__ void km_pick_index_kernel(long nr, const int* __restrict__ lab,
                                     const double* __restrict__ best,
                                     const unsigned long long* __restrict__ mind,
                                     int* __restrict__ minr) {
  const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (r < nr && dbits(best[r]) == mind[lab[r]]) atomicMin(&minr[lab[r]], (int)r);
}

int grid_for(long n) { return (int)((n + KT - 1) / KT); }

}  // namespace
}  // namespace gwl

using namespace gwl;

extern "C" gwl_status gwl_isdf_kmeans(gwl_ctx* ctx, const int* init_points, int n_init,
                                      int max_iter, int* points_out, int* n_points,
                                      int* n_assign) {
  try {
    GWL_CHECK(ctx != nullptr, GWL_EINVAL, "null context");
    gwl_ctx& c = *ctx;
    GWL_CHECK(init_points && points_out && n_points && n_assign, GWL_EINVAL, "null pointer");
    GWL_CHECK(n_init >= 1 && n_init <= c.nr, GWL_EINVAL, "need 1 <= n_init <= N_r");
    GWL_CHECK(max_iter >= 0, GWL_EINVAL, "max_iter must be >= 0");
    const long nr = c.nr;
    const long yz = (long)c.ny * c.nz;
    std::vector<double> cent0((size_t)n_init * 3);
    for (int i = 0; i < n_init; ++i) {
      const long p = init_points[i];
      GWL_CHECK(p >= 0 && p < nr, GWL_EINVAL, "initial point out of range");
      cent0[3 * i] = (double)(p / yz);
      cent0[3 * i + 1] = (double)((p % yz) / c.nz);
      cent0[3 * i + 2] = (double)(p % c.nz);
    }
    hipStream_t st = c.stream;
    const double hx = c.lx / c.nx, hy = c.ly / c.ny, hz = c.lz / c.nz;
    DevBuf<double> w, cent, best;
    DevBuf<long long> W;
    DevBuf<int> lab, flag, minr;
    DevBuf<unsigned long long> wmax, s0, s1, mind;
    w.ensure(nr);
    W.ensure(nr);
    best.ensure(nr);
    lab.ensure(nr);
    flag.ensure(1);
    wmax.ensure(1);
    cent.ensure((size_t)n_init * 3);
    s0.ensure(n_init);
    s1.ensure((size_t)n_init * 3);
    mind.ensure(n_init);
    minr.ensure(n_init);
    GWL_HIP(hipMemcpyAsync(cent.p, cent0.data(), cent0.size() * 8, hipMemcpyHostToDevice, st));

    km_weight_kernel<<<grid_for(nr), KT, 0, st>>>(c.psi_t.p, c.gd.nrp, nr, c.nv, c.gd.nvp, c.nc,
                                                 w.p, wmax.p);
    GWL_HIP(hipGetLastError());
    unsigned long long wm = 0;
    GWL_HIP(hipMemcpyAsync(&wm, wmax.p, 8, hipMemcpyDeviceToHost, st));
    GWL_HIP(hipStreamSynchronize(st));
    double wmd;
    std::memcpy(&wmd, &wm, 8);
    GWL_CHECK(wmd > 0.0, GWL_EINVAL, "the K-means weights vanish everywhere");
    km_quant_kernel<<<grid_for(nr), KT, 0, st>>>(w.p, nr, wmax.p, W.p);
    GWL_HIP(hipGetLastError());

    int assigned = 0;
    for (int it = 0; it <= max_iter; ++it) {
      GWL_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
      km_assign_kernel<<<grid_for(nr), KT, 0, st>>>(nr, c.nx, c.ny, c.nz, hx, hy, hz, cent.p,
                                                   n_init, lab.p, best.p, flag.p, it == 0);
      GWL_HIP(hipGetLastError());
      ++assigned;
      int changed = 1;
      GWL_HIP(hipMemcpyAsync(&changed, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
      GWL_HIP(hipStreamSynchronize(st));
      if (it > 0 && !changed) break;
      if (it == max_iter) break;
      GWL_HIP(hipMemsetAsync(s0.p, 0, (size_t)n_init * 8, st));
      GWL_HIP(hipMemsetAsync(s1.p, 0, (size_t)n_init * 24, st));
      km_accum_kernel<<<grid_for(nr), KT, 0, st>>>(nr, c.nx, c.ny, c.nz, lab.p, W.p, cent.p,
                                                  s0.p, s1.p);
      GWL_HIP(hipGetLastError());
      km_update_kernel<<<grid_for(n_init), KT, 0, st>>>(n_init, c.nx, c.ny, c.nz, s0.p, s1.p,
                                                       cent.p);
      GWL_HIP(hipGetLastError());
    }
    GWL_HIP(hipMemsetAsync(mind.p, 0xff, (size_t)n_init * 8, st));
    GWL_HIP(hipMemsetAsync(minr.p, 0x7f, (size_t)n_init * sizeof(int), st));
    km_pick_dist_kernel<<<grid_for(nr), KT, 0, st>>>(nr, lab.p, best.p, mind.p);
    GWL_HIP(hipGetLastError());
    km_pick_index_kernel<<<grid_for(nr), KT, 0, st>>>(nr, lab.p, best.p, mind.p, minr.p);
    GWL_HIP(hipGetLastError());
    std::vector<int> mr(n_init);
    GWL_HIP(hipMemcpyAsync(mr.data(), minr.p, (size_t)n_init * sizeof(int),
                           hipMemcpyDeviceToHost, st));
    GWL_HIP(hipStreamSynchronize(st));
    std::vector<int> pts;
    for (int k = 0; k < n_init; ++k)
      if (mr[k] < nr) pts.push_back(mr[k]);
    std::sort(pts.begin(), pts.end());
    std::copy(pts.begin(), pts.end(), points_out);
    *n_points = (int)pts.size();
    *n_assign = assigned;
    return GWL_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GWL_ENOMEM;
  }
}
