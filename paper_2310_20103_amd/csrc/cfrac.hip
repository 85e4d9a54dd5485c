// Continued fraction (Haydock, Eq. 14) and assembly of Sigma(w, n) (Eq. 12):
//   R(zeta) = ||P||^2 / (zeta - a_0 - b_1^2 / (zeta - a_1 - ...)),
//   Sigma(w, n) = [R(-eta_n z_n) - R(0)] / z_n,  z_n = w - e_n - i eta_n delta.
// Tamm-Dancoff (B = 0 in the Casida matrix, Lanczos on A from (nm|vc)):
//   Sigma(w, n) = -eta_n R_A(-eta_n z_n).
// FP64 complex.  One thread per (pair, frequency); the pair's coefficients are
// staged in LDS.  Both evaluation points are off the spectrum (Im = +delta, or
// 0 below the positive spectrum of D), so the backward recurrence never
// divides by zero.
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

constexpr int CF_MAXL = 4000;

__global__ void __launch_bounds__(256)
cfrac_kernel(const double* __restrict__ ca, const double* __restrict__ cb,
             const int* __restrict__ lens, const double* __restrict__ norm2, int ld,
             const double* __restrict__ e_n, const double* __restrict__ eta_n,
             const double* __restrict__ omega, int nomega, double delta, int tda,
             double* __restrict__ sig) {
  __shared__ double sa[CF_MAXL];
  __shared__ double sb2[CF_MAXL];
  __shared__ double r0_sh;
  const int p = blockIdx.y;
  const int L = lens[p];
  const double n2 = norm2[p];
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    sa[k] = ca[(long)p * ld + k];
    const double b = (k + 1 < L) ? cb[(long)p * ld + k] : 0.0;  // b_{k+1}
    sb2[k] = b * b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r0 = 0.0;
    if (L > 0 && n2 > 0.0) {
      double t = -sa[L - 1];
      for (int k = L - 2; k >= 0; --k) t = -sa[k] - sb2[k] / t;
      r0 = n2 / t;
    }
    r0_sh = r0;
  }
  __syncthreads();
  const double r0 = r0_sh;
  const double en = e_n[p], eta = eta_n[p];
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nomega; w += gridDim.x * blockDim.x) {
    double sr = 0.0, si = 0.0;
    if (L > 0 && n2 > 0.0) {
      const double zr = omega[w] - en, zi = -eta * delta;
      // zeta = -eta z
      const double xr = -eta * zr, xi = -eta * zi;
      double tr = xr - sa[L - 1], ti = xi;
      for (int k = L - 2; k >= 0; --k) {
        const double inv = sb2[k] / (tr * tr + ti * ti);
        // t = zeta - a_k - b^2 / t ;  b^2 / t = b^2 conj(t) / |t|^2
        tr = xr - sa[k] - inv * tr;
        ti = xi + inv * ti;
      }
      // R(zeta) = n2 / t
      const double d = 1.0 / (tr * tr + ti * ti);
      const double rr = n2 * tr * d, ri = -n2 * ti * d;
      if (tda) {
        sr = -eta * rr;
        si = -eta * ri;
      } else {
        // (R - r0) / z
        const double nr = rr - r0, ni = ri;
        const double dz = 1.0 / (zr * zr + zi * zi);
        sr = (nr * zr + ni * zi) * dz;
        si = (ni * zr - nr * zi) * dz;
      }
    }
    sig[((long)p * nomega + w) * 2] = sr * kHartreeEv;
    sig[((long)p * nomega + w) * 2 + 1] = si * kHartreeEv;
  }
}

__global__ void sum_groups_kernel(const double* __restrict__ sig, int per, int nomega,
                                  double* __restrict__ out) {
  const int q = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * nomega; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < per; ++i) s += sig[((long)(q * per + i) * nomega) * 2 + e];
    out[(long)q * nomega * 2 + e] = s;
  }
}

}  // namespace

void cfrac_sigma(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                 const double* norm2, int ld, const double* e_n, const double* eta_n,
                 const double* omega_ha, int nomega, double delta_ha, int tda, double* sig,
                 hipStream_t st) {
  if (npairs <= 0 || nomega <= 0) return;
  GWL_CHECK(ld <= CF_MAXL, GWL_EINVAL, "Lanczos length exceeds 4000");
  dim3 grid(ceil_div(nomega, 256), npairs);
  cfrac_kernel<<<grid, 256, 0, st>>>(coef_a, coef_b, lens, norm2, ld, e_n, eta_n, omega_ha,
                                     nomega, delta_ha, tda, sig);
  GWL_HIP(hipGetLastError());
}

void sum_groups(const double* sig, int ngroups, int per, int nomega, double* out,
                hipStream_t st) {
  if (ngroups <= 0) return;
  dim3 grid(ceil_div(2 * nomega, 256), ngroups);
  sum_groups_kernel<<<grid, 256, 0, st>>>(sig, per, nomega, out);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
