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

// ---------------------------------------------------------------- interval check
// Number of eigenvalues of the L x L tridiagonal T below tau: the negative
// pivots of T - tau I = L D L^T (Sylvester's law of inertia).  A zero pivot
// is replaced by a tiny negative one, as in bisection codes.
__device__ inline int sturm_below(const double* __restrict__ a, const double* __restrict__ b,
                                  int L, double tau) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < L; ++i) {
    d = (a[i] - tau) - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
    if (fabs(d) < 1e-280) d = -1e-280;
    cnt += d < 0.0;
  }
  return cnt;
}

__global__ void __launch_bounds__(256)
interval_check_kernel(int npairs, const double* __restrict__ ca, const double* __restrict__ cb,
                      const int* __restrict__ lens, int ld, double t_lo, double t_hi,
                      int* __restrict__ bad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int L = lens[p];
  const double* a = ca + (long)p * ld;
  const double* b = cb + (long)p * ld;
  int out = 0;
  if (L > 0) out = sturm_below(a, b, L, t_lo) > 0 || sturm_below(a, b, L, t_hi) < L;
  bad[p] = out;
}

// ---------------------------------------------------------------- quadrature
// Lanczos on C + Gauss quadrature: the eigenvalues theta_k of each pair's
// tridiagonal T and the first components u_k(0) of its eigenvectors, by the
// implicit QL iteration with shifts (Bowdler, Martin, Reinsch and Wilkinson)
// applying each plane rotation to the first row of the eigenvector matrix
// only (Golub and Welsch).  One thread per pair; d, e, z are that pair's rows
// of the scratch arrays (FP64).  On return d = theta, z = ||P||^2 u(0)^2.
// status[p] = 1 if an eigenvalue needed more than 60 sweeps.
__global__ void quad_eig_kernel(int npairs, const double* __restrict__ ca,
                                const double* __restrict__ cb, const int* __restrict__ lens,
                                const double* __restrict__ norm2, int ld, double* __restrict__ qd,
                                double* __restrict__ qe, double* __restrict__ qz,
                                int* __restrict__ status) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int n = lens[p];
  double* d = qd + (long)p * ld;
  double* e = qe + (long)p * ld;
  double* z = qz + (long)p * ld;
  for (int i = 0; i < n; ++i) {
    d[i] = ca[(long)p * ld + i];
    e[i] = (i + 1 < n) ? cb[(long)p * ld + i] : 0.0;  // e[i] couples i and i + 1
    z[i] = (i == 0) ? 1.0 : 0.0;
  }
  int bad = 0;
  for (int l = 0; l < n; ++l) {
    int sweeps = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = fabs(d[m]) + fabs(d[m + 1]);
        if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;  // below one ulp of the diagonal
      }
      if (m == l) break;
      if (++sweeps > 60) {
        bad = 1;
        break;
      }
      // shift from the leading 2 x 2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      int i = m - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        const double zf = z[i + 1];
        z[i + 1] = s * z[i] + c * zf;
        z[i] = c * z[i] - s * zf;
      }
      if (underflow) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  const double n2 = norm2[p];
  for (int i = 0; i < n; ++i) z[i] = n2 * z[i] * z[i];
  status[p] = bad;
}

// Sigma(w, n) = sum_k w_k [1/sqrt(theta_k) - 1/(sqrt(theta_k) + eta z)] / z.
__global__ void __launch_bounds__(256)
quad_sigma_kernel(const double* __restrict__ qd, const double* __restrict__ qz,
                  const int* __restrict__ lens, int ld, const double* __restrict__ e_n,
                  const double* __restrict__ eta_n, const double* __restrict__ omega, int nomega,
                  double delta, double* __restrict__ sig) {
  __shared__ double so[CF_MAXL];
  __shared__ double sw[CF_MAXL];
  const int p = blockIdx.y;
  const int L = lens[p];
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    so[k] = sqrt(fmax(qd[(long)p * ld + k], 0.0));
    sw[k] = qz[(long)p * ld + k];
  }
  __syncthreads();
  const double en = e_n[p], eta = eta_n[p];
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < nomega; w += gridDim.x * blockDim.x) {
    const double zr = omega[w] - en, zi = -eta * delta;
    double ar = 0.0, ai = 0.0;  // sum_k w_k [1/O_k - 1/(O_k + eta z)]
    for (int k = 0; k < L; ++k) {
      const double o = so[k];
      if (o <= 0.0 || sw[k] == 0.0) continue;
      const double dr = o + eta * zr, di = eta * zi;
      const double inv = 1.0 / (dr * dr + di * di);
      ar += sw[k] * (1.0 / o - dr * inv);
      ai += sw[k] * (di * inv);
    }
    const double dz = 1.0 / (zr * zr + zi * zi);
    const double sr = (ar * zr + ai * zi) * dz;
    const double si = (ai * zr - ar * zi) * dz;
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

// out[e] = (sum_n sig[2n][e] - sig[2n+1][e]) / 4, n in order: the
// polarisation identity over runs from P_nm + P_nm' (even pairs) and
// P_nm - P_nm' (odd pairs)
__global__ void sum_polar_kernel(const double* __restrict__ sig, int nn, int nomega,
                                 double* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * nomega; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int n = 0; n < nn; ++n)
      s += sig[((long)(2 * n) * nomega) * 2 + e] - sig[((long)(2 * n + 1) * nomega) * 2 + e];
    out[e] = 0.25 * s;
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

void quad_sigma(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                const double* norm2, int ld, const double* e_n, const double* eta_n,
                const double* omega_ha, int nomega, double delta_ha, double* qd, double* qe,
                double* qz, int* status, double* sig, hipStream_t st) {
  if (npairs <= 0 || nomega <= 0) return;
  GWL_CHECK(ld <= CF_MAXL, GWL_EINVAL, "Lanczos length exceeds 4000");
  quad_eig_kernel<<<ceil_div(npairs, 64), 64, 0, st>>>(npairs, coef_a, coef_b, lens, norm2, ld,
                                                        qd, qe, qz, status);
  GWL_HIP(hipGetLastError());
  dim3 grid(ceil_div(nomega, 256), npairs);
  quad_sigma_kernel<<<grid, 256, 0, st>>>(qd, qz, lens, ld, e_n, eta_n, omega_ha, nomega,
                                          delta_ha, sig);
  GWL_HIP(hipGetLastError());
}

void sum_groups(const double* sig, int ngroups, int per, int nomega, double* out,
                hipStream_t st) {
  if (ngroups <= 0) return;
  dim3 grid(ceil_div(2 * nomega, 256), ngroups);
  sum_groups_kernel<<<grid, 256, 0, st>>>(sig, per, nomega, out);
  GWL_HIP(hipGetLastError());
}

void sum_polar(const double* sig, int nn, int nomega, double* out, hipStream_t st) {
  if (nn <= 0 || nomega <= 0) return;
  sum_polar_kernel<<<ceil_div(2 * nomega, 256), 256, 0, st>>>(sig, nn, nomega, out);
  GWL_HIP(hipGetLastError());
}

void lz_interval_check(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                       int ld, double t_lo, double t_hi, int* bad, hipStream_t st) {
  if (npairs <= 0) return;
  interval_check_kernel<<<(npairs + 255) / 256, 256, 0, st>>>(npairs, coef_a, coef_b, lens, ld,
                                                              t_lo, t_hi, bad);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
