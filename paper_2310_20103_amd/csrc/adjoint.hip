// Reverse-mode derivative (vector-Jacobian product) of Sigma_c with respect to
// the orbital energies and the orbital grid values.
//
// The scalar is l = sum_{q,w} Re(conj(G_qw) Sigma_q(w)).  The chain, for each
// (m, n) start vector, reverses the forward path:
//   continued fraction (Eq. 14) and assembly (Eq. 12)  -> a_bar, b_bar, N_bar, e_bar
//   Lanczos recurrence without reorthogonalisation (Eq. 13), vectors
//   recomputed from checkpoints                          -> q_bar, w_bar per step
//   Chebyshev series of p_g(C) (paragraph after Eq. 12) -> C_bar as outer products
//   C = Delta^2 + 2 Delta^1/2 K Delta^1/2 (Eq. 4)       -> Delta_bar, K_bar
//   coupling vectors P = (nm|vc) Delta^1/2               -> Delta_bar, k_bar
//   K and (nm|vc) as grid integrals (Eqs. 2-3)           -> orbital gradients.
// All reductions are fixed-order (no atomics), so two runs agree bitwise.
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

constexpr int NT = 256;
constexpr int ADJ_MAXL = 1024;

__device__ inline double wave_sum_a(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum_a(double v, double* sh) {
  v = wave_sum_a(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += sh[i];
  __syncthreads();
  return t;
}

struct cd {
  double r, i;
};
__device__ inline cd cmk(double r, double i) { return {r, i}; }
__device__ inline cd cadd(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ inline cd csub(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ inline cd cmul(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cd cscale(cd a, double s) { return {a.r * s, a.i * s}; }
__device__ inline cd cdiv(cd a, cd b) {
  const double d = 1.0 / (b.r * b.r + b.i * b.i);
  return {(a.r * b.r + a.i * b.i) * d, (a.i * b.r - a.r * b.i) * d};
}

// One block per pair; threads over frequencies.  Forward fractions t_k(w)
// are kept in tscr [pair][k][w] for the backward sweep.
__global__ void __launch_bounds__(NT)
cf_adjoint_kernel(const double* __restrict__ ca, const double* __restrict__ cb,
                  const int* __restrict__ lens, const double* __restrict__ norm2, int ld,
                  const double* __restrict__ e_n, const double* __restrict__ eta_n,
                  const int* __restrict__ qidx, const double* __restrict__ omega, int nomega,
                  double delta, const double* __restrict__ G, cd* __restrict__ tscr,
                  double* __restrict__ abar, double* __restrict__ bbar, double* __restrict__ nbar,
                  double* __restrict__ ebar, double* __restrict__ sig) {
  __shared__ double sa[ADJ_MAXL], sb2[ADJ_MAXL], t0r[ADJ_MAXL], acca[ADJ_MAXL], accb[ADJ_MAXL];
  __shared__ double sh[NT / 64];
  __shared__ double r0_sh;
  const int p = blockIdx.x, tid = threadIdx.x;
  const int L = lens[p];
  const double N = norm2[p];
  const bool empty = (L <= 0 || !(N > 0.0));
  for (int k = tid; k < ld; k += NT) {
    if (!empty && k < L) {
      sa[k] = ca[(long)p * ld + k];
      const double b = (k + 1 < L) ? cb[(long)p * ld + k] : 0.0;
      sb2[k] = b * b;
    }
    acca[k] = 0.0;
    accb[k] = 0.0;
  }
  __syncthreads();
  if (empty) {
    for (int k = tid; k < ld; k += NT) {
      abar[(long)p * ld + k] = 0.0;
      bbar[(long)p * ld + k] = 0.0;
    }
    for (int w = tid; w < nomega; w += NT) {
      sig[((long)p * nomega + w) * 2] = 0.0;
      sig[((long)p * nomega + w) * 2 + 1] = 0.0;
    }
    if (tid == 0) {
      nbar[p] = 0.0;
      ebar[p] = 0.0;
    }
    return;
  }
  if (tid == 0) {
    t0r[L - 1] = -sa[L - 1];
    for (int k = L - 2; k >= 0; --k) t0r[k] = -sa[k] - sb2[k] / t0r[k + 1];
    r0_sh = N / t0r[0];
  }
  __syncthreads();
  const double R0 = r0_sh;
  const double en = e_n[p], eta = eta_n[p];
  const int q = qidx[p];
  double r0bar = 0.0, nb = 0.0, eb = 0.0;
  cd* tp = tscr + (long)p * ld * nomega;
  for (int w0 = 0; w0 < nomega; w0 += NT) {
    const int w = w0 + tid;
    const bool valid = w < nomega;
    cd tbar = cmk(0, 0), zetabar = cmk(0, 0), c = cmk(0, 0), z = cmk(1, 0), S = cmk(0, 0);
    if (valid) {
      z = cmk(omega[w] - en, -eta * delta);
      const cd zeta = cscale(z, -eta);
      cd t = cmk(zeta.r - sa[L - 1], zeta.i);
      tp[(long)(L - 1) * nomega + w] = t;
      for (int k = L - 2; k >= 0; --k) {
        t = csub(cmk(zeta.r - sa[k], zeta.i), cdiv(cmk(sb2[k], 0), t));
        tp[(long)k * nomega + w] = t;
      }
      const cd R = cdiv(cmk(N, 0), t);
      S = cdiv(cmk(R.r - R0, R.i), z);
      sig[((long)p * nomega + w) * 2] = S.r * kHartreeEv;
      sig[((long)p * nomega + w) * 2 + 1] = S.i * kHartreeEv;
      const double* gq = G + ((long)q * nomega + w) * 2;
      c = cmk(gq[0] * kHartreeEv, -gq[1] * kHartreeEv);  // conj(G) E_h
      const cd rbar = cdiv(c, z);
      r0bar += -rbar.r;
      nb += cdiv(rbar, t).r;
      tbar = cmul(rbar, cdiv(cmk(-N, 0), cmul(t, t)));
    }
    for (int k = 0; k < L; ++k) {
      double ea = 0.0, eb2 = 0.0;
      if (valid) {
        ea = -tbar.r;
        zetabar = cadd(zetabar, tbar);
        if (k + 1 < L) {
          const cd tn = tp[(long)(k + 1) * nomega + w];
          eb2 = -cdiv(tbar, tn).r;
          tbar = cmul(tbar, cdiv(cmk(sb2[k], 0), cmul(tn, tn)));
        }
      }
      const double sA = block_sum_a(ea, sh);
      const double sB = block_sum_a(eb2, sh);
      if (tid == 0) {
        acca[k] += sA;
        accb[k] += sB;
      }
    }
    if (valid) eb += (cmul(c, cdiv(S, z))).r + eta * zetabar.r;
  }
  r0bar = block_sum_a(r0bar, sh);
  nb = block_sum_a(nb, sh);
  eb = block_sum_a(eb, sh);
  if (tid == 0) {
    // R(0) = N / t0_0: its cotangent r0bar is real
    nb += r0bar / t0r[0];
    double tb = r0bar * (-N / (t0r[0] * t0r[0]));
    for (int k = 0; k < L; ++k) {
      acca[k] += -tb;
      if (k + 1 < L) {
        accb[k] += -tb / t0r[k + 1];
        tb = tb * sb2[k] / (t0r[k + 1] * t0r[k + 1]);
      }
    }
    nbar[p] = nb;
    ebar[p] = eb;
  }
  __syncthreads();
  for (int k = tid; k < ld; k += NT) {
    abar[(long)p * ld + k] = k < L ? acca[k] : 0.0;
    // b_bar_{k+1} = 2 b_{k+1} (b^2)_bar
    bbar[(long)p * ld + k] = (k + 1 < L) ? 2.0 * cb[(long)p * ld + k] * accb[k] : 0.0;
  }
}

// One reverse Lanczos step k for every slot (see the forward in lanczos.hip):
//   r_k = w_k - a_k q_k - b_k q_{k-1},  b_{k+1} = |r_k|,  q_{k+1} = r_k / b_{k+1},
//   a_k = q_k . w_k,  w_k = D q_k.
// qb_next holds q_bar_{k+1} (complete), qb_cur / qb_prev receive the
// contributions to q_bar_k / q_bar_{k-1}; wbar receives w_bar_k (the
// cotangent that is pushed through D by the caller); pend carries the
// contribution of step k to b_bar_k.
__global__ void __launch_bounds__(NT)
lzb_step_kernel(int k, const int* __restrict__ pair_of_slot, const int* __restrict__ lens,
                int ld, const double* __restrict__ ca, const double* __restrict__ cb,
                const double* __restrict__ abar, const double* __restrict__ bbar,
                const double* __restrict__ q_next, const double* __restrict__ q_cur,
                const double* __restrict__ q_prev, const double* __restrict__ w_cur,
                const double* __restrict__ qb_next, double* __restrict__ qb_cur,
                double* __restrict__ qb_prev, double* __restrict__ wbar,
                double* __restrict__ pend, long nvc) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x;
  const int p = pair_of_slot[b];
  const long o = (long)b * nvc;
  const int Lp = p >= 0 ? lens[p] : 0;
  if (k >= Lp) {
    for (long i = threadIdx.x; i < nvc; i += NT) wbar[o + i] = 0.0;
    return;
  }
  const double ak = ca[(long)p * ld + k];
  const double abk = abar[(long)p * ld + k];
  if (k == Lp - 1) {
    for (long i = threadIdx.x; i < nvc; i += NT) {
      wbar[o + i] = abk * q_cur[o + i];
      qb_cur[o + i] += abk * w_cur[o + i];
    }
    __syncthreads();
    if (threadIdx.x == 0) pend[b] = 0.0;
    return;
  }
  const double b1 = cb[(long)p * ld + k];
  const double bk = k >= 1 ? cb[(long)p * ld + k - 1] : 0.0;
  const double pd = pend[b];
  double part = 0.0;
  for (long i = threadIdx.x; i < nvc; i += NT) part += qb_next[o + i] * q_next[o + i];
  const double d1 = block_sum_a(part, sh);
  const double B1 = bbar[(long)p * ld + k] + pd - d1 / b1;
  const double ib1 = 1.0 / b1;
  double p2 = 0.0, p3 = 0.0;
  for (long i = threadIdx.x; i < nvc; i += NT) {
    const double rb = qb_next[o + i] * ib1 + B1 * q_next[o + i];
    p2 += rb * q_cur[o + i];
    if (k >= 1) p3 += rb * q_prev[o + i];
  }
  const double d2 = block_sum_a(p2, sh);
  const double d3 = block_sum_a(p3, sh);
  const double atot = abk - d2;
  for (long i = threadIdx.x; i < nvc; i += NT) {
    const double rb = qb_next[o + i] * ib1 + B1 * q_next[o + i];
    qb_cur[o + i] += -ak * rb + atot * w_cur[o + i];
    if (k >= 1) qb_prev[o + i] += -bk * rb;
    wbar[o + i] = rb + atot * q_cur[o + i];
  }
  if (threadIdx.x == 0) pend[b] = -d3;
}

// Start vector: q_0 = P/|P|, N = |P|^2; P = (nm|vc) Delta^1/2.
// P_bar = (q_bar_0 - q_0 (q_0 . q_bar_0)) / |P| + 2 N_bar P;
// Delta_bar += P_bar P / (2 Delta);  k_bar = P_bar Delta^1/2 (row of the slot;
// zero for an empty slot or a zero start vector).
__global__ void __launch_bounds__(NT)
lzb_start_kernel(const int* __restrict__ pair_of_slot, const double* __restrict__ norm2,
                 const double* __restrict__ nbar, const double* __restrict__ P,
                 const double* __restrict__ qb0, const double* __restrict__ sdelta,
                 double* __restrict__ dbar,
                 double* __restrict__ kbar, long nvc) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x;
  const int p = pair_of_slot[b];
  const long o = (long)b * nvc;
  const double N = p >= 0 ? norm2[p] : 0.0;
  if (!(N > 0.0)) {
    for (long i = threadIdx.x; i < nvc; i += NT) kbar[o + i] = 0.0;
    return;
  }
  const double s = sqrt(N), is = 1.0 / s;
  double part = 0.0;
  for (long i = threadIdx.x; i < nvc; i += NT) part += P[o + i] * is * qb0[o + i];
  const double d = block_sum_a(part, sh);
  const double nb2 = 2.0 * nbar[p];
  for (long i = threadIdx.x; i < nvc; i += NT) {
    const double pi = P[o + i];
    const double pbar = (qb0[o + i] - pi * is * d) * is + nb2 * pi;
    dbar[o + i] += pbar * pi / (2.0 * sdelta[i] * sdelta[i]);
    kbar[o + i] = pbar * sdelta[i];
  }
}

// Chebyshev adjoint step after the product C s_j:
//   s_{j-1} = c_{j-1} x + sigma C~ s_j - s_{j+1},  C~ = (2C - (hi+lo))/(hi-lo),
// also K~ s_j = K Delta^1/2 s_j; optional cast of s_{j-1} for the next product.
__global__ void combine_adj_kernel(PairGeom g, int nb, int splitk, const double* __restrict__ ypart,
                                   const double* __restrict__ sj, const double* __restrict__ sj1,
                                   const double* __restrict__ seed, double cprev, double sigma,
                                   double lo, double hi, double* __restrict__ out,
                                   double* __restrict__ ks, double* __restrict__ u) {
  const int b = blockIdx.y;
  const long stride_s = (long)nb * g.nvp * g.ncp;
  const double* yb = ypart + (long)b * g.nvp * g.ncp;
  const double inv = 1.0 / (hi - lo);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < g.nvc; i += (long)gridDim.x * blockDim.x) {
    const int v = (int)i / g.nc, c = (int)i - v * g.nc;  // (N_v N_c < 2^31)
    const long off = (long)v * g.ncp + c;
    double y = 0.0;
    for (int s = 0; s < splitk; ++s) y += yb[s * stride_s + off];
    const long o = (long)b * g.nvc + i;
    const double x = sj[o];
    const double k = g.dv * y;
    const double cx = g.delta2[i] * x + 2.0 * g.sdelta[i] * k;
    const double ct = (2.0 * cx - (hi + lo) * x) * inv;
    const double nv = cprev * seed[o] + sigma * ct - (sj1 ? sj1[o] : 0.0);
    out[o] = nv;
    ks[o] = k;
    if (u) u[(long)b * g.nvp * g.ncp + off] = g.sdelta[i] * nv;
  }
}

__global__ void scale_copy_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                  double c, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = c * src[i];
}

__global__ void axpy_kernel(double* __restrict__ dst, const double* __restrict__ src, double a,
                            long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] += a * src[i];
}

// dst[i] = sum over rows r < nrows of src[r][i], in row order
__global__ void sum_rows_kernel(double* __restrict__ dst, const double* __restrict__ src,
                                int nrows, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double s = dst[i];
    for (int r = 0; r < nrows; ++r) s += src[(long)r * n + i];
    dst[i] = s;
  }
}

// S = A + A^T for an n x n matrix
// grad_n += dV phi_m Vk_p, grad_m += dV phi_n Vk_p for every pair p, in pair order
__global__ void orb_grad_nm_kernel(const double* __restrict__ psi_t, const double* __restrict__ Vk,
                                   long ld, int nr, const int* __restrict__ mrow,
                                   const int* __restrict__ nrow, int npairs, double dv,
                                   double* __restrict__ grad) {
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < nr; r += (long)gridDim.x * blockDim.x) {
    for (int p = 0; p < npairs; ++p) {
      const double vk = dv * Vk[(long)p * ld + r];
      const int mr = mrow[p], nrw = nrow[p];
      grad[(long)nrw * ld + r] += psi_t[(long)mr * ld + r] * vk;
      grad[(long)mr * ld + r] += psi_t[(long)nrw * ld + r] * vk;
    }
  }
}

// user layout [n_orb][nr] from the internal padded [nvp + ncp][ld], in the
// orbitals' own type
template <typename T>
__global__ void gather_orbitals_kernel(const double* __restrict__ src, long ld, int nr, int nv,
                                       int nvp, T* __restrict__ dst) {
  const int a = blockIdx.y;
  const long row = a < nv ? a : nvp + (a - nv);
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < nr; r += (long)gridDim.x * blockDim.x)
    dst[(long)a * nr + r] = (T)src[row * ld + r];
}

inline int gelems(long n) {
  long g = (n + NT - 1) / NT;
  return (int)(g > 1024 ? 1024 : (g < 1 ? 1 : g));
}

}  // namespace

void adj_cfrac(int npairs, const double* ca, const double* cb, const int* lens,
               const double* norm2, int ld, const double* e_n, const double* eta_n,
               const int* qidx, const double* omega_ha, int nomega, double delta_ha,
               const double* G, void* tscr, double* abar, double* bbar, double* nbar,
               double* ebar, double* sig, hipStream_t st) {
  if (npairs <= 0) return;
  GWL_CHECK(ld <= ADJ_MAXL, GWL_EINVAL, "adjoint supports at most 1024 Lanczos steps");
  cf_adjoint_kernel<<<npairs, NT, 0, st>>>(ca, cb, lens, norm2, ld, e_n, eta_n, qidx, omega_ha,
                                           nomega, delta_ha, G, static_cast<cd*>(tscr), abar,
                                           bbar, nbar, ebar, sig);
  GWL_HIP(hipGetLastError());
}

void adj_lanczos_step(int k, int nb, const int* pair_of_slot, const int* lens, int ld,
                      const double* ca, const double* cb, const double* abar, const double* bbar,
                      const double* q_next, const double* q_cur, const double* q_prev,
                      const double* w_cur, const double* qb_next, double* qb_cur, double* qb_prev,
                      double* wbar, double* pend, long nvc, hipStream_t st) {
  lzb_step_kernel<<<nb, NT, 0, st>>>(k, pair_of_slot, lens, ld, ca, cb, abar, bbar, q_next,
                                     q_cur, q_prev, w_cur, qb_next, qb_cur, qb_prev, wbar, pend,
                                     nvc);
  GWL_HIP(hipGetLastError());
}

void adj_start(int nb, const int* pair_of_slot, const double* norm2, const double* nbar,
               const double* P, const double* qb0, const double* sdelta, double* dbar,
               double* kbar, long nvc, hipStream_t st) {
  lzb_start_kernel<<<nb, NT, 0, st>>>(pair_of_slot, norm2, nbar, P, qb0, sdelta, dbar, kbar, nvc);
  GWL_HIP(hipGetLastError());
}

void adj_combine(const PairGeom& g, int nb, int splitk, const double* ypart, const double* sj,
                 const double* sj1, const double* seed, double cprev, double sigma, double lo,
                 double hi, double* out, double* ks, double* u, hipStream_t st) {
  dim3 grid(gelems(g.nvc), nb);
  combine_adj_kernel<<<grid, NT, 0, st>>>(g, nb, splitk, ypart, sj, sj1, seed, cprev, sigma, lo,
                                          hi, out, ks, u);
  GWL_HIP(hipGetLastError());
}

void adj_scale_copy(double* dst, const double* src, double c, long n, hipStream_t st) {
  scale_copy_kernel<<<gelems(n), NT, 0, st>>>(dst, src, c, n);
  GWL_HIP(hipGetLastError());
}

void adj_axpy(double* dst, const double* src, double a, long n, hipStream_t st) {
  axpy_kernel<<<gelems(n), NT, 0, st>>>(dst, src, a, n);
  GWL_HIP(hipGetLastError());
}

void adj_sum_rows(double* dst, const double* src, int nrows, long n, hipStream_t st) {
  sum_rows_kernel<<<gelems(n), NT, 0, st>>>(dst, src, nrows, n);
  GWL_HIP(hipGetLastError());
}

void adj_orb_grad_nm(const double* psi_t, const double* Vk, long ld, int nr, const int* mrow,
                     const int* nrow, int npairs, double dv, double* grad, hipStream_t st) {
  orb_grad_nm_kernel<<<gelems(nr), NT, 0, st>>>(psi_t, Vk, ld, nr, mrow, nrow, npairs, dv, grad);
  GWL_HIP(hipGetLastError());
}

void adj_gather_orbitals(const double* src, long ld, int nr, int nv, int nvp, int norb,
                         void* dst, bool f32, hipStream_t st) {
  const dim3 grid(gelems(nr), norb);
  if (f32)
    gather_orbitals_kernel<float><<<grid, NT, 0, st>>>(src, ld, nr, nv, nvp,
                                                       static_cast<float*>(dst));
  else
    gather_orbitals_kernel<double><<<grid, NT, 0, st>>>(src, ld, nr, nv, nvp,
                                                        static_cast<double*>(dst));
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
