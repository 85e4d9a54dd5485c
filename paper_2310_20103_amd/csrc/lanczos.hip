// Pair-space kernels: the Chebyshev combination that turns C-products into
// p_g(C) x (paragraph after Eq. 12), the coupling-vector finish
// (P_nm = (nm|vc) Delta^1/2), and the batched FP64 Lanczos recurrence of
// Eq. 13 with optional reorthogonalisation.
//
// All reductions are deterministic: a fixed wavefront shuffle tree followed by
// a fixed-order sum over the block's waves; no atomics.  One block per Lanczos
// slot for dots and norms (pair vectors are at most a few MB), grid-stride
// elementwise kernels elsewhere.
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

constexpr int NT = 256;
// a_k and b_k run one block per slot: 1,024 threads keep a slot's whole
// vector in flight from one CU
constexpr int NTS = 1024;

// Pair-space rows are read as 16-byte pairs when every row starts 16 bytes
// apart (N_v N_c even; basis rows are whole multiples of a pair vector).
__device__ inline const double2* as_d2(const double* p) {
  return reinterpret_cast<const double2*>(p);
}
__device__ inline double2* as_d2(double* p) { return reinterpret_cast<double2*>(p); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum; result broadcast to every thread.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) t += sh[i];
  __syncthreads();
  return t;
}

template <typename U>
__device__ inline U to_op(double v);
template <>
__device__ inline double to_op<double>(double v) { return v; }
template <>
__device__ inline f16_t to_op<f16_t>(double v) { return f32_to_f16((float)v); }

__global__ void pair_product_kernel(const double* __restrict__ psi_t, long ld, int nr,
                                    const int* __restrict__ m_idx, const int* __restrict__ n_idx,
                                    double* __restrict__ rho) {
  const int i = blockIdx.y;
  const double* a = psi_t + (long)m_idx[i] * ld;
  const double* b = psi_t + (long)n_idx[i] * ld;
  double* o = rho + (long)i * ld;
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < ld; r += (long)gridDim.x * blockDim.x)
    o[r] = a[r] * b[r];
}

template <typename U>
__global__ void cast_u_kernel(PairGeom g, const double* __restrict__ x, long ldx, U* __restrict__ u) {
  const int b = blockIdx.y;
  const int slot = g.rows ? g.rows[b] : b;
  const double* xb = x + (long)slot * ldx;
  U* ub = u + (long)b * g.nvp * g.ncp;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < g.nvc; i += (long)gridDim.x * blockDim.x) {
    const int v = (int)i / g.nc, c = (int)i - v * g.nc;  // (N_v N_c < 2^31)
    ub[(long)v * g.ncp + c] = to_op<U>(g.uscale * (g.tda ? xb[i] : g.sdelta[i] * xb[i]));
  }
}

template <typename T> struct Two;
template <> struct Two<float> { typedef float2 T; };
template <> struct Two<double> { typedef double2 T; };
template <typename U> struct TwoOp;
template <> struct TwoOp<double> {
  typedef double2 T;
  __device__ static T make(double a, double b) { return T{a, b}; }
};
template <> struct TwoOp<f16_t> {
  struct T { f16_t a, b; };
  __device__ static T make(double a, double b) { return T{to_op<f16_t>(a), to_op<f16_t>(b)}; }
};

// The same per element as the loop below, two consecutive elements of one
// occupied row per thread with 8- and 16-byte accesses (N_c even, every
// pointer 16-byte aligned: checked on the host).
template <typename Y, typename U>
__device__ inline void combine_pairs(const PairGeom& g, int b, long stride_s, const Y* yb,
                                     const double* xb, long obase, int splitk,
                                     const double* __restrict__ tp, double* __restrict__ out,
                                     double* __restrict__ acc, int mode, double lo, double hi,
                                     double inv, double ysc, double c0, double cj,
                                     U* __restrict__ u, double* __restrict__ kx_out) {
  const long n2 = g.nvc >> 1;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n2; p += (long)gridDim.x * blockDim.x) {
    const int i = 2 * (int)p;
    const int v = i / g.nc, c = i - v * g.nc;  // c even: both elements in row v
    const long off = (long)v * g.ncp + c;
    double y0 = 0.0, y1 = 0.0;
    for (int s = 0; s < splitk; ++s) {
      const typename Two<Y>::T t = *reinterpret_cast<const typename Two<Y>::T*>(yb + s * stride_s + off);
      y0 += (double)t.x;
      y1 += (double)t.y;
    }
    y0 *= ysc;
    y1 *= ysc;
    const double2 xi = as_d2(xb)[p];
    const long o = obase + i;
    if (mode == 3) {  // A x = Delta x + K x
      const double2 dl = as_d2(g.delta)[p];
      as_d2(out + o)[0] = double2{dl.x * xi.x + g.dv * y0, dl.y * xi.y + g.dv * y1};
      continue;
    }
    const double2 sd = as_d2(g.sdelta)[p], d2 = as_d2(g.delta2)[p];
    const double cx0 = d2.x * xi.x + 2.0 * g.dv * sd.x * y0;
    const double cx1 = d2.y * xi.y + 2.0 * g.dv * sd.y * y1;
    if (kx_out) as_d2(kx_out + o)[0] = double2{g.dv * y0, g.dv * y1};
    if (mode == 0) {
      as_d2(out + o)[0] = double2{cx0, cx1};
      continue;
    }
    const double ct0 = (2.0 * cx0 - (hi + lo) * xi.x) * inv;
    const double ct1 = (2.0 * cx1 - (hi + lo) * xi.y) * inv;
    double tn0, tn1;
    if (mode == 1) {
      tn0 = ct0;
      tn1 = ct1;
      as_d2(acc + o)[0] = double2{c0 * xi.x + cj * tn0, c0 * xi.y + cj * tn1};
    } else {
      const double2 tq = as_d2(tp + o)[0];
      tn0 = 2.0 * ct0 - tq.x;
      tn1 = 2.0 * ct1 - tq.y;
      double2 a = as_d2(acc + o)[0];
      a.x += cj * tn0;
      a.y += cj * tn1;
      as_d2(acc + o)[0] = a;
    }
    as_d2(out + o)[0] = double2{tn0, tn1};
    if (u)
      *reinterpret_cast<typename TwoOp<U>::T*>(u + (long)b * g.nvp * g.ncp + off) =
          TwoOp<U>::make(g.uscale * sd.x * tn0, g.uscale * sd.y * tn1);
  }
}

template <typename Y, typename U>
__global__ void combine_kernel(PairGeom g, int nb, int splitk, const Y* __restrict__ ypart,
                               const double* __restrict__ x, const double* __restrict__ tp,
                               double* __restrict__ out, double* __restrict__ acc, int mode,
                               double lo, double hi, double c0, double cj, U* __restrict__ u,
                               double* __restrict__ kx_out, int pairs) {
  const int b = blockIdx.y;
  const int slot = g.rows ? g.rows[b] : b;
  const long stride_s = (long)nb * g.nvp * g.ncp;
  const Y* yb = ypart + (long)b * g.nvp * g.ncp;
  const double* xb = x + (long)slot * g.nvc;
  const double inv = 1.0 / (hi - lo);
  // the potential's scale of the mixed product is divided out with the others
  const double ysc = g.vexp ? ldexp(g.yscale, -g.vexp[b]) : g.yscale;
  if (pairs) {
    combine_pairs<Y, U>(g, b, stride_s, yb, xb, (long)slot * g.nvc, splitk, tp, out, acc, mode,
                        lo, hi, inv, ysc, c0, cj, u, kx_out);
    return;
  }
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < g.nvc; i += (long)gridDim.x * blockDim.x) {
    const int v = (int)i / g.nc, c = (int)i - v * g.nc;  // (N_v N_c < 2^31)
    const long off = (long)v * g.ncp + c;
    double y = 0.0;
    for (int s = 0; s < splitk; ++s) y += (double)yb[s * stride_s + off];
    y *= ysc;
    const double xi = xb[i];
    const long o = (long)slot * g.nvc + i;
    if (mode == 3) {  // A x = Delta x + K x
      out[o] = g.delta[i] * xi + g.dv * y;
      continue;
    }
    const double sd = g.sdelta[i];
    const double cx = g.delta2[i] * xi + 2.0 * g.dv * sd * y;
    if (kx_out) kx_out[o] = g.dv * y;  // K Delta^1/2 x
    if (mode == 0) {
      out[o] = cx;
      continue;
    }
    const double ct = (2.0 * cx - (hi + lo) * xi) * inv;
    double tn;
    if (mode == 1) {
      tn = ct;
      acc[o] = c0 * xi + cj * tn;
    } else {
      tn = 2.0 * ct - tp[o];
      acc[o] += cj * tn;
    }
    out[o] = tn;
    if (u) u[(long)b * g.nvp * g.ncp + off] = to_op<U>(g.uscale * sd * tn);
  }
}

template <typename Y>
__global__ void coupling_finish_kernel(PairGeom g, int cnt, int splitk, const Y* __restrict__ ypart,
                                       double* __restrict__ p, long ldp) {
  const int i = blockIdx.y;
  const long stride_s = (long)cnt * g.nvp * g.ncp;
  const Y* yb = ypart + (long)i * g.nvp * g.ncp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < g.nvc; e += (long)gridDim.x * blockDim.x) {
    const int v = (int)e / g.nc, c = (int)e - v * g.nc;  // (N_v N_c < 2^31)
    const long off = (long)v * g.ncp + c;
    double y = 0.0;
    for (int s = 0; s < splitk; ++s) y += (double)yb[s * stride_s + off];
    // P_nm = (nm|vc) Delta^1/2, or (nm|vc) itself for Tamm-Dancoff
    p[(long)i * ldp + e] = g.tda ? g.dv * y : g.dv * g.sdelta[e] * y;
  }
}

__device__ inline bool slot_active(const SlotState& s, int b) {
  return s.pair[b] >= 0 && !s.dead[b] && s.k[b] < s.len[b];
}

__global__ void __launch_bounds__(NT)
lz_start_kernel(SlotState s, const int* __restrict__ slot_list, double* __restrict__ q,
                double* __restrict__ qprev, double* __restrict__ basis, long bstride, long nvc) {
  __shared__ double sh[NT / 64];
  const int b = slot_list[blockIdx.x];
  const int pair = s.pair[b];
  double* qb = q + (long)b * nvc;
  double part = 0.0;
  for (long i = threadIdx.x; i < nvc; i += NT) part += qb[i] * qb[i];
  const double n2 = block_sum(part, sh);
  const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  double* pb = qprev + (long)b * nvc;
  double* bb = basis ? basis + (long)b * bstride : nullptr;
  for (long i = threadIdx.x; i < nvc; i += NT) {
    const double v = qb[i] * inv;
    qb[i] = v;
    pb[i] = 0.0;
    if (bb) bb[i] = v;
  }
  if (threadIdx.x == 0) {
    s.norm2[pair] = n2;
    s.k[b] = 0;
    s.dead[b] = (n2 > 0.0) ? 0 : 1;
    s.amax[b] = 0.0;
    s.bprev[b] = 0.0;
    s.out_len[pair] = 0;
  }
}

__global__ void __launch_bounds__(NTS)
lz_alpha_kernel(SlotState s, const double* __restrict__ q, const double* __restrict__ qprev,
                double* __restrict__ w, long nvc) {
  __shared__ double sh[NTS / 64];
  const int b = blockIdx.x;
  if (!slot_active(s, b)) return;
  const double* qb = q + (long)b * nvc;
  const double* pb = qprev + (long)b * nvc;
  double* wb = w + (long)b * nvc;
  const bool pairs = (nvc & 1) == 0;
  const long n2 = nvc >> 1;
  double part = 0.0;
  if (pairs) {
    for (long i = threadIdx.x; i < n2; i += NTS) {
      const double2 x = as_d2(qb)[i], y = as_d2(wb)[i];
      part += x.x * y.x;
      part += x.y * y.y;
    }
  } else {
    for (long i = threadIdx.x; i < nvc; i += NTS) part += qb[i] * wb[i];
  }
  const double a = block_sum(part, sh);
  const double bp = s.bprev[b];
  if (pairs) {
    for (long i = threadIdx.x; i < n2; i += NTS) {
      const double2 x = as_d2(qb)[i], y = as_d2(pb)[i];
      double2 z = as_d2(wb)[i];
      z.x = z.x - a * x.x - bp * y.x;
      z.y = z.y - a * x.y - bp * y.y;
      as_d2(wb)[i] = z;
    }
  } else {
    for (long i = threadIdx.x; i < nvc; i += NTS) wb[i] = wb[i] - a * qb[i] - bp * pb[i];
  }
  if (threadIdx.x == 0) {
    const int pair = s.pair[b], k = s.k[b];
    s.coef_a[(long)pair * s.ld + k] = a;
    s.amax[b] = fmax(s.amax[b], fabs(a));
    s.out_len[pair] = k + 1;
  }
}

__device__ inline bool needs_beta(const SlotState& s, int b) {
  return slot_active(s, b) && s.k[b] < s.len[b] - 1;
}

// h[b][j] = basis_j . w  (FULL: j <= k; LOCAL: j in {k-1, k} read from q, qprev).
// skip (optional): slots whose second pass is not needed; wn0 (optional):
// ||w||^2 before the pass, from the j = 0 block.
__global__ void __launch_bounds__(NT)
lz_dots_kernel(SlotState s, int mode, const double* __restrict__ basis, long bstride,
               const double* __restrict__ q, const double* __restrict__ qprev,
               const double* __restrict__ w, double* __restrict__ h, int hld, long nvc,
               const int* __restrict__ skip, double* __restrict__ wn0) {
  __shared__ double sh[NT / 64];
  const int j = blockIdx.x, b = blockIdx.y;
  if (!needs_beta(s, b)) return;
  if (skip && skip[b]) return;
  const int k = s.k[b];
  const double* vb;
  if (mode == GWL_REORTH_FULL) {
    if (j > k) return;
    vb = basis + (long)b * bstride + (long)j * nvc;
  } else {
    if (j > 1 || (j == 1 && k == 0)) {
      if (threadIdx.x == 0) h[(long)b * hld + j] = 0.0;
      return;
    }
    vb = (j == 0 ? q : qprev) + (long)b * nvc;
  }
  const double* wb = w + (long)b * nvc;
  double part = 0.0, ww = 0.0;
  const bool norm = wn0 && j == 0;
  if ((nvc & 1) == 0) {
    const long n2 = nvc >> 1;
    double p1 = 0.0;
#pragma unroll 4
    for (long i = threadIdx.x; i < n2; i += NT) {
      const double2 x = as_d2(wb)[i], y = as_d2(vb)[i];
      part += y.x * x.x;
      p1 += y.y * x.y;
      if (norm) ww += x.x * x.x + x.y * x.y;
    }
    part += p1;
  } else {
    for (long i = threadIdx.x; i < nvc; i += NT) {
      const double x = wb[i];
      part += vb[i] * x;
      if (norm) ww += x * x;
    }
  }
  const double t = block_sum(part, sh);
  if (threadIdx.x == 0) h[(long)b * hld + j] = t;
  if (norm) {
    const double n2 = block_sum(ww, sh);
    if (threadIdx.x == 0) wn0[b] = n2;
  }
}

// w -= sum_j h[b][j] basis_j; part (optional): per-block ||w_new||^2 partial
// sums [nb][gridDim.x]
__global__ void __launch_bounds__(NT)
lz_project_kernel(SlotState s, int mode, const double* __restrict__ basis, long bstride,
                  const double* __restrict__ q, const double* __restrict__ qprev,
                  double* __restrict__ w, const double* __restrict__ h, int hld, long nvc,
                  const int* __restrict__ skip, double* __restrict__ part) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.y;
  if (!needs_beta(s, b)) return;
  if (skip && skip[b]) return;
  const int k = s.k[b];
  const double* hb = h + (long)b * hld;
  double* wb = w + (long)b * nvc;
  double ww = 0.0;
  if ((nvc & 1) == 0) {
    const long n2 = nvc >> 1;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n2;
         i += (long)gridDim.x * blockDim.x) {
      double2 acc = {0.0, 0.0};
      if (mode == GWL_REORTH_FULL) {
        const double2* bb = as_d2(basis + (long)b * bstride) + i;
#pragma unroll 4
        for (int j = 0; j <= k; ++j) {
          const double2 v = bb[(long)j * n2];
          acc.x += hb[j] * v.x;
          acc.y += hb[j] * v.y;
        }
      } else {
        const double2 v = as_d2(q + (long)b * nvc)[i];
        acc.x = hb[0] * v.x;
        acc.y = hb[0] * v.y;
        if (k > 0) {
          const double2 u = as_d2(qprev + (long)b * nvc)[i];
          acc.x += hb[1] * u.x;
          acc.y += hb[1] * u.y;
        }
      }
      double2 x = as_d2(wb)[i];
      x.x -= acc.x;
      x.y -= acc.y;
      as_d2(wb)[i] = x;
      ww += x.x * x.x;
      ww += x.y * x.y;
    }
  } else {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nvc;
         i += (long)gridDim.x * blockDim.x) {
      double acc = 0.0;
      if (mode == GWL_REORTH_FULL) {
        const double* bb = basis + (long)b * bstride + i;
        for (int j = 0; j <= k; ++j) acc += hb[j] * bb[(long)j * nvc];
      } else {
        acc = hb[0] * q[(long)b * nvc + i];
        if (k > 0) acc += hb[1] * qprev[(long)b * nvc + i];
      }
      const double x = wb[i] - acc;
      wb[i] = x;
      ww += x * x;
    }
  }
  if (part) {
    const double t = block_sum(ww, sh);
    if (threadIdx.x == 0) part[(long)b * gridDim.x + blockIdx.x] = t;
  }
}

// Second-pass test (Daniel, Gragg, Kaufman and Stewart): the first pass
// removed little of w when ||w_1||^2 >= ||w_0||^2 / 2, and a second pass
// would change it only at rounding level, so it is skipped.  Partial sums in
// a fixed order.
__global__ void __launch_bounds__(NT)
lz_dgks_kernel(SlotState s, const double* __restrict__ part, int nblk,
               const double* __restrict__ wn0, int* __restrict__ skip) {
  __shared__ double sh[NT / 64];
  const int b = blockIdx.x;
  if (!needs_beta(s, b)) {
    if (threadIdx.x == 0) skip[b] = 1;
    return;
  }
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += NT) v += part[(long)b * nblk + i];
  const double n1 = block_sum(v, sh);
  if (threadIdx.x == 0) skip[b] = (n1 >= 0.5 * wn0[b]) ? 1 : 0;
}

__global__ void __launch_bounds__(NTS)
lz_beta_kernel(SlotState s, double* __restrict__ q, double* __restrict__ qprev,
               double* __restrict__ w, double* __restrict__ basis, long bstride,
               int store_basis, long nvc) {
  __shared__ double sh[NTS / 64];
  const int b = blockIdx.x;
  if (!slot_active(s, b)) return;
  const int k = s.k[b];
  if (k >= s.len[b] - 1) {
    __syncthreads();
    if (threadIdx.x == 0) s.k[b] = k + 1;
    return;
  }
  double* wb = w + (long)b * nvc;
  const bool pairs = (nvc & 1) == 0;
  const long n2 = nvc >> 1;
  double part = 0.0;
  if (pairs) {
    for (long i = threadIdx.x; i < n2; i += NTS) {
      const double2 x = as_d2(wb)[i];
      part += x.x * x.x;
      part += x.y * x.y;
    }
  } else {
    for (long i = threadIdx.x; i < nvc; i += NTS) part += wb[i] * wb[i];
  }
  const double bn = sqrt(block_sum(part, sh));
  const int pair = s.pair[b];
  if (!(bn > 1e-12 * s.amax[b])) {
    // exact invariant subspace (or non-finite norm): the fraction ends here
    if (threadIdx.x == 0) {
      s.dead[b] = 1;
      s.k[b] = k + 1;
    }
    return;
  }
  const double inv = 1.0 / bn;
  double* qb = q + (long)b * nvc;
  double* pb = qprev + (long)b * nvc;
  double* bb = store_basis ? basis + (long)b * bstride + (long)(k + 1) * nvc : nullptr;
  if (pairs) {
    for (long i = threadIdx.x; i < n2; i += NTS) {
      const double2 x = as_d2(wb)[i];
      const double2 nq = {x.x * inv, x.y * inv};
      as_d2(pb)[i] = as_d2(qb)[i];
      as_d2(qb)[i] = nq;
      if (bb) as_d2(bb)[i] = nq;
    }
  } else {
    for (long i = threadIdx.x; i < nvc; i += NTS) {
      const double nq = wb[i] * inv;
      pb[i] = qb[i];
      qb[i] = nq;
      if (bb) bb[i] = nq;
    }
  }
  if (threadIdx.x == 0) {
    s.coef_b[(long)pair * s.ld + k] = bn;
    s.bprev[b] = bn;
    s.k[b] = k + 1;
  }
}

inline int grid_elems(long n) {
  long g = (n + NT - 1) / NT;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// dst[2i] = a_i + b_i, dst[2i + 1] = a_i - b_i (rows of length n)
__global__ void polar_rows_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                  long n, double* __restrict__ dst) {
  const int i = blockIdx.y;
  const double* ai = a + (long)i * n;
  const double* bi = b + (long)i * n;
  double* dp = dst + (long)(2 * i) * n;
  double* dm = dp + n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    dp[e] = ai[e] + bi[e];
    dm[e] = ai[e] - bi[e];
  }
}

void polar_rows(const double* a, const double* b, long n, int cnt, double* dst, hipStream_t st) {
  if (cnt <= 0) return;
  polar_rows_kernel<<<dim3(grid_elems(n), cnt), NT, 0, st>>>(a, b, n, dst);
  GWL_HIP(hipGetLastError());
}

void pair_product(const double* psi_t, long ld, int nr, const int* m_idx, const int* n_idx,
                  int cnt, double* rho, hipStream_t st) {
  if (cnt <= 0) return;
  dim3 grid(grid_elems(ld), cnt);
  pair_product_kernel<<<grid, NT, 0, st>>>(psi_t, ld, nr, m_idx, n_idx, rho);
  GWL_HIP(hipGetLastError());
}

// out[i] = dv sum_{r < nr} rho_i(r) V_i(r), fixed reduction order.
__global__ void pair_energy_kernel(const double* __restrict__ rho, const double* __restrict__ vpot,
                                   long ld, int nr, double dv, double* __restrict__ out) {
  __shared__ double red[NT];
  const double* a = rho + (long)blockIdx.x * ld;
  const double* b = vpot + (long)blockIdx.x * ld;
  double acc = 0.0;
  for (long i = threadIdx.x; i < nr; i += blockDim.x) acc += a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = dv * red[0];
}

void pair_energy(const double* rho, const double* vpot, long ld, int nr, double dv, int cnt,
                 double* out, hipStream_t st) {
  if (cnt <= 0) return;
  pair_energy_kernel<<<cnt, NT, 0, st>>>(rho, vpot, ld, nr, dv, out);
  GWL_HIP(hipGetLastError());
}

__global__ void row_norm2_kernel(const double* __restrict__ x, long n, double* __restrict__ out) {
  __shared__ double red[NT];
  const double* xr = x + (long)blockIdx.x * n;
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) acc += xr[i] * xr[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

void row_norm2(const double* x, long n, int nrows, double* out, hipStream_t st) {
  if (nrows <= 0) return;
  row_norm2_kernel<<<nrows, NT, 0, st>>>(x, n, out);
  GWL_HIP(hipGetLastError());
}

template <typename U>
void cast_u(const PairGeom& g, int nb, const double* x, long ldx, U* u, hipStream_t st) {
  if (nb <= 0) return;
  dim3 grid(grid_elems(g.nvc), nb);
  cast_u_kernel<U><<<grid, NT, 0, st>>>(g, x, ldx, u);
  GWL_HIP(hipGetLastError());
}
template void cast_u<double>(const PairGeom&, int, const double*, long, double*, hipStream_t);
template void cast_u<f16_t>(const PairGeom&, int, const double*, long, f16_t*, hipStream_t);

template <typename Y, typename U>
void combine(const PairGeom& g, int nb, int splitk, const Y* ypart, const double* x,
             const double* tp, double* out_tn, double* acc, int mode, double lo, double hi,
             double c0, double cj, U* u, hipStream_t st, double* kx_out) {
  if (nb <= 0) return;
  // element pairs when every row of every operand starts 16 bytes apart
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool pairs = (g.nc % 2 == 0) && al(ypart) && al(x) && al(tp) && al(out_tn) && al(acc) &&
                     al(u) && al(kx_out) && al(g.delta2) && al(g.sdelta) && al(g.delta);
  dim3 grid(grid_elems(pairs ? g.nvc / 2 : g.nvc), nb);
  combine_kernel<Y, U><<<grid, NT, 0, st>>>(g, nb, splitk, ypart, x, tp, out_tn, acc, mode, lo,
                                            hi, c0, cj, u, kx_out, pairs ? 1 : 0);
  GWL_HIP(hipGetLastError());
}
template void combine<double, double>(const PairGeom&, int, int, const double*, const double*,
                                      const double*, double*, double*, int, double, double,
                                      double, double, double*, hipStream_t, double*);
template void combine<float, f16_t>(const PairGeom&, int, int, const float*, const double*,
                                    const double*, double*, double*, int, double, double,
                                    double, double, f16_t*, hipStream_t, double*);

template <typename Y>
void coupling_finish(const PairGeom& g, int cnt, int splitk, const Y* ypart, double* p_out,
                     long ldp, hipStream_t st) {
  if (cnt <= 0) return;
  dim3 grid(grid_elems(g.nvc), cnt);
  coupling_finish_kernel<Y><<<grid, NT, 0, st>>>(g, cnt, splitk, ypart, p_out, ldp);
  GWL_HIP(hipGetLastError());
}
template void coupling_finish<double>(const PairGeom&, int, int, const double*, double*, long,
                                      hipStream_t);
template void coupling_finish<float>(const PairGeom&, int, int, const float*, double*, long,
                                     hipStream_t);

void lz_start(const SlotState& s, int nb_slots, const int* slot_list, int cnt, double* q,
              double* qprev, double* basis, long bstride, long nvc, hipStream_t st) {
  (void)nb_slots;
  if (cnt <= 0) return;
  lz_start_kernel<<<cnt, NT, 0, st>>>(s, slot_list, q, qprev, basis, bstride, nvc);
  GWL_HIP(hipGetLastError());
}

void lz_alpha(const SlotState& s, int nb, const double* q, const double* qprev, double* w,
              long nvc, hipStream_t st) {
  lz_alpha_kernel<<<nb, NTS, 0, st>>>(s, q, qprev, w, nvc);
  GWL_HIP(hipGetLastError());
}

void lz_reorth(const SlotState& s, int nb, int kmax, int mode, const double* basis,
               long bstride, const double* q, const double* qprev, double* w, double* hbuf,
               const ReorthScratch& rs, long nvc, hipStream_t st) {
  if (mode == GWL_REORTH_NONE) return;
  const bool full = (mode == GWL_REORTH_FULL);
  const int nd = full ? kmax + 1 : 2;
  const int hld = full ? s.ld + 1 : 2;
  // (the projection runs over element pairs when N_v N_c is even; the
  // partial-norm buffer holds grid_elems(nvc) entries per slot)
  const int ge = grid_elems((nvc & 1) == 0 ? nvc / 2 : nvc);
  // FULL: classical Gram-Schmidt, the second pass only where the first
  // removed more than half of ||w||^2; LOCAL: always two passes
  lz_dots_kernel<<<dim3(nd, nb), NT, 0, st>>>(s, mode, basis, bstride, q, qprev, w, hbuf, hld,
                                              nvc, nullptr, full ? rs.wn0 : nullptr);
  lz_project_kernel<<<dim3(ge, nb), NT, 0, st>>>(s, mode, basis, bstride, q, qprev, w, hbuf,
                                                 hld, nvc, nullptr, full ? rs.part : nullptr);
  if (full) lz_dgks_kernel<<<nb, NT, 0, st>>>(s, rs.part, ge, rs.wn0, rs.skip);
  const int* sk = full ? rs.skip : nullptr;
  lz_dots_kernel<<<dim3(nd, nb), NT, 0, st>>>(s, mode, basis, bstride, q, qprev, w, hbuf, hld,
                                              nvc, sk, nullptr);
  lz_project_kernel<<<dim3(ge, nb), NT, 0, st>>>(s, mode, basis, bstride, q, qprev, w, hbuf,
                                                 hld, nvc, sk, nullptr);
  GWL_HIP(hipGetLastError());
}

long reorth_part_len(long nvc) { return grid_elems(nvc); }

void lz_beta(const SlotState& s, int nb, double* q, double* qprev, double* w, double* basis,
             long bstride, int store_basis, long nvc, hipStream_t st) {
  lz_beta_kernel<<<nb, NTS, 0, st>>>(s, q, qprev, w, basis, bstride, store_basis, nvc);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
