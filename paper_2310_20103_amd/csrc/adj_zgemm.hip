// Orbital gradient of the coupling part of C, factored (no N_vc x N_vc
// cotangent, no per-pair potentials on the grid).
//
// The coupling block of C (Eq. 4) is 2 Delta^1/2 K Delta^1/2 with
// K_{vc,v'c'} = dV sum_r phi_v phi_c(r) V[phi_v' phi_c'](r) (Eqs. 2-3).  The
// reverse Chebyshev sweep gives the cotangent of C as a sum of outer products
// s t^T of pair vectors; for each of them the derivative of
// s^T Delta^1/2 K Delta^1/2 t with respect to the orbital grid values is
//   d/dphi_v(r) = dV sum_c phi_c(r) Z(r, v, c),
//   d/dphi_c(r) = dV sum_v phi_v(r) Z(r, v, c),
//   Z(r, v, c)  = sum_k V_k(r) U_k(v, c),
// with the pairs (U_k, V_k) = (Delta^1/2 s, V[rho of Delta^1/2 t]) and
// (Delta^1/2 t, V[rho of Delta^1/2 s]); the potentials are the ones the FFT
// Poisson solve already produced inside the forward and reverse products.
// The same form covers the coupling integrals (nm|vc) of the start vectors,
// with U = k_bar and V = V[phi_n phi_m].
//
// One kernel computes Z tile by tile on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64) and contracts each tile at once, so Z never
// reaches memory: a block owns 64 conduction indices c and 128 grid points r
// and walks the occupied indices two at a time, K over all outer products of
// the launch; each wave holds both occupied indices of a pair for half the
// block's c.  The conduction gradient is added to its grid row in place after
// every pair (each element has one owner, one wave of one block, so the
// additions run in a fixed order), which keeps the kernel at two waves per
// SIMD; the occupied gradient of the block's 64 c is written as a partial sum
// per c tile and reduced in fixed order at the end, so runs are bitwise
// reproducible.
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int ZM = 128;       // rows: 2 occupied x 64 conduction indices
constexpr int ZN = 128;       // columns: grid points
constexpr int ZK = 16;        // K step
constexpr int ZLD = ZM + 4;   // LDS row of one k (doubles)
constexpr int NT = 256;

__device__ inline int xcd_remap_z(int bid, int total) {
  if (total % 8 != 0) return bid;
  return (bid & 7) * (total >> 3) + (bid >> 3);
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2)))
zgemm_kernel(GemmDims d, int nv, ZSeg s0, ZSeg s1, const double* __restrict__ psi_c_rc,
             const double* __restrict__ psi_v_rv, double dv, double* __restrict__ grad_c,
             double* __restrict__ gvpart) {
  // one operand tile pair [ZK][ZLD] during the K loop; the exchange of the
  // occupied-gradient halves between the wave pairs after it
  __shared__ double As[ZK][ZLD];
  __shared__ double Bs[ZK][ZLD];
  __shared__ double xs[2][ZN];
  const int nct = d.ncp / 64, nrt = d.nrp / ZN;
  const int lid = xcd_remap_z(blockIdx.x, nct * nrt);
  const int rt = lid / nct, ct = lid - rt * nct;
  const int r0 = rt * ZN, c0 = ct * 64;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int K = s0.k + s1.k;
  // loader: k row lk of the step, 8 consecutive doubles at column lm
  // (columns: 64 conduction indices of v0, then 64 of v0 + 1)
  const int lk = t >> 4, lm = (t & 15) * 8;
  const int lvo = lm >> 6, lc = c0 + (lm & 63);
  const long ld_u = (long)d.nvp * d.ncp;
  // wave (wm, wn) computes Z for both v of the pair, conduction indices
  // c0 + 32 wm + [0, 32), grid points r0 + 64 wn + [0, 64): MFMA row block i
  // is v offset i >> 1, conduction offset 32 wm + 16 (i & 1)
  int acol[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acol[i] = (i >> 1) * 64 + wm * 32 + 16 * (i & 1) + (l & 15);

  for (int v0 = 0; v0 < nv; v0 += 2) {
    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = d4{0, 0, 0, 0};
    const int lv = v0 + lvo;
    double ra[8], rb[8];
    auto gload = [&](int k0) {
      const int k = k0 + lk;
      const double* up = nullptr;
      const double* vp = nullptr;
      if (k < s0.k) {
        up = s0.u + (long)k * ld_u;
        vp = s0.vf + (long)k * d.nrp;
      } else if (k < K) {
        up = s1.u + (long)(k - s0.k) * ld_u;
        vp = s1.vf + (long)(k - s0.k) * d.nrp;
      }
      if (up && lv < nv) {
        const double* p = up + (long)lv * d.ncp + lc;
#pragma unroll
        for (int i = 0; i < 8; ++i) ra[i] = p[i];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) ra[i] = 0.0;
      }
      if (vp) {
        const double* p = vp + r0 + lm;
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[i] = p[i];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[i] = 0.0;
      }
    };
    auto lstore = [&]() {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        As[lk][lm + i] = ra[i];
        Bs[lk][lm + i] = rb[i];
      }
    };
    gload(0);
    __syncthreads();  // the previous pair's epilogue has read xs
    lstore();
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += ZK) {
      const bool more = k0 + ZK < K;
      if (more) gload(k0 + ZK);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int kk = 4 * ks + (l >> 4);
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = As[kk][acol[i]];
          b[i] = Bs[kk][wn * 64 + 16 * i + (l & 15)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
      if (more) {
        lstore();
        __syncthreads();
      }
    }
    // epilogue of the pair: acc[i][j][q] is Z at v = v0 + (i >> 1),
    // c = c0 + 32 wm + 16 (i & 1) + (l >> 4) + 4 q, r = r0 + 64 wn + 16 j + (l & 15).
    // Conduction gradient: dV (phi_v0 Z_v0 + phi_v0+1 Z_v0+1) added in place
    // (every element of grad_c has one owner: this block, this wave), pair
    // after pair.  Occupied gradient: each wave sums its 32 c, the two halves
    // meet through LDS and go to this c tile's partial row.
    double sv[2][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + wn * 64 + 16 * j + (l & 15);
      // (v0 + 1 < N_vp: N_vp is a multiple of 64 and v0 is even; padded rows are zero)
      const double pv0 = psi_v_rv[(long)r * d.nvp + v0];
      const double pv1 = psi_v_rv[(long)r * d.nvp + v0 + 1];
      const double* wc = psi_c_rc + (long)r * d.ncp + c0 + wm * 32 + (l >> 4);
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double z0 = acc[i2][j][q], z1 = acc[2 + i2][j][q];
          const double cw = wc[16 * i2 + 4 * q];
          a0 += cw * z0;
          a1 += cw * z1;
          double* o = grad_c + (long)(c0 + wm * 32 + 16 * i2 + (l >> 4) + 4 * q) * d.nrp + r;
          *o += dv * (pv0 * z0 + pv1 * z1);
        }
      a0 += __shfl_xor(a0, 16, 64);
      a0 += __shfl_xor(a0, 32, 64);
      a1 += __shfl_xor(a1, 16, 64);
      a1 += __shfl_xor(a1, 32, 64);
      sv[0][j] = a0;
      sv[1][j] = a1;
      // one j at a time: hoisting the loads of all four next to the
      // accumulators would exceed the register budget of two waves per SIMD
      __builtin_amdgcn_sched_barrier(0);
    }
    if (wm == 1 && l < 16) {
#pragma unroll
      for (int vo = 0; vo < 2; ++vo)
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[vo][wn * 64 + 16 * j + l] = sv[vo][j];
    }
    __syncthreads();
    if (wm == 0 && l < 16) {
#pragma unroll
      for (int vo = 0; vo < 2; ++vo) {
        const int v = v0 + vo;
        if (v >= nv) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rl = wn * 64 + 16 * j + l;
          double* o = gvpart + ((long)ct * nv + v) * d.nrp + r0 + rl;
          *o += dv * (sv[vo][j] + xs[vo][rl]);
        }
      }
    }
  }
}

// grad_v[v][r] += sum over c tiles (in order) of gvpart[ct][v][r]
__global__ void gv_reduce_kernel(const double* __restrict__ gvpart, int nct, int nv, long nrp,
                                 double* __restrict__ grad_v) {
  const long n = (long)nv * nrp;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    double s = grad_v[e];
    for (int ct = 0; ct < nct; ++ct) s += gvpart[(long)ct * n + e];
    grad_v[e] = s;
  }
}

// Per Chebyshev term j: Delta_bar += alpha [2 Delta s t + (s K~t + t K~s)/Delta^1/2];
// U_s = kappa Delta^1/2 s and U_t = kappa Delta^1/2 t into the padded
// [nb][N_vp][N_cp] layout (pads are never written and stay zero).
__global__ void dbar_zops_kernel(PairGeom g, const double* __restrict__ s,
                                 const double* __restrict__ ks, const double* __restrict__ t,
                                 const double* __restrict__ kt, double alpha, double kappa,
                                 double* __restrict__ dbar, double* __restrict__ us,
                                 double* __restrict__ ut) {
  const int b = blockIdx.y;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < g.nvc; i += (long)gridDim.x * blockDim.x) {
    const long o = (long)b * g.nvc + i;
    const int v = (int)i / g.nc, c = (int)i - v * g.nc;  // (N_v N_c < 2^31)
    const long op = ((long)b * g.nvp + v) * g.ncp + c;
    const double sd = g.sdelta[i];
    const double si = s[o], ti = t[o];
    dbar[o] += alpha * (2.0 * sd * sd * si * ti + (si * kt[o] + ti * ks[o]) / sd);
    us[op] = kappa * sd * si;
    ut[op] = kappa * sd * ti;
  }
}

inline int gelems(long n) {
  long g = (n + NT - 1) / NT;
  return (int)(g > 2048 ? 2048 : (g < 1 ? 1 : g));
}

}  // namespace

void adj_zgemm(const GemmDims& d, int nv, const ZSeg& s0, const ZSeg& s1, const double* psi_c_rc,
               const double* psi_v_rv, double dv, double* grad_c, double* gvpart,
               hipStream_t st) {
  if (s0.k + s1.k <= 0 || nv <= 0) return;
  GWL_CHECK(d.ncp % 64 == 0 && d.nrp % ZN == 0, GWL_EINVAL, "adjoint tile layout");
  const int blocks = (d.ncp / 64) * (d.nrp / ZN);
  zgemm_kernel<<<blocks, NT, 0, st>>>(d, nv, s0, s1, psi_c_rc, psi_v_rv, dv, grad_c, gvpart);
  GWL_HIP(hipGetLastError());
}

void adj_gv_reduce(const double* gvpart, int nct, int nv, long nrp, double* grad_v,
                   hipStream_t st) {
  if (nv <= 0) return;
  gv_reduce_kernel<<<gelems((long)nv * nrp), NT, 0, st>>>(gvpart, nct, nv, nrp, grad_v);
  GWL_HIP(hipGetLastError());
}

void adj_dbar_zops(const PairGeom& g, int nb, const double* s, const double* ks, const double* t,
                   const double* kt, double alpha, double kappa, double* dbar, double* us,
                   double* ut, hipStream_t st) {
  dim3 grid(gelems(g.nvc), nb);
  dbar_zops_kernel<<<grid, NT, 0, st>>>(g, s, ks, t, kt, alpha, kappa, dbar, us, ut);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
