// Factored pair-space product, plain LDS-tiled FMA version (FP64, and the
// mixed path's FP16 operands with FP32 accumulation).  The MFMA kernels
// are checked against it.
//
// First GEMM with fused row-dot (the density of a pair vector u = Delta^1/2 x):
//   rho_b(r) = sum_v phi_v(r) sum_c phi_c(r) u_b[v, c]
// Second GEMM (the Hartree integrals back into pair space):
//   y_b[v, c] = sum_r phi_v(r) V_b(r) phi_c(r)
// (the two halves of K applied through the grid, Eqs. 2-4).
//
// Tiles: 64 x 64 outputs per 256-thread block, 4 x 4 per thread, K step 16.
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, LDT = 64 + 1;

__device__ inline double ldx(const double* p, long i) { return p[i]; }
__device__ inline float ldx(const bf16_t* p, long i) { return bf16_to_f32(p[i]); }
__device__ inline float ldx(const f16_t* p, long i) { return f16_to_f32(p[i]); }
__device__ inline float ldx(const float* p, long i) { return p[i]; }

// A = accumulation type (double or float); TO = operand storage; TW = weights.
template <typename A, typename TO, typename TW>
__global__ void __launch_bounds__(256)
gemm1_simple_kernel(GemmDims d, const TO* __restrict__ psi_c_rc,
                 const TW* __restrict__ psi_v_rv, const TO* __restrict__ u,
                 A* __restrict__ rho_part, int nb) {
  __shared__ A As[TK][LDT];
  __shared__ A Bs[TK][LDT];
  __shared__ A red[16][TM + 1];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tv = tid >> 4;
  const int r0 = blockIdx.x * TM, v0 = blockIdx.y * TN, b = blockIdx.z;
  const TO* ub = u + (long)b * d.nvp * d.ncp;
  A acc[4][4] = {};
  for (int c0 = 0; c0 < d.ncp; c0 += TK) {
    for (int e = tid; e < TK * TM; e += 256) {
      const int kk = e & (TK - 1), i = e >> 4;
      As[kk][i] = ldx(psi_c_rc, (long)(r0 + i) * d.ncp + c0 + kk);
      Bs[kk][i] = ldx(ub, (long)(v0 + i) * d.ncp + c0 + kk);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      A a[4], bb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][tr + 16 * q];
        bb[q] = Bs[kk][tv + 16 * q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], bb[w], acc[q][w]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + tr + 16 * q;
    A s = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s = fma((A)ldx(psi_v_rv, (long)r * d.nvp + v0 + tv + 16 * w), acc[q][w], s);
    red[tv][tr + 16 * q] = s;
  }
  __syncthreads();
  if (tid < TM) {
    A s = 0;
    for (int j = 0; j < 16; ++j) s += red[j][tid];
    rho_part[((long)blockIdx.y * nb + b) * d.nrp + r0 + tid] = s;
  }
}

template <typename A, typename TO, typename TV>
__global__ void __launch_bounds__(256)
gemm2_simple_kernel(GemmDims d, const TO* __restrict__ psi_v_t,
                 const TO* __restrict__ psi_c_t, const TV* __restrict__ vpot,
                 A* __restrict__ ypart, int nb, int splitk, int kchunk, int round16, long ph) {
  // orbital (row, r): K panels of 32 points when ph > 0, else rows of N_rp
  auto at = [&](int row, int r) {
    return ph ? (long)(r >> 5) * ph + (long)row * 32 + (r & 31) : (long)row * d.nrp + r;
  };
  __shared__ A As[TK][LDT];
  __shared__ A Bs[TK][LDT];
  const int tid = threadIdx.x;
  const int ti = tid & 15, tj = tid >> 4;
  const int c0 = blockIdx.x * TN, v0 = blockIdx.y * TM;
  const int b = blockIdx.z / splitk, s = blockIdx.z - b * splitk;
  const int rbeg = s * kchunk;
  const int rend = min(d.nrp, rbeg + kchunk);
  const TV* vb = vpot + (long)b * d.nrp;
  A acc[4][4] = {};
  for (int r = rbeg; r < rend; r += TK) {
    for (int e = tid; e < TK * TM; e += 256) {
      const int kk = e & (TK - 1), i = e >> 4;
      A av = (A)ldx(psi_v_t, at(v0 + i, r + kk)) * (A)ldx(vb, r + kk);
      // mixed path: the operand phi_v V_b is rounded to FP16 as in the MFMA kernel
      if (round16) av = (A)(float)(_Float16)(float)av;
      As[kk][i] = av;
      Bs[kk][i] = ldx(psi_c_t, at(c0 + i, r + kk));
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      A a[4], bb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ti + 16 * q];
        bb[q] = Bs[kk][tj + 16 * q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], bb[w], acc[q][w]);
    }
    __syncthreads();
  }
  A* out = ypart + ((long)s * nb + b) * d.nvp * d.ncp;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w)
      out[(long)(v0 + ti + 16 * q) * d.ncp + c0 + tj + 16 * w] = acc[q][w];
}

}  // namespace

int gemm1_f64_vtiles(const GemmDims& d) { return d.nvp / TN; }

void gemm1_f64(const GemmDims& d, int nb, const double* psi_c_rc, const double* psi_v_rv,
               const double* u, double* rho_part, hipStream_t st) {
  if (nb <= 0) return;
  dim3 grid(d.nrp / TM, d.nvp / TN, nb);
  gemm1_simple_kernel<double, double, double><<<grid, 256, 0, st>>>(d, psi_c_rc, psi_v_rv, u,
                                                                    rho_part, nb);
  GWL_HIP(hipGetLastError());
}

int gemm1_f16s_vtiles(const GemmDims& d) { return d.nvp / TN; }

void gemm1_f16s(const GemmDims& d, int nb, const f16_t* psi_c_rc, const float* psi_v_rv,
                const f16_t* u, float* rho_part, hipStream_t st) {
  if (nb <= 0) return;
  dim3 grid(d.nrp / TM, d.nvp / TN, nb);
  gemm1_simple_kernel<float, f16_t, float><<<grid, 256, 0, st>>>(d, psi_c_rc, psi_v_rv, u,
                                                                  rho_part, nb);
  GWL_HIP(hipGetLastError());
}

void gemm2_f16s(const GemmDims& d, int nb, int splitk, const f16_t* psi_v_t,
                const f16_t* psi_c_t, const f16_t* vpot, float* ypart, hipStream_t st) {
  if (nb <= 0) return;
  const int kchunk = (int)round_up(ceil_div(d.nrp, splitk), TK);
  dim3 grid(d.ncp / TN, d.nvp / TM, nb * splitk);
  gemm2_simple_kernel<float, f16_t, f16_t><<<grid, 256, 0, st>>>(d, psi_v_t, psi_c_t, vpot, ypart,
                                                          nb, splitk, kchunk, 1, orb16_panel_halves(d));
  GWL_HIP(hipGetLastError());
}

void gemm2_f64(const GemmDims& d, int nb, int splitk, const double* psi_v_t,
               const double* psi_c_t, const double* vpot, double* ypart, hipStream_t st) {
  if (nb <= 0) return;
  const int kchunk = (int)round_up(ceil_div(d.nrp, splitk), TK);
  dim3 grid(d.ncp / TN, d.nvp / TM, nb * splitk);
  gemm2_simple_kernel<double, double, double><<<grid, 256, 0, st>>>(d, psi_v_t, psi_c_t, vpot, ypart,
                                                             nb, splitk, kchunk, 0, 0);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
