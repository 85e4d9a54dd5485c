// Orbital packing of the setup on the GPU: the caller's orbitals (FP64 or
// FP32 rows of N_r grid values, in HBM) become the layouts the kernels read,
// with no host staging (at 128^3 and 1,536 orbitals the host loops took about
// 100 s, the device passes well under a second):
//   psi_t       FP64 rows [N_vp + N_cp][N_rp] (occupied rows, then the
//               conduction rows; pads zero),
//   psi_c_rc64  FP64 [N_rp][N_cp]   psi_v_rv64  FP64 [N_rp][N_vp]  (transposes),
//   psi_t16     FP16 rows or K panels of psi_t (orb16_index), scaled by os,
//   psi_c_rc16  FP16 [N_rp][N_cp], psi_v_rv32 FP32 and psi_v_rv16 FP16
//               [N_rp][N_vp], all scaled by os,
// where os is the power of two that the host picks from max |phi| (read back
// between the two halves).  Every value is converted exactly as the
// corresponding host expression would (FP64 products, then the
// round-to-nearest conversions), so the layouts do not depend on where they
// were built.  The maxima are order-independent (bit patterns of
// non-negative numbers compare like unsigned integers), so runs are
// reproducible.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

constexpr int PT = 256;

// psi_t row orb_row(n) <- orbital n (pads zero); flags a non-finite value
template <typename T>
__global__ void __launch_bounds__(PT)
pack_rows_kernel(const T* __restrict__ src, int nv, int nvp, long nr, long nrp,
                 double* __restrict__ psi_t, int* __restrict__ bad) {
  const int n = blockIdx.y;
  const int row = n < nv ? n : nvp + (n - nv);
  const T* s = src + (long)n * nr;
  double* d = psi_t + (long)row * nrp;
  int nonfinite = 0;
  for (long r = blockIdx.x * (long)PT + threadIdx.x; r < nrp; r += (long)gridDim.x * PT) {
    const double v = r < nr ? (double)s[r] : 0.0;
    nonfinite |= !isfinite(v);
    d[r] = v;
  }
  if (nonfinite) *bad = 1;
}

__device__ inline void block_max_bits(unsigned long long v, unsigned long long* out) {
  __shared__ unsigned long long sh[PT / 64];
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < PT / 64; ++i) v = sh[i] > v ? sh[i] : v;
    atomicMax(out, v);
  }
}

// out <- max(out, bits of max |a_i|)
__global__ void __launch_bounds__(PT)
absmax_kernel(const double* __restrict__ a, long n, unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (long i = blockIdx.x * (long)PT + threadIdx.x; i < n; i += (long)gridDim.x * PT)
    m = fmax(m, fabs(a[i]));
  block_max_bits((unsigned long long)__double_as_longlong(m), out);
}

// dst[r][i] = src[i][r] for i < rows, r < nrp (src rows nrp apart), through a
// 32 x 32 tile in LDS
__global__ void __launch_bounds__(PT)
transpose_kernel(const double* __restrict__ src, int rows, long nrp, double* __restrict__ dst) {
  __shared__ double tile[32][33];
  const long r0 = (long)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = i0 + k;
    const long r = r0 + tx;
    tile[k][tx] = (i < rows && r < nrp) ? src[(long)i * nrp + r] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const long r = r0 + k;
    const int i = i0 + tx;
    if (i < rows && r < nrp) dst[r * rows + i] = tile[tx][k];
  }
}

// psi_t16 <- f16(os psi_t) in rows or K panels; pv_bits <- max |f16 value|
// over the occupied rows
__global__ void __launch_bounds__(PT)
orb16_kernel(GemmDims d, const double* __restrict__ psi_t, double os, f16_t* __restrict__ t16,
             unsigned long long* __restrict__ pv_bits) {
  const int row = blockIdx.y;
  const long nrp = d.nrp;
  float m = 0.0f;
  for (long r = blockIdx.x * (long)PT + threadIdx.x; r < nrp; r += (long)gridDim.x * PT) {
    const f16_t h = f32_to_f16((float)(os * psi_t[(long)row * nrp + r]));
    t16[orb16_index(d, row, r)] = h;
    m = fmaxf(m, fabsf(f16_to_f32(h)));
  }
  if (row < d.nvp) block_max_bits((unsigned long long)__float_as_uint(m), pv_bits);
}

// scaled FP16 / FP32 copies of the transposed FP64 layouts
__global__ void __launch_bounds__(PT)
scaled_copies_kernel(const double* __restrict__ crc, long ncrc, const double* __restrict__ vrv,
                     long nvrv, double os, f16_t* __restrict__ c16, float* __restrict__ v32,
                     f16_t* __restrict__ v16) {
  for (long i = blockIdx.x * (long)PT + threadIdx.x; i < ncrc; i += (long)gridDim.x * PT)
    c16[i] = f32_to_f16((float)(os * crc[i]));
  for (long i = blockIdx.x * (long)PT + threadIdx.x; i < nvrv; i += (long)gridDim.x * PT) {
    const float f = (float)(os * vrv[i]);
    v32[i] = f;
    v16[i] = f32_to_f16(f);
  }
}

inline unsigned grid_1d(long n) {
  const long g = (n + PT - 1) / PT;
  return (unsigned)std::max(1L, std::min(g, 4096L));
}

}  // namespace

void pack_orbitals64(const GemmDims& d, const void* src, int orb_dtype, int n_orb, long nr,
                     double* psi_t, double* psi_c_rc64, double* psi_v_rv64, int* bad,
                     unsigned long long* omax_bits, hipStream_t st) {
  const long nrp = d.nrp;
  const dim3 gr((unsigned)std::min<long>((nrp + PT - 1) / PT, 1024), (unsigned)n_orb);
  if (orb_dtype == 8)
    pack_rows_kernel<double><<<gr, PT, 0, st>>>(static_cast<const double*>(src), d.nv, d.nvp,
                                                nr, nrp, psi_t, bad);
  else
    pack_rows_kernel<float><<<gr, PT, 0, st>>>(static_cast<const float*>(src), d.nv, d.nvp, nr,
                                               nrp, psi_t, bad);
  const long rows = (long)d.nvp + d.ncp;
  absmax_kernel<<<grid_1d(rows * nrp), PT, 0, st>>>(psi_t, rows * nrp, omax_bits);
  const unsigned rt = (unsigned)((nrp + 31) / 32);
  transpose_kernel<<<dim3(rt, (unsigned)((d.ncp + 31) / 32)), PT, 0, st>>>(
      psi_t + (long)d.nvp * nrp, d.ncp, nrp, psi_c_rc64);
  transpose_kernel<<<dim3(rt, (unsigned)((d.nvp + 31) / 32)), PT, 0, st>>>(psi_t, d.nvp, nrp,
                                                                          psi_v_rv64);
  GWL_HIP(hipGetLastError());
}

void pack_orbitals16(const GemmDims& d, const double* psi_t, const double* psi_c_rc64,
                     const double* psi_v_rv64, double os, f16_t* psi_t16, f16_t* psi_c_rc16,
                     float* psi_v_rv32, f16_t* psi_v_rv16, unsigned long long* pvmax_bits,
                     hipStream_t st) {
  const long nrp = d.nrp;
  const dim3 gr((unsigned)std::min<long>((nrp + PT - 1) / PT, 1024), (unsigned)(d.nvp + d.ncp));
  orb16_kernel<<<gr, PT, 0, st>>>(d, psi_t, os, psi_t16, pvmax_bits);
  const long ncrc = nrp * d.ncp, nvrv = nrp * d.nvp;
  scaled_copies_kernel<<<grid_1d(std::max(ncrc, nvrv)), PT, 0, st>>>(
      psi_c_rc64, ncrc, psi_v_rv64, nvrv, os, psi_c_rc16, psi_v_rv32, psi_v_rv16);
  GWL_HIP(hipGetLastError());
}

}  // namespace gwl
