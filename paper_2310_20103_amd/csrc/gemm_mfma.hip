// Factored pair-space product on the CDNA4 matrix cores.
//
// Both GEMMs are "NT" products over stacked batches, M = B * N_v rows (pair
// vector b, occupied orbital v), with both operands contiguous along K:
//
//   first GEMM   C1[(b,v), r] = sum_c u_b[v, c] phi_c(r)          K = N_c
//                rho_b(r)     = sum_v phi_v(r) C1[(b,v), r]         (epilogue)
//   second GEMM  y_b[v, c]    = sum_r (phi_v(r) V_b(r)) phi_c(r)   K = N_r, split
//
// (the two halves of K x, Eqs. 2-4).  The density of the first GEMM is
// reduced over v inside the tile, so the N_r x N_v intermediate never reaches
// memory; the second GEMM forms its A operand phi_v(r) V_b(r) while staging it
// into LDS, so the per-vector operand never exists in HBM either.
//
// FP64: v_mfma_f64_16x16x4f64, block tile 128 x 128 x 16, 4 waves of 64 x 64.
// Mixed path: both GEMMs on FP16 operands (v_mfma_f32_32x32x16_f16) with FP32
// accumulation; every operand carries a power-of-two scale that puts it
// inside FP16's range (the pair vector per batch, the orbitals once, and
// phi_v V_b per pair vector from the maximum of its potential), undone
// exactly in FP64 by the combine; block tiles 256 x 128 x 32 (4 waves of
// 128 x 64) and, for the second GEMM, 256 x 256 x 32.
// Tiles are staged through LDS with the K steps prefetched into registers
// (two XOR-swizzled LDS stages, one barrier per K step, two register stages:
// the loads of the step after next in flight during the current step's MFMAs).
// Block ids are remapped so that blocks sharing the large operand tile run on
// the same XCD (one L2 per XCD).
#include "common.h"
#include "kernels.h"

namespace gwl {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Consecutive logical ids land on one XCD: hardware dispatches block i to
// XCD i % 8.
__device__ inline int xcd_remap(int bid, int total) {
  if (total % 8 != 0) return bid;
  return (bid & 7) * (total >> 3) + (bid >> 3);
}

// Tile map of the first GEMM (mt x nt tiles, A = pair vectors is the small
// operand, B = orbitals the large one).  With mt >= 8 each XCD owns a fixed
// eighth of the M tiles and walks them in chunks of ch tiles, all N tiles per
// chunk, so the chunk's slice of A (ch tiles of tile_bytes, sized to 2 MB)
// stays in that XCD's 4 MB L2 while the orbital tiles stream past once per
// chunk; with mt < 8 each XCD owns an eighth of the N tiles instead.  Returns
// false for the padding blocks of the grid.
__host__ __device__ inline int gemm1_grid(int mt, int nt) {
  return mt >= 8 ? 8 * ((mt + 7) / 8) * nt : 8 * ((nt + 7) / 8) * mt;
}
__device__ inline bool gemm1_tile(int bid, int mt, int nt, long tile_bytes, int& mi, int& ni) {
  const int x = bid & 7, loc = bid >> 3;
  if (mt >= 8) {
    const int mpx = (mt + 7) / 8;
    long c2 = (2l << 20) / tile_bytes;
    const int ch = (int)(c2 < 1 ? 1 : (c2 > mpx ? mpx : c2));
    const int c = loc / (ch * nt);           // chunk (every full chunk holds ch * nt blocks)
    const int within = loc - c * ch * nt;
    const int sz = min(ch, mpx - c * ch);    // tiles of this chunk
    mi = x * mpx + c * ch + within % sz;
    ni = within / sz;
  } else {
    const int npx = (nt + 7) / 8;
    mi = loc % mt;
    ni = x * npx + loc / mt;
  }
  return mi < mt && ni < nt;
}

// ---------------------------------------------------------------- FP64
constexpr int DM = 128, DN = 128, DK = 16, DLD = DK + 1;

// A operand loader variants for the FP64 kernels.
struct LoadU64 {  // plain [M][K] rows
  const double* a;
  long lda;
  __device__ void load(int m, int k0, int kq, double* v) const {
    const double* p = a + (long)m * lda + k0 + kq;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[i];
  }
};
struct LoadPsiV64 {  // A[(b,v)][r] = phi_v(r) V_b(r)
  const double* psi_v_t;
  const double* vpot;
  long nrp;
  int nvp;
  __device__ void load(int m, int k0, int kq, double* v) const {
    const int b = m / nvp, vv = m - b * nvp;
    const double* p = psi_v_t + (long)vv * nrp + k0 + kq;
    const double* q = vpot + (long)b * nrp + k0 + kq;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[i] * q[i];
  }
};

// Main loop of the FP64 kernels: acc += A[m0.., k] B[n0.., k] for k in [kb, ke).
template <typename LA>
__device__ inline void f64_mainloop(const LA& la, int M, const double* __restrict__ bop, long ldb,
                                    int nvalid, int m0, int n0, int kb, int ke, double (*As)[DLD],
                                    double (*Bs)[DLD], d4 (&acc)[4][4]) {
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int lrow = t >> 1, lkq = (t & 1) * 8;
  double ra[8], rb[8];
  const bool arow_ok = (m0 + lrow) < M;
  auto gload = [&](int k0) {
    if (arow_ok) {
      la.load(m0 + lrow, k0, lkq, ra);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) ra[i] = 0.0;
    }
    if (n0 + lrow < nvalid) {
      const double* p = bop + (long)(n0 + lrow) * ldb + k0 + lkq;
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
      As[lrow][lkq + i] = ra[i];
      Bs[lrow][lkq + i] = rb[i];
    }
  };
  if (kb < ke) {
    gload(kb);
    lstore();
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += DK) {
    const bool more = k0 + DK < ke;
    if (more) gload(k0 + DK);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a[4], b[4];
      const int kk = 4 * ks + (l >> 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[wm * 64 + 16 * i + (l & 15)][kk];
        b[i] = Bs[wn * 64 + 16 * i + (l & 15)][kk];
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
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm1_f64m_kernel(GemmDims d, int M, int nb, const double* __restrict__ psi_c_rc,
                  const double* __restrict__ psi_v_rv, const double* __restrict__ u,
                  double* __restrict__ rho_part) {
  __shared__ double As[DM][DLD];
  __shared__ double Bs[DN][DLD];
  const int mt = (M + DM - 1) / DM, nt = d.nrp / DN;
  int mi, ni;
  if (!gemm1_tile(blockIdx.x, mt, nt, (long)DM * d.ncp * 8, mi, ni)) return;
  const int m0 = mi * DM, n0 = ni * DN;
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0, 0, 0, 0};
  LoadU64 la{u, d.ncp};
  f64_mainloop(la, M, psi_c_rc, d.ncp, d.nrp, m0, n0, 0, d.ncp, As, Bs, acc);
  // epilogue: rho_b(r) = sum over the wave's 64 rows (one b, 64 v) of phi_v(r) C1
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int mw = m0 + wm * 64;
  if (mw >= M) return;
  const int b = mw / d.nvp, vbase = mw - b * d.nvp, vt = vbase / 64;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = n0 + wn * 64 + 16 * j + (l & 15);
    const double* wr = psi_v_rv + (long)r * d.nvp + vbase;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) s += wr[16 * i + (l >> 4) + 4 * q] * acc[i][j][q];
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (l < 16) rho_part[((long)vt * nb + b) * d.nrp + r] = s;
  }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm2_f64m_kernel(GemmDims d, int M, int splitk, int kchunk, const double* __restrict__ psi_v_t,
                  const double* __restrict__ psi_c_t, const double* __restrict__ vpot,
                  double* __restrict__ ypart) {
  __shared__ double As[DM][DLD];
  __shared__ double Bs[DN][DLD];
  const int mt = (M + DM - 1) / DM, nt = (d.ncp + DN - 1) / DN;
  const int lid = xcd_remap(blockIdx.x, mt * nt * splitk);
  const int s = lid / (mt * nt);
  const int rem = lid - s * mt * nt;
  const int m0 = (rem % mt) * DM, n0 = (rem / mt) * DN;
  const int kb = s * kchunk;
  const int ke = min(d.nrp, kb + kchunk);
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0, 0, 0, 0};
  LoadPsiV64 la{psi_v_t, vpot, d.nrp, d.nvp};
  f64_mainloop(la, M, psi_c_t, d.nrp, d.ncp, m0, n0, kb, ke, As, Bs, acc);
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  double* out = ypart + (long)s * M * d.ncp;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = m0 + wm * 64 + 16 * i + (l >> 4) + 4 * q;
      if (m >= M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int n = n0 + wn * 64 + 16 * j + (l & 15);
        if (n < d.ncp) out[(long)m * d.ncp + n] = acc[i][j][q];
      }
    }
}

// ---------------------------------------------------------------- BF16
// Block tile HM x BN (BN = 128 or 256), four waves in a 2 x 2 grid, each
// wave 128 x BN/2 of 32 x 32 MFMA blocks.  BN = 256 gives each wave 256 FP32
// accumulators (held in AGPRs, one wave per SIMD) and halves the LDS and L1
// traffic per flop; BN = 128 runs two waves per SIMD.  The first GEMM uses
// BN = 128 (its per-tile row-dot epilogue needs a second wave per SIMD to
// hide it); the second GEMM takes either, 256 by default.
constexpr int HM = 256, HK = 32, HLD = HK;  // LDS row: 32 bf16 = 64 B, swizzled
// N tiles walked by one first-GEMM block.  One: co-resident blocks then start
// at different times and their row-dot epilogues overlap the other block's
// MFMAs (measured 5 % faster than walks of 2, 4 or 8 tiles).
constexpr int G1_TILES = 1;
template <int BN>
struct BfCfg {
  static constexpr int WN = BN / 64;       // 32-col blocks per wave
  static constexpr int QB = BN * 4 / 256;  // 16-B B chunks per thread and K step
};

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

// 16-bit operand element types of the MFMA kernels: bit patterns in LDS,
// fragments of eight for v_mfma_f32_32x32x16_{bf16,f16}
struct OpBf16 {
  typedef bf8 frag;
  __device__ static f16v mfma(frag a, frag b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
struct OpF16 {
  typedef h8 frag;
  __device__ static f16v mfma(frag a, frag b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <typename OP>
__device__ inline typename OP::frag lds_frag(const bf16_t* p) {
  return __builtin_bit_cast(typename OP::frag, *reinterpret_cast<const u4*>(p));
}
// two floats -> packed bf16 pair, round to nearest even (v_cvt_pk_bf16_f32)
__device__ inline unsigned pack_bf16(float a, float b) {
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
__device__ inline float lo_bf16(unsigned u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_bf16(unsigned u) { return __builtin_bit_cast(float, u & 0xffff0000u); }
__device__ inline float lo_f16(unsigned u) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
}
__device__ inline float hi_f16(unsigned u) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
}

// LDS layout of a 32-wide K slab: rows of 64 bytes (four 16-byte chunks),
// chunk c of row r stored at position c ^ ((r >> 2) & 3).  Both the 16-byte
// staging writes (four threads per row) and the fragment reads (32 rows, one
// chunk) then touch distinct banks.
__device__ inline int swz(int row, int chunk) { return (chunk ^ ((row >> 2) & 3)) * 8; }

// A-tile loaders.  Thread t owns chunks idx = t + 256 q (q < 4) of the
// 256 x 32 tile: row t/4 + 64 q, K offset 8 (t % 4).  load() only issues the
// global loads into registers; finish() turns them into the bf16 chunks
// stored to LDS, after the current step's MFMAs.  Rows up to the 256-row
// tile boundary are always allocated, so no load is guarded.
struct LoadU16 {  // plain [M][K] rows
  const bf16_t* a;
  long lda;
  struct Raw {
    u4 c[4];
  };
  __device__ void load(int m0, int t, int k0, Raw& r) const {
    const bf16_t* p = a + (long)(m0 + (t >> 2)) * lda + k0 + (t & 3) * 8;
#pragma unroll
    for (int q = 0; q < 4; ++q) r.c[q] = *reinterpret_cast<const u4*>(p + (long)64 * q * lda);
  }
  __device__ void prep(Raw&) const {}
  __device__ u4 finish(const Raw& r, int q) const { return r.c[q]; }
};

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
// two floats -> packed FP16 pair, round to nearest even (v_cvt_pk_f16_f32)
__device__ inline unsigned pack_f16(float a, float b) {
  const h2 v = {(_Float16)a, (_Float16)b};
  return __builtin_bit_cast(unsigned, v);
}

// eight packed FP16 products phi_v V (v_pk_mul_f16, round to nearest even:
// the exact product of two FP16 numbers rounded once, as in FP32 and back)
__device__ inline u4 mul8(u4 pv, u4 v) {
  return __builtin_bit_cast(u4, __builtin_bit_cast(h8, pv) * __builtin_bit_cast(h8, v));
}

// A[(b,v)][r] = f16(phi_v(r) V_b(r)), phi_v and V_b in FP16 (both already
// scaled by powers of two into FP16's range).  NVP = padded N_v when it is 64
// or 128 (a thread's four rows then share one or two phi_v rows and use four
// or two potentials), 256 when it is a multiple of 256 (a tile lies inside
// one pair vector: four phi_v rows, one potential), 0 otherwise.
template <int NVP, bool PANEL>
struct LoadPsiV16 {
  const f16_t* psi_v_t;
  const f16_t* vpot;
  long nrp;
  int nvp;
  long ph;  // halves per K panel (PANEL)
  __device__ long at(int row, int k) const {
    if constexpr (PANEL) return (long)(k >> 5) * ph + (long)row * 32 + (k & 31);
    else return (long)row * nrp + k;
  }
  static constexpr int NPV = NVP == 64 ? 1 : (NVP == 128 ? 2 : 4);
  static constexpr int NB = NVP == 128 ? 2 : (NVP == 256 ? 1 : 4);
  static constexpr int kLoads = NPV + NB;  // global loads per thread and K step
  struct Raw {
    u4 pv[NPV];
    u4 v[NB];
  };
  __device__ void load(int m0, int t, int k0, Raw& r) const {
    const int k = k0 + (t & 3) * 8;
    const int r0 = t >> 2;
    if constexpr (NVP == 64) {
      r.pv[0] = *reinterpret_cast<const u4*>(psi_v_t + at(r0, k));
#pragma unroll
      for (int q = 0; q < 4; ++q)
        r.v[q] = *reinterpret_cast<const u4*>(vpot + (long)(m0 / 64 + q) * nrp + k);
    } else if constexpr (NVP == 128) {
      r.pv[0] = *reinterpret_cast<const u4*>(psi_v_t + at(r0, k));
      r.pv[1] = *reinterpret_cast<const u4*>(psi_v_t + at(r0 + 64, k));
#pragma unroll
      for (int h = 0; h < 2; ++h)
        r.v[h] = *reinterpret_cast<const u4*>(vpot + (long)(m0 / 128 + h) * nrp + k);
    } else if constexpr (NVP == 256) {
      const int b = m0 / nvp, v0 = m0 - b * nvp + r0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        r.pv[q] = *reinterpret_cast<const u4*>(psi_v_t + at(v0 + 64 * q, k));
      r.v[0] = *reinterpret_cast<const u4*>(vpot + (long)b * nrp + k);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + r0 + 64 * q;
        const int b = m / nvp, vv = m - b * nvp;
        r.pv[q] = *reinterpret_cast<const u4*>(psi_v_t + at(vv, k));
        r.v[q] = *reinterpret_cast<const u4*>(vpot + (long)b * nrp + k);
      }
    }
  }
  __device__ void prep(Raw&) const {}
  __device__ u4 finish(const Raw& r, int q) const {
    if constexpr (NVP == 64) return mul8(r.pv[0], r.v[q]);
    else if constexpr (NVP == 128) return mul8(r.pv[q & 1], r.v[q >> 1]);
    else if constexpr (NVP == 256) return mul8(r.pv[q], r.v[0]);
    else return mul8(r.pv[q], r.v[q]);
  }
};

template <int BN>
struct BfSmem {
  bf16_t As[2][HM][HLD];
  bf16_t Bs[2][BN][HLD];
};

// One block tile in registers: global loads of one K step of A (raw) and B.
template <typename LA, int BN>
struct BfStage {
  typename LA::Raw a;
  u4 b[BfCfg<BN>::QB];
};

template <typename LA, int BN>
__device__ inline void bf_gload(const LA& la, const bf16_t* __restrict__ bop, long ldb, int m0,
                                int n0, int k0, BfStage<LA, BN>& x) {
  const int t = threadIdx.x;
  la.load(m0, t, k0, x.a);
  const bf16_t* p = bop + (long)(n0 + (t >> 2)) * ldb + k0 + (t & 3) * 8;
#pragma unroll
  for (int q = 0; q < BfCfg<BN>::QB; ++q)
    x.b[q] = *reinterpret_cast<const u4*>(p + (long)64 * q * ldb);
}

// Second GEMM: as bf_gload, with the B operand (conduction orbitals) read
// from K panels when PANEL (bop = the first conduction value, ph = halves per
// panel), else from rows of ldb values.
template <bool PANEL, typename LA, int BN>
__device__ inline void g2_gload(const LA& la, const bf16_t* __restrict__ bop, long ldb, long ph,
                                int m0, int n0, int k0, BfStage<LA, BN>& x) {
  if constexpr (PANEL) {
    const int t = threadIdx.x;
    la.load(m0, t, k0, x.a);
    const bf16_t* p = bop + (long)(k0 >> 5) * ph + (long)(n0 + (t >> 2)) * 32 + (t & 3) * 8;
#pragma unroll
    for (int q = 0; q < BfCfg<BN>::QB; ++q) x.b[q] = *reinterpret_cast<const u4*>(p + 64 * 32 * q);
  } else {
    bf_gload(la, bop, ldb, m0, n0, k0, x);
  }
}

template <typename LA, int BN>
__device__ inline void bf_lstore(const LA& la, BfSmem<BN>& sm, int buf, BfStage<LA, BN>& x) {
  const int t = threadIdx.x;
  la.prep(x.a);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = (t >> 2) + 64 * q;
    *reinterpret_cast<u4*>(&sm.As[buf][row][swz(row, t & 3)]) = la.finish(x.a, q);
  }
#pragma unroll
  for (int q = 0; q < BfCfg<BN>::QB; ++q) {
    const int row = (t >> 2) + 64 * q;
    *reinterpret_cast<u4*>(&sm.Bs[buf][row][swz(row, t & 3)]) = x.b[q];
  }
}

// ZERO: the first 16-wide K slice starts the accumulators from zero (the MFMA
// reads an inline 0 for C) instead of from acc.
template <int BN, typename OP = OpBf16, bool ZERO = false>
__device__ inline void bf_compute(BfSmem<BN>& sm, int buf, f16v (&acc)[4][BfCfg<BN>::WN]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const int ch = 2 * ks + (l >> 5);
    typename OP::frag a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wm * 128 + 32 * i + (l & 31);
      a[i] = lds_frag<OP>(&sm.As[buf][row][swz(row, ch)]);
    }
#pragma unroll
    for (int j = 0; j < BfCfg<BN>::WN; ++j) {
      const int row = wn * (BN / 2) + 32 * j + (l & 31);
      const typename OP::frag b = lds_frag<OP>(&sm.Bs[buf][row][swz(row, ch)]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i][j] = OP::mfma(a[i], b, (ZERO && ks == 0) ? f16v{} : acc[i][j]);
    }
  }
}

// First GEMM.  A block owns one M tile and walks up to G1_TILES consecutive N
// tiles; the first two K steps of the next tile are loaded while the last two
// of the current one compute and its epilogue runs.  SEG = 32-row blocks that
// belong to one pair vector within a wave's 128 rows (4 when N_v padded >=
// 128, 2 when 64).
//
// Epilogue weights phi_v(r): with N_v padded to NVW = 64 or 128 every wave of
// the block uses the same v window, so the tile's BF16 weights [BN][NVW] are
// copied global -> LDS by the direct-to-LDS loads while the K loop runs
// (16-byte chunks XOR-swizzled by row, so the epilogue's 8-byte reads of 32
// rows hit distinct bank groups).  NVW = 0 (larger N_v) reads FP32 weights
// from L2 instead.
template <int BN, int NVW>
struct G1Smem {
  BfSmem<BN> st;
  bf16_t wt[NVW > 0 ? BN : 1][NVW > 0 ? NVW : 1];
};

template <int NVW>
__device__ inline int wswz(int row, int chunk) {
  return (chunk ^ (row & (NVW / 8 - 1))) * 8;
}

// Issue the copies of the weights of rows [n0, n0 + BN), v in [0, NVW): each
// wave moves 1 KB segments, lane l's 16 bytes landing at segment + 16 l.
template <int BN, int NVW>
__device__ inline void g1_weights_dma(G1Smem<BN, NVW>& sm, const f16_t* __restrict__ w16,
                                      int nvp, int n0) {
  constexpr int CPR = NVW / 8;               // 16-byte chunks per row
  constexpr int RPS = 64 / CPR;              // rows per 1 KB segment
  constexpr int SEGS = BN / RPS;             // segments per tile
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  // segment q * 4 + w holds rows (q * 4 + w) * RPS + l / CPR; the swizzled
  // chunk (l % CPR) ^ (row % CPR) does not depend on q
  const int rl0 = w * RPS + l / CPR;
  const int c = (l % CPR) ^ (rl0 & (CPR - 1));
  const f16_t* src = w16 + (long)(n0 + rl0) * nvp + 8 * c;
  bf16_t* dst = &sm.wt[0][0] + w * 512;
  for (int q = 0; q < SEGS / 4; ++q) {
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
    src += (long)4 * RPS * nvp;
    dst += 4 * 512;
  }
}

// Instruction order of one first-GEMM K step (256 x 128 tile, per wave 16
// MFMAs, 12 LDS fragment reads, 6 global loads of the step after next, 6 LDS
// stores of the next step), imposed on the compiler's scheduler: the first
// fragments and all global loads up front, the remaining fragment reads one
// per MFMA, the stores behind the tenth MFMA.  Measured 5 % faster than the
// compiler's own order; loading two steps ahead instead of one gained
// another 3 %.
template <int G>
__device__ inline void g1_sched() {
  if constexpr (G < 16) {
    if constexpr (G == 0) {
      __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);  // LDS reads
      __builtin_amdgcn_sched_group_barrier(0x020, 6, 0);  // global loads
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    if constexpr (G < 6) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    if constexpr (G >= 10) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS writes
    g1_sched<G + 1>();
  }
}

template <int BN, int SEG, int NVW>
__device__ inline void gemm1_f16_body(const GemmDims& d, int M, int nb,
                                      const f16_t* __restrict__ psi_c_rc16,
                                      const float* __restrict__ psi_v_rv,
                                      const f16_t* __restrict__ psi_v_rv16,
                                      const f16_t* __restrict__ u16,
                                      float* __restrict__ rho_part) {
  // FP16 bit patterns travel through the same 16-bit staging as BF16
  const bf16_t* psi_c_rc = reinterpret_cast<const bf16_t*>(psi_c_rc16);
  const bf16_t* u = reinterpret_cast<const bf16_t*>(u16);
  constexpr int WN = BfCfg<BN>::WN;
  __shared__ G1Smem<BN, NVW> sm;
  const int mt = (M + HM - 1) / HM, nt = d.nrp / BN;
  const int ng = (nt + G1_TILES - 1) / G1_TILES;
  int mi, gi;
  if (!gemm1_tile(blockIdx.x, mt, ng, (long)HM * d.ncp * 2, mi, gi)) return;
  const int m0 = mi * HM;
  const int nt0 = gi * G1_TILES, nt1 = min(nt, nt0 + G1_TILES);
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int nsteps = d.ncp / HK;
  LoadU16 la{u, d.ncp};
  // Two register stages: step s of a tile is loaded into x[s & 1] two steps
  // before it computes (N_c is padded to a multiple of 64, so nsteps is even
  // and the next tile's steps 0 and 1 land in x0 and x1 again).
  BfStage<LoadU16, BN> x0, x1;
  bf_gload(la, psi_c_rc, d.ncp, m0, nt0 * BN, 0, x0);
  bf_gload(la, psi_c_rc, d.ncp, m0, nt0 * BN, HK, x1);
  for (int ti = nt0; ti < nt1; ++ti) {
    const int n0 = ti * BN;
    const bool more = ti + 1 < nt1;
    f16v acc[4][WN];
    // The K loop issues at a raised wave priority and the epilogue at the
    // normal one, so that on a SIMD shared by two blocks the one in its K loop
    // keeps the matrix core fed while the other runs its epilogue (1.5 %).
    __builtin_amdgcn_s_setprio(1);
    bf_lstore(la, sm.st, 0, x0);
    __syncthreads();  // also: the previous epilogue has finished reading sm.wt
    if constexpr (NVW > 0) g1_weights_dma<BN, NVW>(sm, psi_v_rv16, d.nvp, n0);
    if (nsteps > 2) {
      bf_gload(la, psi_c_rc, d.ncp, m0, n0, 2 * HK, x0);
      bf_compute<BN, OpF16, true>(sm.st, 0, acc);
      bf_lstore(la, sm.st, 1, x1);
      if constexpr (BN == 128) g1_sched<0>();
      __syncthreads();
      bf_gload(la, psi_c_rc, d.ncp, m0, n0, 3 * HK, x1);
      bf_compute<BN, OpF16>(sm.st, 1, acc);
      bf_lstore(la, sm.st, 0, x0);
      if constexpr (BN == 128) g1_sched<0>();
      __syncthreads();
      for (int i = 2; i + 2 < nsteps; i += 2) {
        bf_gload(la, psi_c_rc, d.ncp, m0, n0, (i + 2) * HK, x0);
        bf_compute<BN, OpF16>(sm.st, 0, acc);
        bf_lstore(la, sm.st, 1, x1);
        if constexpr (BN == 128) g1_sched<0>();
        __syncthreads();
        bf_gload(la, psi_c_rc, d.ncp, m0, n0, (i + 3) * HK, x1);
        bf_compute<BN, OpF16>(sm.st, 1, acc);
        bf_lstore(la, sm.st, 0, x0);
        if constexpr (BN == 128) g1_sched<0>();
        __syncthreads();
      }
      // last two steps: the next tile's first two are loaded
      if (more) bf_gload(la, psi_c_rc, d.ncp, m0, n0 + BN, 0, x0);
      bf_compute<BN, OpF16>(sm.st, 0, acc);
      bf_lstore(la, sm.st, 1, x1);
      __syncthreads();
    } else {
      if (more) bf_gload(la, psi_c_rc, d.ncp, m0, n0 + BN, 0, x0);
      bf_compute<BN, OpF16, true>(sm.st, 0, acc);
      bf_lstore(la, sm.st, 1, x1);
      __syncthreads();
    }
    if (more) bf_gload(la, psi_c_rc, d.ncp, m0, n0 + BN, HK, x1);
    bf_compute<BN, OpF16>(sm.st, 1, acc);
    __syncthreads();
    if constexpr (NVW > 0) {
      // The weight copies were issued before every load still in flight
      // except the next tile's first two K steps (2 (4 + QB) loads); loads
      // complete in issue order, so waiting down to that many leaves the
      // copies done.
      if (more) {
        if constexpr (BN == 128)
          asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
        else
          asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
      } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
      __syncthreads();
    }
    __builtin_amdgcn_s_setprio(0);
    // epilogue: rho_b(r) = sum_v phi_v(r) C1[(b,v), r] over each segment
    const int mw = m0 + wm * 128;
#pragma unroll
    for (int sg = 0; sg < 4; sg += SEG) {
      const int ms = mw + 32 * sg;
      if (ms < M) {
        const int b = ms / d.nvp, vbase = ms - b * d.nvp;
        const int vt = vbase / 128;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int rl = wn * (BN / 2) + 32 * j + (l & 31);
          const int r = n0 + rl;
          float s = 0.f;
          float s4[4] = {0.f, 0.f, 0.f, 0.f};
          if constexpr (NVW > 0) {
#pragma unroll
            for (int i = 0; i < SEG; ++i) {
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                const int ch = (vbase + 32 * i + 8 * g) >> 3;
                const uint2 wv =
                    *reinterpret_cast<const uint2*>(&sm.wt[rl][wswz<NVW>(rl, ch) + 4 * (l >> 5)]);
                s4[0] += lo_f16(wv.x) * acc[sg + i][j][4 * g + 0];
                s4[1] += hi_f16(wv.x) * acc[sg + i][j][4 * g + 1];
                s4[2] += lo_f16(wv.y) * acc[sg + i][j][4 * g + 2];
                s4[3] += hi_f16(wv.y) * acc[sg + i][j][4 * g + 3];
              }
            }
          } else {
            const float* wr = psi_v_rv + (long)r * d.nvp + vbase + 4 * (l >> 5);
#pragma unroll
            for (int i = 0; i < SEG; ++i) {
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                const f4v wv = *reinterpret_cast<const f4v*>(wr + 32 * i + 8 * g);
#pragma unroll
                for (int e = 0; e < 4; ++e) s += wv[e] * acc[sg + i][j][4 * g + e];
              }
            }
          }
          s += (s4[0] + s4[1]) + (s4[2] + s4[3]);  // four shorter FMA chains
          s += __shfl_xor(s, 32, 64);
          if (l < 32) rho_part[((long)vt * nb + b) * d.nrp + r] = s;
        }
      }
    }
  }
}

template <int SEG, int NVW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm1_f16_n128_kernel(GemmDims d, int M, int nb, const f16_t* __restrict__ psi_c_rc,
                      const float* __restrict__ psi_v_rv, const f16_t* __restrict__ psi_v_rv16,
                      const f16_t* __restrict__ u, float* __restrict__ rho_part) {
  gemm1_f16_body<128, SEG, NVW>(d, M, nb, psi_c_rc, psi_v_rv, psi_v_rv16, u, rho_part);
}

// Instruction order of one second-GEMM K step (256 x 256 tile, per wave 32
// MFMAs, 16 LDS fragment reads, NL global loads of the step after next: 8 or
// 9 at N_v = 64, 128, 256, 12 otherwise; 16 packed FP16 products phi_v V and
// 8 LDS stores of the next step), imposed on the compiler's scheduler: four
// fragment reads, then per MFMA one fragment read (first twelve), the
// products two per MFMA over the first eight, the loads one every third MFMA
// (every second for more than ten) and the stores behind MFMAs 14 to 21.
// Spreading the loads is what matters: issuing them all up front made the
// compiler drain the load counter before the stores (4.66 ms per launch at
// the headline shape against 3.69 ms with this order), and so did a load
// left without a slot (514 ms against 314 ms at N_v = 512).
template <int G, int NL>
__device__ inline void g2_sched() {
  constexpr int SP = NL <= 10 ? 3 : 2;
  if constexpr (G < 32) {
    if constexpr (G == 0) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);  // LDS reads
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                       // MFMA
    if constexpr (G < 12) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS reads
    if constexpr (G < 8) __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);   // VALU
    if constexpr (G % SP == 1 && G / SP < NL) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    if constexpr (G >= 14 && G < 22) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS writes
    g2_sched<G + 1, NL>();
  }
}

// Second GEMM over one split of the grid sum: global loads two K steps ahead
// (orbitals from rows or K panels), the A operand of the next step scaled by the
// potential and stored after the current step's MFMAs.
template <int BN, int NVP, bool PANEL>
__device__ inline void gemm2_f16_body(const GemmDims& d, int M, int splitk, int kchunk,
                                      const f16_t* __restrict__ psi_v_t,
                                      const f16_t* __restrict__ psi_c_t16,
                                      const f16_t* __restrict__ vpot,
                                      float* __restrict__ ypart) {
  const bf16_t* psi_c_t = reinterpret_cast<const bf16_t*>(psi_c_t16);  // raw 16-bit rows
  constexpr int WN = BfCfg<BN>::WN;
  __shared__ BfSmem<BN> sm;
  const int mt = (M + HM - 1) / HM, nt = (d.ncp + BN - 1) / BN;
  const int lid = xcd_remap(blockIdx.x, mt * nt * splitk);
  const int s = lid / (mt * nt);
  const int rem = lid - s * mt * nt;
  const int m0 = (rem % mt) * HM, n0 = (rem / mt) * BN;
  const int kb = s * kchunk;
  const int ke = min(d.nrp, kb + kchunk);
  const int nsteps = ke > kb ? (ke - kb) / HK : 0;  // even: kchunk and N_rp are multiples of 2 HK
  f16v acc[4][WN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f16v{};
  const long ph = orb16_panel_halves(d);
  LoadPsiV16<NVP, PANEL> la{psi_v_t, vpot, d.nrp, d.nvp, ph};
  // Two register stages: the loads of step i + 2 are in flight while step i
  // computes and step i + 1 is scaled into the other LDS buffer.  The last
  // steps reload the final slab instead of branching.
  BfStage<LoadPsiV16<NVP, PANEL>, BN> x0, x1;
  if (nsteps > 0) {
    g2_gload<PANEL>(la, psi_c_t, d.nrp, ph, m0, n0, kb, x0);
    g2_gload<PANEL>(la, psi_c_t, d.nrp, ph, m0, n0, kb + HK, x1);
    bf_lstore(la, sm, 0, x0);
  }
  __syncthreads();
  for (int i = 0; i < nsteps; i += 2) {
    g2_gload<PANEL>(la, psi_c_t, d.nrp, ph, m0, n0, kb + min(i + 2, nsteps - 1) * HK, x0);
    bf_compute<BN, OpF16>(sm, 0, acc);
    bf_lstore(la, sm, 1, x1);
    if constexpr (BN == 256) g2_sched<0, LoadPsiV16<NVP, PANEL>::kLoads + BfCfg<BN>::QB>();
    __syncthreads();
    g2_gload<PANEL>(la, psi_c_t, d.nrp, ph, m0, n0, kb + min(i + 3, nsteps - 1) * HK, x1);
    bf_compute<BN, OpF16>(sm, 1, acc);
    bf_lstore(la, sm, 0, x0);
    if constexpr (BN == 256) g2_sched<0, LoadPsiV16<NVP, PANEL>::kLoads + BfCfg<BN>::QB>();
    __syncthreads();
  }
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  float* out = ypart + (long)s * M * d.ncp;
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int n = n0 + wn * (BN / 2) + 32 * j + (l & 31);
    if (n >= d.ncp) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int m = m0 + wm * 128 + 32 * i + 8 * (q >> 2) + 4 * (l >> 5) + (q & 3);
        if (m < M) out[(long)m * d.ncp + n] = acc[i][j][q];
      }
  }
}

template <int NVP, bool PANEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
gemm2_f16_n128_kernel(GemmDims d, int M, int splitk, int kchunk,
                      const f16_t* __restrict__ psi_v_t, const f16_t* __restrict__ psi_c_t,
                      const f16_t* __restrict__ vpot, float* __restrict__ ypart) {
  gemm2_f16_body<128, NVP, PANEL>(d, M, splitk, kchunk, psi_v_t, psi_c_t, vpot, ypart);
}
template <int NVP, bool PANEL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
gemm2_f16_n256_kernel(GemmDims d, int M, int splitk, int kchunk,
                      const f16_t* __restrict__ psi_v_t, const f16_t* __restrict__ psi_c_t,
                      const f16_t* __restrict__ vpot, float* __restrict__ ypart) {
  gemm2_f16_body<256, NVP, PANEL>(d, M, splitk, kchunk, psi_v_t, psi_c_t, vpot, ypart);
}

}  // namespace

int gemm1_f64m_vtiles(const GemmDims& d) { return d.nvp / 64; }

void gemm1_f64m(const GemmDims& d, int nb, const double* psi_c_rc, const double* psi_v_rv,
                const double* u, double* rho_part, hipStream_t st) {
  if (nb <= 0) return;
  const int M = nb * d.nvp;
  const int blocks = gemm1_grid(ceil_div(M, DM), d.nrp / DN);
  gemm1_f64m_kernel<<<blocks, 256, 0, st>>>(d, M, nb, psi_c_rc, psi_v_rv, u, rho_part);
  GWL_HIP(hipGetLastError());
}

void gemm2_f64m(const GemmDims& d, int nb, int splitk, const double* psi_v_t,
                const double* psi_c_t, const double* vpot, double* ypart, hipStream_t st) {
  if (nb <= 0) return;
  const int M = nb * d.nvp;
  const int kchunk = (int)round_up(ceil_div(d.nrp, splitk), DK);
  const int blocks = ceil_div(M, DM) * ceil_div(d.ncp, DN) * splitk;
  gemm2_f64m_kernel<<<blocks, 256, 0, st>>>(d, M, splitk, kchunk, psi_v_t, psi_c_t, vpot, ypart);
  GWL_HIP(hipGetLastError());
}

int gemm1_f16_vtiles(const GemmDims& d) { return d.nvp >= 128 ? d.nvp / 128 : 1; }

void gemm1_f16(const GemmDims& d, int nb, const f16_t* psi_c_rc, const float* psi_v_rv,
               const f16_t* psi_v_rv16, const f16_t* u, float* rho_part, hipStream_t st) {
  if (nb <= 0) return;
  const int M = nb * d.nvp;
  const int blocks = gemm1_grid(ceil_div(M, HM), ceil_div(d.nrp / 128, G1_TILES));
#define GWL_G1(SEGV, NVWV)                                                                   \
  gemm1_f16_n128_kernel<SEGV, NVWV><<<blocks, 256, 0, st>>>(d, M, nb, psi_c_rc, psi_v_rv, \
                                                            psi_v_rv16, u, rho_part)
  if (d.nvp == 64) GWL_G1(2, 64);
  else if (d.nvp == 128) GWL_G1(4, 128);
  else GWL_G1(4, 0);
#undef GWL_G1
  GWL_HIP(hipGetLastError());
}

int gemm2_f16_blocks(const GemmDims& d, int nb, int bn) {
  return ceil_div(nb * d.nvp, HM) * ceil_div(d.ncp, bn);
}

void gemm2_f16(const GemmDims& d, int nb, int bn, int splitk, const f16_t* psi_v_t,
               const f16_t* psi_c_t, const f16_t* vpot, float* ypart, hipStream_t st) {
  if (nb <= 0) return;
  const int M = nb * d.nvp;
  const int kchunk = (int)round_up(ceil_div(d.nrp, splitk), 2 * HK);
  const int blocks = gemm2_f16_blocks(d, nb, bn) * splitk;
  const bool panel = orb16_panel_halves(d) != 0;
#define GWL_G2(BNV, NVPV)                                                                    \
  do {                                                                                       \
    if (panel)                                                                               \
      gemm2_f16_n##BNV##_kernel<NVPV, true><<<blocks, 256, 0, st>>>(d, M, splitk, kchunk,    \
                                                                    psi_v_t, psi_c_t, vpot,  \
                                                                    ypart);                  \
    else                                                                                     \
      gemm2_f16_n##BNV##_kernel<NVPV, false><<<blocks, 256, 0, st>>>(d, M, splitk, kchunk,   \
                                                                     psi_v_t, psi_c_t, vpot, \
                                                                     ypart);                 \
  } while (0)
  if (bn == 256) {
    if (d.nvp == 64) GWL_G2(256, 64);
    else if (d.nvp == 128) GWL_G2(256, 128);
    else if (d.nvp % 256 == 0) GWL_G2(256, 256);
    else GWL_G2(256, 0);
  } else {
    if (d.nvp == 64) GWL_G2(128, 64);
    else if (d.nvp == 128) GWL_G2(128, 128);
    else if (d.nvp % 256 == 0) GWL_G2(128, 256);
    else GWL_G2(128, 0);
  }
#undef GWL_G2
  GWL_HIP(hipGetLastError());
}

int gemm2_f64m_blocks(const GemmDims& d, int nb) {
  return ceil_div(nb * d.nvp, DM) * ceil_div(d.ncp, DN);
}

}  // namespace gwl
