// Internal launch interfaces of the gfx950 kernels.  Not part of the C ABI.
#pragma once

#include "common.h"

namespace gwl {

// ---------------------------------------------------------------- FFT Poisson
struct FftPlan {
  int nstages;
  int radix[8];
  int ok;
};
FftPlan make_plan(int n);
// Once per device at setup: lets the yz-plane and x-slab passes use up to 80 KB of LDS.
void poisson_prepare_device();

template <typename T>
struct PoissonGeom {
  int nx, ny, nz;
  FftPlan px, py, pz;
  const cplx<T>* twx;  // exp(-2 pi i k / n), k < n, per axis
  const cplx<T>* twy;
  const cplx<T>* twz;
  const T* g2x;        // |G_x|^2 per index, fftfreq convention
  const T* g2y;
  const T* g2z;
  T vscale;            // kernel_scale * 4 pi / N_r
};

// rin: [nparts][nf][ld_in] partial densities (summed); rout: [nf][ld_out].
// scratch: [(nf+1)/2][N_r] complex.  With vexp (the mixed product), every
// output field f is multiplied by 2^vexp[f], the power of two that keeps
// |phi| |V_f| 2^vexp[f] below 2^14 for orbital values up to 2^pexp (from a
// bound of |V_f| the solve records in xmax, [(nf+1)/2] scratch), and written
// rounded to FP16 into rout16 (same layout as rout) instead of rout.
template <typename T>
void poisson_launch(const PoissonGeom<T>& g, const T* rin, long ld_in, long part_stride,
                    int nparts, T* rout, long ld_out, int nf, cplx<T>* scratch,
                    hipStream_t st, unsigned* xmax = nullptr, int* vexp = nullptr,
                    int pexp = 0, f16_t* rout16 = nullptr);

// ---------------------------------------------------------------- GEMMs
// Padded operand layouts (NRp, NVp, NCp multiples of the tile sizes):
//   psi_c_rc [NRp][NCp]  (GEMM1 B operand, c contiguous)
//   psi_v_rv [NRp][NVp]  (GEMM1 epilogue weights)
//   psi_v_t  [NVp][NRp], psi_c_t [NCp][NRp]  (GEMM2 operands, r contiguous)
//   u        [B][NVp][NCp]  (Delta^1/2 x in operand precision)
//   rho      [nvt][B][NRp]  partial densities, one per v tile (summed by the FFT)
//   vpot     [B][NRp]
//   ypart    [S][B][NVp][NCp] split-K partial sums of the second GEMM
struct GemmDims {
  int nr, nrp, nv, nvp, nc, ncp;
};

// Padding: N_r to 256; N_c to 64; N_v to 64, 128 or a multiple of 256 (the
// BF16 tile of 256 rows must hold whole pair vectors or lie inside one).
constexpr int kPadR = 256;
constexpr int kPadC = 64;
inline int pad_nv(int nv) { return nv <= 64 ? 64 : (nv <= 128 ? 128 : (int)round_up(nv, 256)); }
// The BF16 tiles read whole 256-row A tiles and 128-row B tiles without
// bounds checks: pair-vector operand rows are allocated to a multiple of 256,
// potentials to the pair vectors those rows touch, orbital rows of the
// second GEMM's B operand to a multiple of 256.
inline long alloc_rows_u(long nb, int nvp) { return round_up(nb * nvp, 256); }
inline long alloc_rows_v(long nb, int nvp) { return alloc_rows_u(nb, nvp) / nvp + 1; }
inline long alloc_rows_c(int ncp) { return round_up(ncp, 256); }
// FP16 orbitals of the mixed second GEMM: rows of N_rp values (N_vp occupied
// rows, then the conduction rows), or, once rows are 2 MB or more apart
// (N_rp >= 2^20), K panels: the grid axis is cut into panels of 32 points,
// and a panel holds 32 consecutive values of every orbital row, so value
// (row, r) sits at (r / 32) * panel_halves + row * 32 + r % 32.  One K step
// of a tile is then one contiguous run per 16 rows, where long rows would put
// every row on its own memory page (at 128^3, 4 MB apart: the address
// translations, not the bytes, limited that layout: 488 against 280 ms per
// launch).  At 64^3 the rows are faster (3.69 against 4.05 ms).
__host__ __device__ inline long panel_rows(const GemmDims& d) {
  return d.nvp + ((long)d.ncp + 255) / 256 * 256;  // N_vp + alloc_rows_c(N_cp)
}
__host__ __device__ inline long panel_halves(const GemmDims& d) { return panel_rows(d) * 32; }
// halves per K panel of the FP16 orbitals, 0 when they are stored in rows
__host__ __device__ inline long orb16_panel_halves(const GemmDims& d) {
  return d.nrp >= (1 << 20) ? panel_halves(d) : 0;
}
// index of orbital value (row, r) in the FP16 copy
__host__ __device__ inline long orb16_index(const GemmDims& d, long row, long r) {
  const long ph = orb16_panel_halves(d);
  return ph ? (r >> 5) * ph + row * 32 + (r & 31) : row * d.nrp + r;
}

// FP64 (plain tiled FMA; reference-quality GPU path).
int gemm1_f64_vtiles(const GemmDims& d);
void gemm1_f64(const GemmDims& d, int nb, const double* psi_c_rc, const double* psi_v_rv,
               const double* u, double* rho_part, hipStream_t st);
void gemm2_f64(const GemmDims& d, int nb, int splitk, const double* psi_v_t,
               const double* psi_c_t, const double* vpot, double* ypart, hipStream_t st);

// FP16 operands, FP32 accumulation, plain FMA tiles (checks the MFMA kernels;
// the second GEMM's operand phi_v V_b is rounded to FP16 as there).
int gemm1_f16s_vtiles(const GemmDims& d);
void gemm1_f16s(const GemmDims& d, int nb, const f16_t* psi_c_rc, const float* psi_v_rv,
                const f16_t* u, float* rho_part, hipStream_t st);
// psi_v_t, psi_c_t: the FP16 orbitals (psi_c_t = the first conduction value,
// orb16_index(d, N_vp, 0))
void gemm2_f16s(const GemmDims& d, int nb, int splitk, const f16_t* psi_v_t,
                const f16_t* psi_c_t, const f16_t* vpot, float* ypart, hipStream_t st);

// FP64 on MFMA (v_mfma_f64_16x16x4).
int gemm1_f64m_vtiles(const GemmDims& d);
void gemm1_f64m(const GemmDims& d, int nb, const double* psi_c_rc, const double* psi_v_rv,
                const double* u, double* rho_part, hipStream_t st);
void gemm2_f64m(const GemmDims& d, int nb, int splitk, const double* psi_v_t,
                const double* psi_c_t, const double* vpot, double* ypart, hipStream_t st);

// FP16 operands, FP32 accumulation, on MFMA.
int gemm1_f16_vtiles(const GemmDims& d);
// First GEMM of the mixed path: FP16 operands (u scaled by a power of two),
// FP32 accumulation.  psi_v_rv: FP32 [N_rp][N_vp] epilogue weights;
// psi_v_rv16: the same in FP16 (used when N_vp is 64 or 128)
void gemm1_f16(const GemmDims& d, int nb, const f16_t* psi_c_rc, const float* psi_v_rv,
               const f16_t* psi_v_rv16, const f16_t* u, float* rho_part, hipStream_t st);
// Second GEMM of the mixed path: A = phi_v V_b formed while staging by
// packed FP16 products (psi_v_t, psi_c_t: the FP16 orbitals scaled by the
// orbital scale, psi_c_t = the first conduction value, orb16_index(d, N_vp,
// 0); vpot: the FP16 potentials [b][N_rp] as the Poisson solve scaled them).
// bn = block tile width (128 or 256).
int gemm2_f16_blocks(const GemmDims& d, int nb, int bn);  // blocks per split of the K range
int gemm2_f64m_blocks(const GemmDims& d, int nb);
void gemm2_f16(const GemmDims& d, int nb, int bn, int splitk, const f16_t* psi_v_t,
               const f16_t* psi_c_t, const f16_t* vpot, float* ypart, hipStream_t st);

// ---------------------------------------------------------------- pair-space ops
struct PairGeom {
  int nv, nc, nvp, ncp;
  long nvc;
  const double* delta2;  // Delta^2   [nvc]
  const double* sdelta;  // Delta^1/2 [nvc]
  double dv;
  const double* delta = nullptr;  // Delta [nvc] (Tamm-Dancoff product)
  // FP16 operand scaling: cast_u writes uscale * value; combine multiplies the
  // second GEMM's sum by yscale = 1 / uscale (powers of two, exact)
  double uscale = 1.0, yscale = 1.0;
  // Tamm-Dancoff: the operand is x itself (no Delta^1/2), combine mode 3 gives
  // A x = Delta x + K x, coupling vectors are (nm|vc)
  int tda = 0;
  // cast_u / combine only: GEMM operand row b belongs to pair-vector slot
  // rows[b] (device, nb entries); nullptr = row b is slot b
  const int* rows = nullptr;
  // mixed second GEMM: row b of its sum also carries the potential's scale
  // 2^vexp[b] (set by the Poisson solve), divided out next to yscale
  const int* vexp = nullptr;
};

// Elementwise orbital products rho_i = phi_{n_i} phi_{m_i} (FP64), [cnt][NRp].
void pair_product(const double* psi_t, long ld, int nr, const int* m_idx, const int* n_idx,
                  int cnt, double* rho, hipStream_t st);

// out[i] = dv sum_{r < nr} rho_i(r) V_i(r) for cnt fields (row stride ld).
void pair_energy(const double* rho, const double* vpot, long ld, int nr, double dv, int cnt,
                 double* out, hipStream_t st);

// out[i] = ||x_i||_2 for nrows rows of length n (FP64, fixed reduction order).
void row_norm2(const double* x, long n, int nrows, double* out, hipStream_t st);

// u[b] = cast(Delta^1/2 * x[slot(b)]) into the padded operand layout.
template <typename U>
void cast_u(const PairGeom& g, int nb, const double* x, long ldx, U* u, hipStream_t st);

// Chebyshev/C combine after the second GEMM.  y = sum_s ypart[s];
// cx = Delta^2 x + 2 dV Delta^1/2 y.  mode 0: out = cx.  mode 1 (first
// Chebyshev step): tn = (2 cx - (hi+lo) x)/(hi-lo); acc = c0 x + c1 tn.
// mode 2: tn = 2 (2 cx - (hi+lo) x)/(hi-lo) - tp; acc += cj tn.
// mode 3 (Tamm-Dancoff, g.tda): out = Delta x + dV y.
// Row b of ypart / u pairs with slot g.rows[b] of x, tp, out, acc, kx_out.
// If u != null also writes u = cast(Delta^1/2 tn) (mode 1, 2) for the next product;
// if kx_out != null also writes the coupling part K Delta^1/2 x = dV y.
template <typename Y, typename U>
void combine(const PairGeom& g, int nb, int splitk, const Y* ypart, const double* x,
             const double* tp, double* out_tn, double* acc, int mode, double lo, double hi,
             double c0, double cj, U* u, hipStream_t st, double* kx_out = nullptr);

// Coupling finish: P_i = dV Delta^1/2 sum_s ypart[s][i]; writes P (compact)
// to p_out[i] (ld ldp).
template <typename Y>
void coupling_finish(const PairGeom& g, int cnt, int splitk, const Y* ypart, double* p_out,
                     long ldp, hipStream_t st);

// ---------------------------------------------------------------- Lanczos
struct SlotState {
  int* pair;       // [B] pair id, -1 = empty slot
  int* k;          // [B] current step index
  int* len;        // [B] steps to run
  int* dead;       // [B] breakdown flag
  double* amax;    // [B] max |a_j| so far
  double* bprev;   // [B] b_k of the three-term update
  double* coef_a;  // [n_pairs][ld]
  double* coef_b;  // [n_pairs][ld]
  int* out_len;    // [n_pairs]
  double* norm2;   // [n_pairs]
  int ld;
};

// Start: from P in q (slot rows listed in slots), compute ||P||^2, q = P/||P||,
// store basis row 0, reset slot state.
void lz_start(const SlotState& s, int nb_slots, const int* slot_list, int cnt, double* q,
              double* qprev, double* basis, long basis_slot_stride, long nvc, hipStream_t st);
// a_k = q.w; w -= a_k q + b_k q_prev.
void lz_alpha(const SlotState& s, int nb, const double* q, const double* qprev, double* w,
              long nvc, hipStream_t st);
// Scratch of the full reorthogonalisation: wn0 [nb], part [nb][reorth_part_len],
// skip [nb].
struct ReorthScratch {
  double* wn0;
  double* part;
  int* skip;
};
long reorth_part_len(long nvc);
// full (classical Gram-Schmidt against basis rows 0..k, a second pass where
// the first removed more than half of ||w||^2) or local (two passes against
// q_k, q_{k-1}) reorthogonalisation.
void lz_reorth(const SlotState& s, int nb, int kmax, int mode, const double* basis,
               long basis_slot_stride, const double* q, const double* qprev, double* w,
               double* hbuf, const ReorthScratch& rs, long nvc, hipStream_t st);
// b_{k+1} = ||w||; breakdown test; q_prev = q; q = w / b; basis row k+1 = q; k += 1.
void lz_beta(const SlotState& s, int nb, double* q, double* qprev, double* w, double* basis,
             long basis_slot_stride, int store_basis, long nvc, hipStream_t st);

// Sturm counts of each run's tridiagonal T (a_0..a_{L-1}, b_1..b_{L-1} in
// [npairs][ld], L = lens[p]): bad[p] = 1 when T has an eigenvalue below t_lo
// or above t_hi, else 0.  One thread per run.
void lz_interval_check(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                       int ld, double t_lo, double t_hi, int* bad, hipStream_t st);

// ---------------------------------------------------------------- continued fraction
// sig[p][w] (complex, eV) for pairs p, Eq. 12 with Eq. 14.
void cfrac_sigma(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                 const double* norm2, int ld, const double* e_n, const double* eta_n,
                 const double* omega_ha, int nomega, double delta_ha, int tda, double* sig,
                 hipStream_t st);
// Lanczos-on-C Gauss quadrature: per pair, eigenvalues and first components
// of T by implicit QL (qd, qe, qz, status: device scratch [npairs][ld] and
// [npairs]), then Sigma(w, n) = sum_k w_k [theta_k^-1/2 - (theta_k^1/2 +
// eta z)^-1] / z into sig [npairs][nomega][2] (eV).
void quad_sigma(int npairs, const double* coef_a, const double* coef_b, const int* lens,
                const double* norm2, int ld, const double* e_n, const double* eta_n,
                const double* omega_ha, int nomega, double delta_ha, double* qd, double* qe,
                double* qz, int* status, double* sig, hipStream_t st);
// out[q][w] = sum_{p in [q*per, (q+1)*per)} sig[p][w], fixed order.
// dst rows 2i, 2i + 1 = a_i + b_i, a_i - b_i (cnt rows of length n each)
void polar_rows(const double* a, const double* b, long n, int cnt, double* dst, hipStream_t st);
// out [nomega][2] = (sum_n sig[2n] - sig[2n+1]) / 4 over nn pairs of rows
void sum_polar(const double* sig, int nn, int nomega, double* out, hipStream_t st);
void sum_groups(const double* sig, int ngroups, int per, int nomega, double* out,
                hipStream_t st);

// ---------------------------------------------------------------- adjoint
void adj_cfrac(int npairs, const double* ca, const double* cb, const int* lens,
               const double* norm2, int ld, const double* e_n, const double* eta_n,
               const int* qidx, const double* omega_ha, int nomega, double delta_ha,
               const double* G, void* tscr, double* abar, double* bbar, double* nbar,
               double* ebar, double* sig, hipStream_t st);
void adj_lanczos_step(int k, int nb, const int* pair_of_slot, const int* lens, int ld,
                      const double* ca, const double* cb, const double* abar, const double* bbar,
                      const double* q_next, const double* q_cur, const double* q_prev,
                      const double* w_cur, const double* qb_next, double* qb_cur, double* qb_prev,
                      double* wbar, double* pend, long nvc, hipStream_t st);
void adj_start(int nb, const int* pair_of_slot, const double* norm2, const double* nbar,
               const double* P, const double* qb0, const double* sdelta, double* dbar,
               double* kbar, long nvc, hipStream_t st);
void adj_combine(const PairGeom& g, int nb, int splitk, const double* ypart, const double* sj,
                 const double* sj1, const double* seed, double cprev, double sigma, double lo,
                 double hi, double* out, double* ks, double* u, hipStream_t st);
void adj_scale_copy(double* dst, const double* src, double c, long n, hipStream_t st);
void adj_axpy(double* dst, const double* src, double a, long n, hipStream_t st);
void adj_sum_rows(double* dst, const double* src, int nrows, long n, hipStream_t st);
void adj_orb_grad_nm(const double* psi_t, const double* Vk, long ld, int nr, const int* mrow,
                     const int* nrow, int npairs, double dv, double* grad, hipStream_t st);
// user layout [n_orb][nr] (FP32 if f32, else FP64) from the padded [nvp + ncp][ld]
void adj_gather_orbitals(const double* src, long ld, int nr, int nv, int nvp, int norb,
                         void* dst, bool f32, hipStream_t st);

// Factored orbital gradient of pair-vector outer products (adj_zgemm.hip).
// A segment pairs k potentials vf [k][N_rp] with k padded pair vectors
// u [k][N_vp][N_cp]; with Z(r, v, c) = sum over both segments of vf(r) u(v, c):
//   grad_c[c][r] += dv sum_v phi_v(r) Z(r, v, c)          (rows [N_cp][N_rp])
//   gvpart[ct][v][r] += dv sum_{c in tile ct} phi_c(r) Z   (ct = c / 64)
struct ZSeg {
  const double* vf;
  const double* u;
  int k;
};
void adj_zgemm(const GemmDims& d, int nv, const ZSeg& s0, const ZSeg& s1, const double* psi_c_rc,
               const double* psi_v_rv, double dv, double* grad_c, double* gvpart,
               hipStream_t st);
// grad_v[v][r] += sum over the nct c tiles, in order, of gvpart[ct][v][r]
void adj_gv_reduce(const double* gvpart, int nct, int nv, long nrp, double* grad_v,
                   hipStream_t st);
// Per Chebyshev term: Delta_bar += alpha [2 Delta s t + (s K~t + t K~s)/Delta^1/2]
// and the padded operands us = kappa Delta^1/2 s, ut = kappa Delta^1/2 t.
void adj_dbar_zops(const PairGeom& g, int nb, const double* s, const double* ks, const double* t,
                   const double* kt, double alpha, double kappa, double* dbar, double* us,
                   double* ut, hipStream_t st);

// ---------------------------------------------------------------- allocation-free entry
// Takes the device address of the static scratch array of the allocation-free
// entry point for the current device (once per device).
// Setup: the caller's orbitals (device, FP64 or FP32 rows of nr values) into
// psi_t and its FP64 transposes; *bad set if a value is not finite, and
// *omax_bits raised to the bits of max |phi| (both cleared by the caller).
void pack_orbitals64(const GemmDims& d, const void* src, int orb_dtype, int n_orb, long nr,
                     double* psi_t, double* psi_c_rc64, double* psi_v_rv64, int* bad,
                     unsigned long long* omax_bits, hipStream_t st);
// The scaled 16- and 32-bit copies (scale os); *pvmax_bits raised to the bits
// (as float) of the largest |FP16 value| of the occupied rows.
void pack_orbitals16(const GemmDims& d, const double* psi_t, const double* psi_c_rc64,
                     const double* psi_v_rv64, double os, f16_t* psi_t16, f16_t* psi_c_rc16,
                     float* psi_v_rv32, f16_t* psi_v_rv16, unsigned long long* pvmax_bits,
                     hipStream_t st);
void noalloc_bind_current_device();

}  // namespace gwl
