/*
 * gwl.h -- C ABI of the MI355X (gfx950) library for the full-frequency GW
 * correlation self-energy by the Lanczos method of Gao, Tang, Zhao and
 * Chelikowsky, "Efficient Full-frequency GW Calculations using a Lanczos
 * Method".
 *
 * What the library computes (paper notation; QP state m, summed state n):
 *
 *   Sigma_mm(w) = sum_n Sigma_mm(w, n)                                (Eq. 10)
 *   Sigma_mm(w, n) = (1/z_n) <P_nm| D^-1 - (D + eta_n z_n)^-1 |P_nm>   (Eq. 12)
 *   z_n = w - e_n - i eta_n delta,  eta_n = +1 occupied / -1 empty    (Eq. 11)
 *   (P_nm)_vc = (nm|vc) (e_c - e_v)^1/2      (definition before Eq. 9)
 *   D = C^1/2 ~ p_g(C),  C = Delta^2 + 2 Delta^1/2 K Delta^1/2          (Eq. 4 and
 *                                            the paragraph after Eq. 12)
 *   K_{vc,v'c'} = (vc|v'c')                                           (Eqs. 2-3)
 *
 * D is never formed.  Each (m, n) start vector P_nm runs L Lanczos steps on
 * p_g(C) (Eq. 13); the tridiagonal coefficients give Sigma at every
 * frequency through the continued fraction of Eq. 14:
 *   Sigma_mm(w, n) = [R(-eta_n z_n) - R(0)] / z_n,
 *   R(zeta) = ||P||^2 / (zeta - a_0 - b_1^2 / (zeta - a_1 - ...)).
 * The pair-space product C x is applied in factored form on the real-space
 * grid: rho = sum_vc phi_v phi_c (Delta^1/2 x)_vc  (GEMM with a fused
 * row-dot), V = FFT^-1[v(G) FFT[rho]] with v(G) = 4 pi/|G|^2, v(0) = 0,
 * (K u)_vc = dV sum_r phi_v(r) V(r) phi_c(r)  (GEMM).
 *
 * Conventions shared by every entry point
 *   - Indexing is 0-based.  Orbitals [0, n_occ) are occupied, [n_occ, n_orb)
 *     are empty.  Pair index vc = v * N_c + c (v-major), N_c = n_orb - n_occ.
 *   - Units: energies, frequencies, broadening and Sigma in eV; the grid box
 *     in bohr; orbitals grid-normalised (dV * sum_r phi_k phi_l = delta_kl).
 *   - Grid points are stored C-order, r = (ix * ny + iy) * nz + iz.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the context's device.  All pointers are borrowed for
 *     the duration of the call only (except orbitals, see gwl_setup).
 *   - Every call returns a gwl_status; on failure gwl_last_error() gives a
 *     message (thread-local).  No C++ exception crosses the ABI.  Calls on
 *     one context are not thread-safe.  Work is queued on the context stream
 *     and every entry point returns after that stream has finished it.
 *   - The library allocates and owns its working device memory (operand
 *     copies, Lanczos basis, FFT scratch) at setup and on first use of a
 *     larger batch; gwl_destroy frees it.
 */
#ifndef GWL_H
#define GWL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gwl_ctx gwl_ctx;

typedef enum {
  GWL_OK = 0,
  GWL_EINVAL = -1,        /* bad argument (sizes, ranges, NaN, null pointer) */
  GWL_ENOMEM = -2,        /* device allocation failed */
  GWL_EDEVICE = -3,       /* HIP runtime error */
  GWL_ENUMERIC = -4,      /* non-finite Lanczos coefficient, interval violated */
  GWL_ESTATE = -5,        /* call not valid in the context's state */
  GWL_EUNSUPPORTED = -6   /* grid size or option not supported */
} gwl_status;

/* Arithmetic of the pair-space product C x.  The Lanczos recurrence, the
 * Chebyshev combination, reorthogonalisation and the continued fraction are
 * FP64 in every mode. */
typedef enum {
  GWL_FP64 = 0,            /* GEMMs and FFT in FP64 */
  GWL_MIXED_F16 = 1,       /* both GEMMs on FP16 operands with FP32 accumulation; each
                              operand carries a power of two that puts it inside FP16's
                              range (pair vectors per batch, orbitals once, phi_v V_b
                              per pair vector from the maximum of its potential, which
                              the Poisson solve records); FFT in FP32 */
  GWL_MIXED_BF16X3 = 2,    /* three-term BF16 split of each operand: not built
                              (GWL_EUNSUPPORTED); the 16-bit path already meets the
                              1 meV bar on the smooth stress inputs */
  GWL_MIXED_FP32 = 3       /* FP32 operands: not built (GWL_EUNSUPPORTED); FP32
                              matrix throughput is twice FP64's, too little to
                              pay for the separate kernels */
} gwl_precision;

/* Reorthogonalisation of the Lanczos vectors (the paper does not prescribe
 * one; it notes resolvents are free of ghost eigenvalue problems). */
typedef enum {
  GWL_REORTH_NONE = 0,   /* plain three-term recurrence */
  GWL_REORTH_LOCAL = 1,  /* re-project against q_k and q_{k-1} */
  GWL_REORTH_FULL = 2    /* classical Gram-Schmidt against all q_j, with a second
                            pass for the slots whose first pass removed more than
                            half of ||w||^2 */
} gwl_reorth;

typedef struct {
  int nx, ny, nz;     /* grid points; each must factor into 2, 3, 4, 8 and be <= 256 */
  double lx, ly, lz;  /* periodic box edges, bohr (orthorhombic) */
} gwl_grid;

typedef struct {
  int precision;        /* gwl_precision, default GWL_FP64 */
  int poly_degree;      /* g, default 7 (the paper's Table 1 uses g = 7) */
  double poly_lo;       /* Chebyshev interval [lo, hi] in hartree^2; <= 0 selects */
  double poly_hi;       /*   lo = (min Delta)^2 and hi = Lanczos estimate of max eig C */
  int reorth;           /* gwl_reorth, default GWL_REORTH_FULL */
  int block;            /* number of concurrent Lanczos slots B; 0 = automatic */
  double kernel_scale;  /* multiplies 4 pi/|G|^2; default 1 (as printed; 0 = no coupling) */
  void* stream;         /* hipStream_t to run on; NULL = library-owned stream */
} gwl_options;

/* Fill *opts with the defaults listed above. */
void gwl_default_options(gwl_options* opts);

/* Create a context: validate the inputs, pack the orbitals into the GEMM
 * layouts, build Delta, the Coulomb factors and the Chebyshev coefficients.
 *   orbitals      [n_orb][nx*ny*nz] values, orb_dtype 8 = float64, 4 = float32;
 *                 host memory if orb_on_device == 0, else device memory.  The
 *                 library copies them into its own layouts, so the caller may
 *                 free them after the call.
 *   energies_ev   host [n_orb] KS energies; every empty energy must exceed
 *                 every occupied one (Delta_vc > 0).
 *   grid, opts    host structs; opts may be NULL for the defaults.
 *   out           receives the context; unchanged on failure.
 * Errors: GWL_EINVAL (n_occ not in [1, n_orb-1], NaN, Delta <= 0, null
 * pointers), GWL_EUNSUPPORTED (grid, or N_v N_c >= 2^31), GWL_ENOMEM,
 * GWL_EDEVICE. */
gwl_status gwl_setup(const void* orbitals, int orb_dtype, int orb_on_device,
                     int n_orb, int n_occ, const double* energies_ev,
                     const gwl_grid* grid, const gwl_options* opts,
                     gwl_ctx** out);

/* Sigma^corr_mm(w) for every m in qp_states (Eqs. 10-14).
 *   qp_states   host [n_qp] orbital indices m.
 *   omega_ev    host [n_omega] frequencies.
 *   eta_ev      broadening delta > 0 (the paper's delta; not its eta_n).
 *   n_lanczos   L >= 1: Lanczos steps = D-matvecs = diagonal entries a_k.
 *   sigma_out   host [n_qp][n_omega][2] (re, im), eV.
 * The n-sum runs over all n_orb orbitals, n = m included.  Each (m, n) run
 * ends early if b_{k+1} <= 1e-12 max_j |a_j| (exact invariant subspace).
 * Interval check: p_g approximates the square root only on [lo, hi] (the
 * paragraph after Eq. 12) and extrapolates wildly outside it.  After the
 * recurrence every run's tridiagonal T is tested by Sturm counts: an
 * eigenvalue of T above max p_g or below min p_g on [lo, hi] by more than
 * 0.5 % of max p_g means C has spectrum outside [lo, hi] that the start
 * vector sees (about 1 % beyond hi), and the call fails with GWL_ENUMERIC
 * instead of returning a corrupted Sigma (Tamm-Dancoff and quadrature runs
 * use no polynomial and are not tested).
 * Errors: GWL_EINVAL, GWL_ENUMERIC (non-finite coefficients, spectrum outside
 * the Chebyshev interval), GWL_EDEVICE. */
gwl_status gwl_sigma_c(gwl_ctx* ctx, const int* qp_states, int n_qp,
                       const double* omega_ev, int n_omega, double eta_ev,
                       int n_lanczos, double* sigma_out);

/* Off-diagonal Sigma^corr_mm2(w) of two states (the paper's closing remarks
 * point to a band Lanczos for off-diagonal elements).  The per-n term of
 * Eqs. 12-14 is a quadratic form in the Lanczos start vector, so the
 * bilinear form is a quarter of the difference of the runs from
 * P_nm + P_nm2 and P_nm - P_nm2 (polarisation identity): 2 n_orb Lanczos
 * runs of length n_lanczos, otherwise as gwl_sigma_c (the same precision,
 * Tamm-Dancoff, quadrature and ISDF options apply).  m2 = m gives
 * gwl_sigma_c's diagonal element.  sigma_out: host [n_omega][2] (re, im), eV.
 * Device scratch: 2 n_orb N_vc doubles for the start vectors, freed on
 * return.  Errors as gwl_sigma_c. */
gwl_status gwl_sigma_c_offdiag(gwl_ctx* ctx, int m, int m2, const double* omega_ev, int n_omega,
                               double eta_ev, int n_lanczos, double* sigma_out);

/* Partial sum of Eq. 10: for every m in qp_states, sigma_out[q][w] =
 * sum_{n = n_begin}^{n_end - 1} Sigma_mm(w, n), same units and layout as
 * gwl_sigma_c (which is the range [0, n_orb)).  Disjoint n-ranges add up to
 * the full self-energy, so a range is also the unit of work to spread over
 * several devices.  Errors as gwl_sigma_c, plus GWL_EINVAL for
 * 0 <= n_begin < n_end <= n_orb not holding. */
gwl_status gwl_sigma_c_range(gwl_ctx* ctx, const int* qp_states, int n_qp, int n_begin,
                             int n_end, const double* omega_ev, int n_omega, double eta_ev,
                             int n_lanczos, double* sigma_out);

/* Batched Lanczos over arbitrary (m, n) start vectors of uneven length
 * (Eq. 13), scheduled over the context's B slots with refill.
 *   m_idx, n_idx, lengths   host [n_pairs]; lengths in [1, 4000].
 *   alpha     host [n_pairs][ld]   a_0 .. a_{len-1} in hartree (rest zero)
 *   beta      host [n_pairs][ld]   b_1 .. b_{len-1} in hartree (rest zero)
 *   p_norm2   host [n_pairs]       ||P_nm||^2 in hartree^3
 *   out_len   host [n_pairs]       steps actually taken (< lengths on breakdown); may be NULL
 *   ld        leading dimension >= max(lengths). */
gwl_status gwl_lanczos_pairs(gwl_ctx* ctx, const int* m_idx, const int* n_idx,
                             const int* lengths, int n_pairs, double* alpha,
                             double* beta, double* p_norm2, int* out_len, int ld);

/* Continued fraction and assembly (Eqs. 12, 14) on the GPU for given
 * coefficients: sigma_out[p][w] = Sigma_mm(w, n_idx[p]) in eV for pair p,
 * with the same layouts as gwl_lanczos_pairs (host pointers). */
gwl_status gwl_sigma_from_coeffs(gwl_ctx* ctx, const int* n_idx, int n_pairs,
                                 const double* alpha, const double* beta,
                                 const double* p_norm2, const int* lens, int ld,
                                 const double* omega_ev, int n_omega,
                                 double eta_ev, double* sigma_out);

/* Allocation-free variant of gwl_sigma_from_coeffs, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts, units and
 * results (the same kernels); the device buffers it needs (the staged
 * coefficients, per-pair energies and signs, frequencies in hartree and the
 * per-pair Sigma) are carved from one static 32 MiB array per device
 * instead of the context's allocations, so it calls no hipMalloc, hipFree or
 * other allocating routine.  Need, in bytes, each of its ten pieces rounded
 * up to 256: 16 n_pairs (ld + n_omega + 2) + 8 (n_orb + n_omega); more is
 * GWL_EINVAL with the figure in gwl_last_error.  Every call on a device
 * shares that device's array and leaves its contents behind; each call
 * writes every byte it reads first.  Calls that can overlap on one device
 * (from several threads, whatever their contexts or streams) race; calls
 * made one after another do not.  The polynomial continued fraction
 * and the Tamm-Dancoff option are covered; the quadrature option returns
 * GWL_EUNSUPPORTED.  The current device must be the context's (GWL_EINVAL
 * otherwise).  Synchronous on the context stream. */
gwl_status gwl_sigma_from_coeffs_noalloc(gwl_ctx* ctx, const int* n_idx, int n_pairs,
                                         const double* alpha, const double* beta,
                                         const double* p_norm2, const int* lens, int ld,
                                         const double* omega_ev, int n_omega,
                                         double eta_ev, double* sigma_out);

/* Vector-Jacobian product of the self-energy (reverse-mode derivative).
 * For the scalar l = sum_{q,w} Re(conj(G_qw) Sigma_q(w)) with
 *   grad_sigma  host [n_qp][n_omega][2]: G (re, im), per eV of Sigma,
 * returns
 *   grad_energies  host [n_orb]: dl/de_a (per eV of energy),
 *   grad_orbitals  device [n_orb][nx*ny*nz] in the orbitals' type (float64,
 *                  or float32 when gwl_setup was given FP32 orbitals):
 *                  dl/dphi_a(r), accumulated in FP64,
 *   sigma_out      host [n_qp][n_omega][2] or NULL: the forward Sigma (eV).
 * The forward is the path of gwl_sigma_c in FP64 with the three-term
 * recurrence only (no reorthogonalisation, so the Lanczos vectors can be
 * recomputed exactly); the derivative is exact for that forward.  The
 * backward needs, per step k, q_k, p_g(C) q_k, the Chebyshev iterates of that
 * product and the Hartree potentials formed inside it.  By default the
 * forward keeps only (q_{k-1}, q_k) every ceil(sqrt(L)) steps and the
 * backward recomputes one such segment at a time (one more p_g(C) product
 * per step), except the last, whose iterates the forward keeps as it ends;
 * with GWL_KEY_ADJOINT_STORE = 1 the forward keeps the whole run when it fits
 * in GWL_ADJOINT_STORE_MAX.  The orbital gradient is contracted
 * step by step from the outer products of the reverse sweep with the FP64
 * matrix-core kernel (no N_vc x N_vc matrix is formed); device memory
 * beyond the context's is about
 *   ceil(sqrt(L)) [(2g + 2) B N_vc + g B N_r] + g B (N_r + 2 N_v N_c)
 *   + (N_v + N_c + N_v N_c / 64) N_r  doubles  (B = block, default 64).
 * Orbitals are free variables (no orthonormality constraint), occupations
 * and the Chebyshev interval [lo, hi] are held fixed.  n_lanczos <= 1024.
 * The paper defines the forward (Eqs. 7-14); the adjoint is this library's. */
gwl_status gwl_sigma_c_vjp(gwl_ctx* ctx, const int* qp_states, int n_qp,
                           const double* omega_ev, int n_omega, double eta_ev, int n_lanczos,
                           const double* grad_sigma, double* sigma_out,
                           double* grad_energies, void* grad_orbitals);

/* The same derivative for the partial sum over n in [n_begin, n_end) that
 * gwl_sigma_c_range returns (gwl_sigma_c_vjp is the range [0, n_orb)):
 * l = sum_{q,w} Re(conj(G_qw) sum_{n_begin <= n < n_end} Sigma_qq(w, n)).
 * Arguments, outputs and errors as gwl_sigma_c_vjp, plus GWL_EINVAL unless
 * 0 <= n_begin < n_end <= n_orb. */
gwl_status gwl_sigma_c_range_vjp(gwl_ctx* ctx, const int* qp_states, int n_qp, int n_begin,
                                 int n_end, const double* omega_ev, int n_omega, double eta_ev,
                                 int n_lanczos, const double* grad_sigma, double* sigma_out,
                                 double* grad_energies, void* grad_orbitals);

/* The same derivative in two calls, for callers that evaluate Sigma first
 * and differentiate later (an autograd forward and backward).
 * gwl_sigma_c_vjp_forward runs the forward of gwl_sigma_c_range_vjp for
 * qp_states x [n_begin, n_end) (arguments as there; [0, n_orb) is the full
 * sum), writes the forward Sigma to sigma_out (host [n_qp][n_omega][2], eV,
 * required) and keeps in the context, per block of start vectors, the
 * recurrence's checkpoints (q_{k-1}, q_k and the slot state every
 * ceil(sqrt(L)) steps), the start vectors P_nm and the potentials
 * V[phi_n phi_m], and per pair the Lanczos coefficients:
 *   (2 ceil(L / ceil(sqrt(L))) + 1) P N_vc + P N_r + 2 P L  doubles
 * for P = n_qp (n_end - n_begin) start vectors (GWL_KEY_ADJOINT_STORE does
 * not apply).  The state is kept until the next gwl_sigma_c_vjp_forward on
 * the context or gwl_destroy.
 * gwl_sigma_c_vjp_backward then returns grad_energies and grad_orbitals for
 * the cotangent grad_sigma ([n_qp][n_omega][2], host) exactly as
 * gwl_sigma_c_range_vjp would with the same arguments (the same kernels in
 * the same order), recomputing every segment from the kept checkpoints
 * instead of running the forward again; it may be called several times.
 * Errors: as gwl_sigma_c_range_vjp; gwl_sigma_c_vjp_backward returns
 * GWL_EINVAL when no forward was kept, or when the interval, polynomial
 * degree, block size, GEMM split or kernel choice of the context changed
 * since (the recompute must repeat the forward's arithmetic). */
gwl_status gwl_sigma_c_vjp_forward(gwl_ctx* ctx, const int* qp_states, int n_qp, int n_begin,
                                   int n_end, const double* omega_ev, int n_omega, double eta_ev,
                                   int n_lanczos, double* sigma_out);
gwl_status gwl_sigma_c_vjp_backward(gwl_ctx* ctx, const double* grad_sigma,
                                    double* grad_energies, void* grad_orbitals);

/* ---- component entry points (the steps of the path, for parity checks) ---- */

/* Hartree potential V = FFT^-1[kernel_scale 4 pi/|G|^2 FFT[rho]] of n_fields
 * real densities.  rho, v: device [n_fields][nx*ny*nz] in float64 if
 * precision == GWL_FP64, float32 if GWL_MIXED_F16. */
gwl_status gwl_poisson(gwl_ctx* ctx, const void* rho, void* v, int n_fields,
                       int precision);

/* Pair densities of the factored product, the first GEMM with its fused
 * row-dot (the density of Eqs. 2-3 for a pair vector):
 *   rho_b(r) = sum_vc phi_v(r) phi_c(r) u_b,vc,  u = Delta^1/2 x
 * (u = x under the Tamm-Dancoff option), for n_vec pair vectors in batches
 * of up to 128.  x: device float64 [n_vec][N_v*N_c]; rho: device float64
 * [n_vec][N_r] (the caller's buffers).  GWL_MIXED_F16: FP16 operands, FP32
 * accumulation, the operand scales divided out in FP64.  GWL_EUNSUPPORTED
 * while the ISDF product is switched on. */
gwl_status gwl_pair_density(gwl_ctx* ctx, const double* x, double* rho, int n_vec,
                            int precision);

/* The second GEMM alone (the back-projection of Eqs. 2-3): for n_vec
 * potentials V_b on the grid,
 *   y_b,vc = dV sum_r phi_v(r) V_b(r) phi_c(r)
 * (with V_b the Hartree potential of a pair density this is (K u_b)_vc), in
 * batches of up to 128.  v: device float64 [n_vec][N_r]; y: device float64
 * [n_vec][N_v*N_c] (the caller's buffers).  GWL_MIXED_F16: each V_b is scaled
 * by the power of two the Poisson solve would give it and rounded to FP16,
 * phi_v V_b is formed in FP16, sums in FP32, scales divided out in FP64.
 * GWL_EUNSUPPORTED while the ISDF product is switched on. */
gwl_status gwl_potential_product(gwl_ctx* ctx, const double* v, double* y, int n_vec,
                                 int precision);

/* y = C x for n_vec pair vectors (Eq. 4), factored on the grid.
 * x, y: device float64 [n_vec][N_v*N_c]. */
gwl_status gwl_apply_c(gwl_ctx* ctx, const double* x, double* y, int n_vec,
                       int precision);

/* y = p_g(C) x, the Chebyshev approximation of D x.  Layout as gwl_apply_c. */
gwl_status gwl_apply_d(gwl_ctx* ctx, const double* x, double* y, int n_vec,
                       int precision);

/* Interpolative separable density fitting of the pair densities (Eqs. 15-17)
 * at n_mu caller-chosen grid points (host [n_mu], strictly increasing indices
 * into the C-order grid, z fastest): coefficients C^mu_vc = phi_v(r_mu)
 * phi_c(r_mu), auxiliary functions zeta = Z C^T (C C^T)^-1 (least-squares
 * fit of the pair densities Z), two-centre integrals M = dV zeta^T V[zeta].
 * Afterwards (and whenever GWL_KEY_ISDF is 1) every K product uses
 * K = C^T M C: the first and second GEMMs run on the N_mu sampled orbital
 * values and a dense (M / dV) product replaces the FFT Poisson solve.  The
 * coupling integrals (nm|vc) stay exact on the grid.  An estimated interval
 * (poly_hi <= 0 at setup) is estimated again for the ISDF operator.  Device
 * memory during setup: about 3 N_r N_mu doubles.  GWL_ENUMERIC when C C^T is
 * not numerically positive definite at the points.  The ISDF product runs in
 * FP64 only (GWL_EUNSUPPORTED for the mixed precision): summing over N_mu
 * points instead of N_r averages the 16-bit operand rounding over far fewer
 * terms. */
gwl_status gwl_isdf_setup(gwl_ctx* ctx, const int* points, int n_mu);

/* Interpolation points for gwl_isdf_setup by weighted K-means over the grid
 * (the paper names ISDF but not its point selection; this is the centroidal
 * Voronoi reading).  Weight w(r) = (sum_v phi_v(r)^2)(sum_c phi_c(r)^2) of
 * the context's orbitals, quantised to integers (2^30 at its maximum) so that
 * cluster sums are exact; Lloyd iterations from the n_init initial centroids
 * init_points (host, grid indices r = (x n_y + y) n_z + z, repeats allowed)
 * under the periodic minimum-image distance, ties to the lower centroid; a
 * centroid moves to the W-weighted mean of its members (displacements wrapped
 * into [-n/2, n/2) about its nearest grid point); stops when an assignment
 * repeats the previous one or after max_iter updates.  Each non-empty cluster
 * gives its member nearest the centroid (ties to the lower index).
 * points_out: host [n_init], receives *n_points <= n_init strictly increasing
 * indices (ready for gwl_isdf_setup); *n_assign: assignment passes made.
 * FP64, deterministic bit for bit; device scratch about 28 bytes per grid
 * point, allocated and freed by the call.  GWL_EINVAL for bad arguments or
 * weights that vanish everywhere. */
gwl_status gwl_isdf_kmeans(gwl_ctx* ctx, const int* init_points, int n_init, int max_iter,
                           int* points_out, int* n_points, int* n_assign);

/* Interpolation points for gwl_isdf_setup by column-pivoted QR (the
 * selection the interpolative decomposition uses).  The pair densities
 * Z[(vc), r] = phi_v(r) phi_c(r) of the context's orbitals are sketched with
 * the caller's random factors (gv host [N_v][p], gc host [N_c][p], row-major;
 * the library draws no random numbers):
 *   S[r][k] = (sum_v gv[v][k] phi_v(r)) (sum_c gc[c][k] phi_c(r)),
 * and n_mu steps of column-pivoted Gram-Schmidt over the grid points take,
 * each time, the point whose residual column of S has the largest norm
 * (ties to the lower index), then project its normalised column out of all
 * others (a zero residual is taken without projecting).  points_out: host
 * [n_mu], the pivots in increasing order (ready for gwl_isdf_setup).  FP64,
 * on the device, reproducible bit for bit; device scratch N_r p + 2 N_r
 * doubles, allocated and freed by the call.  GWL_EINVAL unless
 * 1 <= n_mu <= p and n_mu <= N_r; GWL_EUNSUPPORTED for p > 8192 or a sketch
 * over 64 GB. */
gwl_status gwl_isdf_qrcp(gwl_ctx* ctx, const double* gv, const double* gc, int p, int n_mu,
                         int* points_out);

/* Exchange part of the self-energy, Sigma^ex_mm = -sum_v (vm|vm) (Eq. 6; the
 * frequency-independent term of Eq. 5), in eV, for n_qp states: pair
 * densities phi_v phi_m on the grid, the same FFT Poisson solve and kernel as
 * the correlation part (FP64 throughout), and a fixed-order grid sum.
 * qp_states: host [n_qp], 0-based orbital indices; sigma_x_out: host [n_qp].
 * Independent of the precision and Tamm-Dancoff options. */
gwl_status gwl_sigma_x(gwl_ctx* ctx, const int* qp_states, int n_qp, double* sigma_x_out);

/* Quasiparticle energy from the graphical solution of the G0W0 equation
 * E = eps + Sigma^ex + Re Sigma^corr(E) - v_xc on a frequency grid (the
 * paper evaluates Eq. 14 for a series of frequencies for this purpose):
 * the zeros of f(w) = eps + sigma_x + Re sigma_c(w) - vxc - w are located by
 * sign changes between neighbouring grid points and linear interpolation; the
 * root nearest eps is returned in *e_qp with the renormalisation factor
 * *z = 1 / (1 - d Re Sigma^corr / dw) from the slope of that segment.
 * omega_ev: host [n_omega], strictly increasing, n_omega >= 2; sigma_c: host
 * [n_omega][2] (real, imaginary) eV, as returned by gwl_sigma_c; all energies
 * in eV; v_xc comes from the mean-field calculation.  Host only (no context,
 * no device work).  GWL_ENUMERIC (with NaN outputs) when f never changes sign
 * on the grid. */
gwl_status gwl_qp_solve(const double* omega_ev, int n_omega, const double* sigma_c,
                        double eps_ev, double sigma_x_ev, double vxc_ev, double* e_qp,
                        double* z);

/* Coupling vectors P_nm = (nm|vc) Delta^1/2 for count (m, n) pairs.
 * m_idx, n_idx host [count]; p: device float64 [count][N_v*N_c]. */
gwl_status gwl_coupling(gwl_ctx* ctx, const int* m_idx, const int* n_idx,
                        int count, double* p);

/* ---- options, queries, lifetime ---- */

/* Change one option of an existing context (keys below; the value is cast). */
gwl_status gwl_set_option(gwl_ctx* ctx, int key, double value);

/* Read one scalar (keys below) into *out. */
gwl_status gwl_query(gwl_ctx* ctx, int key, double* out);

enum {
  GWL_KEY_PRECISION = 1,   /* set/query */
  GWL_KEY_REORTH = 2,      /* set/query */
  GWL_KEY_BLOCK = 3,       /* set/query: Lanczos slots B */
  GWL_KEY_POLY_LO = 4,     /* query: interval lower end, hartree^2 */
  GWL_KEY_POLY_HI = 5,     /* query: interval upper end, hartree^2 */
  GWL_KEY_POLY_DEGREE = 6, /* query */
  GWL_KEY_N_VC = 7,        /* query: N_v * N_c */
  GWL_KEY_LAST_MS_TOTAL = 9,    /* query: wall ms of the last sigma/lanczos call */
  GWL_KEY_LAST_C_MATVECS = 10,  /* query: vector C-products of the last call */
  GWL_KEY_GEMM_SPLITK = 11,     /* set/query: split of the grid sum in the second GEMM, 0 = auto */
  GWL_KEY_KERNELS = 12,         /* set/query: 1 = MFMA GEMMs (default), 0 = plain FMA tiles */
  GWL_KEY_PROFILE = 13,         /* set/query: 1 = time each GEMM / Poisson launch with HIP
                                   events on the context stream (totals below, per call) */
  GWL_KEY_PROF_MS_GEMM1 = 14,   /* query: summed event ms of first-GEMM launches, last call */
  GWL_KEY_PROF_N_GEMM1 = 15,    /* query: number of those launches */
  GWL_KEY_PROF_VEC_GEMM1 = 16,  /* query: pair vectors processed by those launches */
  GWL_KEY_PROF_MS_GEMM2 = 17,   /* query: same for the second GEMM */
  GWL_KEY_PROF_N_GEMM2 = 18,
  GWL_KEY_PROF_VEC_GEMM2 = 19,
  GWL_KEY_PROF_MS_FFT = 20,     /* query: same for the Poisson solve (all five passes) */
  GWL_KEY_PROF_N_FFT = 21,
  GWL_KEY_PROF_VEC_FFT = 22,
  GWL_KEY_GRAPHS = 23,          /* set/query: 1 (default) = replay a captured HIP graph of the
                                   p_g(C) product each Lanczos step; 0 = launch eagerly.
                                   Graphs are not used while GWL_KEY_PROFILE is on. */
  GWL_KEY_TUNED_BLOCK = 24,     /* query: slots B chosen by the autotuner (block = 0) for the
                                   current precision, 0 before the first tuned call */
  GWL_KEY_TUNED_SPLITK = 25,    /* query: split chosen with it */
  GWL_KEY_BF16_TILE = 26,       /* set/query: block tile width of the second BF16 GEMM, 256
                                   (default: one wave per SIMD, accumulators in AGPRs) or
                                   128 (two waves per SIMD) */
  GWL_KEY_TDA = 27,             /* set/query: 0 (default) = the full method above; 1 =
                                   Tamm-Dancoff approximation (B = 0 in the Casida matrix,
                                   the variant the paper's closing discussion names): the
                                   Lanczos operator is A = Delta + K (no square root, no
                                   polynomial; the interval is unused), start vectors are
                                   k_nm = (nm|vc) (gwl_coupling returns these), and
                                   Sigma(w, n) = -eta_n R_A(-eta_n z_n).  Applies to
                                   gwl_sigma_c, gwl_sigma_c_range, gwl_lanczos_pairs,
                                   gwl_sigma_from_coeffs and gwl_coupling; gwl_apply_c and
                                   gwl_apply_d keep their meaning; gwl_sigma_c_vjp returns
                                   GWL_EUNSUPPORTED while it is set. */
  GWL_KEY_QUADRATURE = 28,      /* set/query: 0 (default) = Lanczos on D = p_g(C) (Eqs. 12-14);
                                   1 = Lanczos on C itself from P_nm, n_lanczos counting
                                   C-products, and Sigma(w, n) evaluated by the Gauss
                                   quadrature of the tridiagonal T (Ritz values theta_k,
                                   weights ||P||^2 u_k(0)^2 from an implicit QL iteration):
                                   sum_k w_k [theta_k^-1/2 - (theta_k^1/2 + eta_n z_n)^-1] / z_n,
                                   i.e. Eq. 11 with the spectral measure of C probed directly,
                                   without the polynomial fit of the square root.  Applies to
                                   gwl_sigma_c, gwl_sigma_c_range, gwl_lanczos_pairs and
                                   gwl_sigma_from_coeffs; ignored while GWL_KEY_TDA is set;
                                   FP64 only (the Ritz-value quadrature amplifies the mixed
                                   product's rounding: 5e-3 eV at L = 28 on a smooth test
                                   case), so the mixed precision returns GWL_EUNSUPPORTED;
                                   gwl_sigma_c_vjp returns GWL_EUNSUPPORTED while it is set. */
  GWL_KEY_ISDF = 29,            /* set/query: 1 = the K product on the ISDF points of the last
                                   gwl_isdf_setup (GWL_ESTATE before one), 0 = on the grid */
  GWL_KEY_ISDF_NMU = 30,        /* query: number of ISDF points set up, 0 if none */
  GWL_KEY_TUNED_TILE = 31,      /* query: second-GEMM block tile (128 or 256) chosen by the
                                   autotuner with GWL_KEY_TUNED_BLOCK (the mixed product
                                   picks it unless GWL_KEY_BF16_TILE was set), 0 before */
  GWL_KEY_ADJOINT_STORE = 32,   /* set/query: 0 (default) = gwl_sigma_c_vjp recomputes the
                                   Lanczos vectors from checkpoints every ceil(sqrt(L))
                                   steps; 1 = it keeps every step's iterates and potentials
                                   from its forward when they fit in GWL_ADJOINT_STORE_MAX
                                   bytes and that much device memory can be allocated
                                   (else it recomputes).  Both give bitwise the same
                                   results. */
  GWL_KEY_ADJOINT_STORED = 33,  /* query: 1 if the last gwl_sigma_c_vjp call kept the
                                   iterates, 0 if it recomputed them, -1 before a call */
  GWL_KEY_HI_RESIDUAL = 34,     /* query: residual bound |b_40 u_40| of the largest Ritz
                                   value in the last estimate of the interval's upper end
                                   (hartree^2; 0 when no estimate ran or the recurrence
                                   ended in an invariant subspace) */
  GWL_KEY_SCHEDULER = 35        /* set/query: 1 (default) = the batched Lanczos runs play the
                                   whole refill schedule out on the host first (a slot runs
                                   its start vector for exactly its length), upload it once
                                   and then only queue work: no host synchronisation inside
                                   the loop, and steps without a refill or a change of the
                                   busy slots replay one graph of the whole step (product,
                                   a_k, reorthogonalisation, b_{k+1}); 0 = the host-driven
                                   loop (a synchronisation and host copies per refill, the
                                   vector kernels launched eagerly).  Same coefficients. */
};

/* Device-memory cap for the run kept by gwl_sigma_c_vjp with
 * GWL_KEY_ADJOINT_STORE: per Lanczos step 2g + 2 vectors of B x N_vc doubles
 * (the iterates t_0..t_g, their coupling parts K Delta^1/2 t_j for j < g, and
 * p_g(C) q_k) and g x B Hartree potentials on the grid. */
#define GWL_ADJOINT_STORE_MAX (32ull << 30)
/* The autotuner runs on the first gwl_sigma_c / gwl_sigma_c_range /
 * gwl_lanczos_pairs call with block = 0: it times one C-product for
 * B in {32, 64, 128, 256} and three splits of the second GEMM, and for the
 * mixed product both block tiles of the second GEMM (unless
 * GWL_KEY_BF16_TILE fixed one).  If the environment variable GWL_TUNE_CACHE
 * names a file, choices are read from and appended to it (text lines
 * "gfx950:N_r:N_v:N_c:precision:kernels:fixed_tile:n_mu B split tile us"). */

/* Message of the last failing call on this thread ("" if none). */
const char* gwl_last_error(void);

/* Free every device allocation of the context.  NULL is ignored. */
void gwl_destroy(gwl_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GWL_H */
