/*
 * lqcd.h - C ABI of the MI355X (gfx950) library for disconnected-loop
 * noise estimation with deflation, perturbative and polynomial subtraction
 * (Baral, Whyte, Wilcox, Morgan, "Disconnected Loop Subtraction Methods in
 * Lattice QCD", arXiv:1903.06986).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice extents dims = {Lx, Ly, Lz, Lt}, each even and >= 2, periodic in
 * all four directions (Sec. 7).  Directions mu = 0..3 are x, y, z, t.
 *
 * External ("LEX") fields are complex128 (interleaved re, im doubles) in
 * lexicographic order [rhs][t][z][y][x][spin][colour]: vector index
 * (s * 4 + spin) * 3 + colour with s = x + Lx (y + Ly (z + Lz t)), the
 * "space-time-color-Dirac" index of Sec. 2.  A field of one right-hand side
 * holds 12 V complex numbers, V = Lx Ly Lz Lt.
 *
 * Links are complex128 [t][z][y][x][mu][row][col] (host memory at create).
 *
 * Gamma matrices: Euclidean, hermitian, chiral basis
 *   g_k = [[0, -i s_k], [i s_k, 0]] (k = 1..3), g_4 = [[0, 1], [1, 0]],
 *   g_5 = g_1 g_2 g_3 g_4 = diag(1, 1, -1, -1).
 * Operators Theta are coded 0 = identity (scalar), 1..4 = g_1..g_4
 * (local vector); Table 2 of the paper.
 *
 * Memory: every field pointer (eta, x, xt, b, in, out) is device memory
 * owned by the caller, read and written on the context's HIP stream.  Host
 * pointers are named *_host or documented as host.  The library owns only
 * the opaque handles and their internal device workspaces.
 *
 * Errors: every call returns an lqcd_status, never aborts and never throws;
 * lqcd_last_error() gives a thread-local message for the last failure.
 * Calls on one context are not thread-safe; use one context per thread.
 * A deflation space (lqcd_defl) may serve several contexts of its lattice
 * and kappa, also from different threads at once: the caches it fills on
 * first use are filled once, under a lock, and complete before any other
 * context reads them.  All users of one space take the same number of
 * eigenpairs Q.
 */
#ifndef LQCD_H
#define LQCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lqcd_ctx lqcd_ctx;
typedef struct lqcd_defl lqcd_defl;

typedef enum {
  LQCD_OK = 0,
  LQCD_EINVAL = 1,      /* invalid argument (null pointer, odd extent, bad enum) */
  LQCD_ENOMEM = 2,      /* device or host allocation failed */
  LQCD_EDEVICE = 3,     /* HIP runtime error */
  LQCD_ENOCONV = 4,     /* solver hit its iteration limit; x holds the best iterate */
  LQCD_EBREAKDOWN = 5,  /* Arnoldi breakdown (zero subdiagonal) */
  LQCD_ENAN = 6         /* NaN or Inf met in a norm */
} lqcd_status;

typedef enum { LQCD_F64 = 0, LQCD_F32 = 1, LQCD_F16 = 2, LQCD_BF16 = 3 } lqcd_prec;

/* Operators of wilson_apply (Sec. 5.1 Eqs. (24)-(25); Sec. 5.4 Eq. (63);
 * the even/odd reduction of Sec. 7):
 *   LQCD_OP_M      M psi     = psi - kappa P psi
 *   LQCD_OP_MDAG   M^+ psi   = g5 M g5 psi
 *   LQCD_OP_MG5    M' psi    = M g5 psi  (hermitian)
 *   LQCD_OP_HOP    P psi,  (P psi)(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                     + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *   LQCD_OP_SCHUR  Mhat psi_e = psi_e - kappa^2 D_eo D_oe psi_e on even
 *                  sites; odd sites of the output are set to zero. */
typedef enum {
  LQCD_OP_M = 0, LQCD_OP_MDAG = 1, LQCD_OP_MG5 = 2, LQCD_OP_HOP = 3, LQCD_OP_SCHUR = 4
} lqcd_op;

/* LQCD_LAYOUT_LEX: complex128 lexicographic fields as above.
 * LQCD_LAYOUT_EO:  the library's internal even/odd layout in the requested
 *   precision (for timing the stencil alone): per right-hand side, parity
 *   blocks [parity][12][V/2] of complex numbers (component-major, so that
 *   consecutive sites are consecutive in memory); LQCD_OP_SCHUR uses only
 *   the even block, [12][V/2] per right-hand side. */
typedef enum { LQCD_LAYOUT_LEX = 0, LQCD_LAYOUT_EO = 1 } lqcd_layout;

/* Subtraction methods (Sec. 5): no subtraction, perturbative, polynomial,
 * hermitian-forced eigenvalue, and the two combinations of Sec. 5.5. */
typedef enum {
  LQCD_NS = 0, LQCD_PS = 1, LQCD_POLY = 2, LQCD_HFES = 3, LQCD_HFPS = 4, LQCD_HFPOLY = 5
} lqcd_method;

/* Modes of deflate_project. */
typedef enum {
  LQCD_DEFL_HFES = 0,     /* weights 1/lambda'_q (Eqs. (66)-(68)) */
  LQCD_DEFL_EIGPOLY = 1,  /* weights 1/lambda'_q - 1/xi'_q for a polynomial (Eqs. (69)-(72)) */
  LQCD_DEFL_ES = 2        /* eigenvalue subtraction (Sec. 5.3) with the even/odd deflation
                             space: right/left eigenvectors of M, weights 1/lambda_q */
} lqcd_defl_mode;

typedef struct {
  int m;             /* Krylov subspace size of GMRES-DR (m > k >= 1) */
  int k;             /* number of deflated (harmonic Ritz) vectors kept */
  int max_cycles;    /* restart-cycle limit per right-hand side */
  double tol;        /* relative true residual |b - A x| / |b| target */
  double tol_super;  /* first right-hand side: residual target of the super-converged solve */
  double eig_tol;    /* first right-hand side: also continue until the n_eig smallest harmonic
                        Ritz pairs satisfy |A y - theta y| <= eig_tol |theta| (0 = off) */
  int n_eig;         /* see eig_tol (0 = k) */
  lqcd_prec inner;   /* precision of the inner Krylov solver: F64 = plain FP64,
                        F32 = FP32 stencil and basis inside FP64 iterative refinement,
                        F16 / BF16 = as F32, with the GMRES(m-k) basis and the
                        stencil's input stored in 16 bits with one FP32 scale per
                        site (arithmetic FP32; op LQCD_OP_SCHUR only) */
  double inner_tol;  /* relative residual reduction per refinement step (mixed precision) */
  int rhs_block;     /* right-hand sides solved together by GMRES-Proj (>= 1) */
  int proj_m;        /* GMRES cycle length of GMRES-Proj (0 = m - k) */
  int method;        /* solver of the first right-hand side: LQCD_KRYLOV_GMRESDR
                        (0) or LQCD_KRYLOV_MINRESDR (1, hermitian LQCD_OP_MG5
                        only); later right-hand sides always use GMRES-Proj */
} lqcd_solve_params;

/* First-right-hand-side solvers (Sec. 7 and Sec. 8).  GMRES-DR(m, k):
 * Arnoldi with classical Gram-Schmidt applied twice, least-squares
 * update, restart with the k harmonic Ritz vectors of smallest |theta| and
 * the residual direction.  MINRES-DR(m, k), used by the paper for the
 * hermitian M' near the critical kappa: the same deflated restarting with a
 * Lanczos three-term recurrence inside a cycle (the first new column after
 * a restart against all kept vectors; each later vector against v_{j-1},
 * v_j, then once more against those and the k + 1 kept vectors), and
 * harmonic Ritz pairs from the hermitian-definite pencil
 * H_m g = mu Hbar_m^H Hbar_m g, theta = 1 / mu, which needs no solve with
 * H_m (singular when a Ritz value of the indefinite M' crosses zero). */
typedef enum { LQCD_KRYLOV_GMRESDR = 0, LQCD_KRYLOV_MINRESDR = 1 } lqcd_krylov;

typedef struct {
  int matvecs;       /* applications of the solved operator (any precision) */
  int cycles;        /* restart cycles (GMRES-DR or GMRES(m-k) cycles of GMRES-Proj) */
  int refinements;   /* FP64 residual recomputations (mixed precision) */
  int reorth;        /* Arnoldi steps whose Gram-Schmidt needed the second pass (DGKS test) */
  double true_resid; /* final |b - A x| / |b| recomputed in FP64 on the full lattice */
} lqcd_solve_stats;

/* Create a context for one lattice on the current HIP device.
 * dims: host int[4]; links_host: host complex128 [V][4][3][3] (not retained);
 * kappa: hopping parameter of Eq. (24); hip_stream: hipStream_t or NULL
 * (the null stream).  Packs the links into the device even/odd layout in
 * FP64 and FP32.  EINVAL for odd or < 2 extents or null pointers. */
lqcd_status lqcd_create(const int dims[4], const double *links_host, double kappa,
                        void *hip_stream, lqcd_ctx **out);
lqcd_status lqcd_set_kappa(lqcd_ctx *ctx, double kappa);
lqcd_status lqcd_set_stream(lqcd_ctx *ctx, void *hip_stream);
lqcd_status lqcd_destroy(lqcd_ctx *ctx);

/* Z(4) noise (Sec. 2): eta^(n)_i = i^k, k = top two bits of the
 * (n * 12V + i)-th output of SplitMix64 seeded with `seed` (Steele, Lea and
 * Flood 2014, Vigna's formulation), for n = first .. first + nrhs - 1.
 * eta: device complex128 LEX [nrhs][12V]; codes: optional device uint8
 * [nrhs][12V] receiving k (may be NULL). */
lqcd_status lqcd_noise_z4(lqcd_ctx *ctx, uint64_t seed, int64_t first, int nrhs,
                          void *eta, uint8_t *codes);

/* Layout conversion between LEX complex128 and the internal even/odd layout
 * (LQCD_LAYOUT_EO, precision prec) for nrhs full fields. */
lqcd_status lqcd_pack_eo(lqcd_ctx *ctx, lqcd_prec prec, const void *lex, void *eo, int nrhs);
lqcd_status lqcd_unpack_eo(lqcd_ctx *ctx, lqcd_prec prec, const void *eo, void *lex, int nrhs);

/* out = g5 in for nrhs LEX complex128 fields (device; in == out allowed),
 * g5 = diag(1, 1, -1, -1) in spin (Sec. 2).  With M' = M g5 hermitian,
 * M^{-1} = g5 M'^{-1}: a right-hand side solved with LQCD_OP_MG5 gives the
 * solution of M through this call (the single-special-right-hand-side
 * production setup of Sec. 10, where the hermitian modes deflate every
 * solve). */
lqcd_status lqcd_gamma5(lqcd_ctx *ctx, const void *in, void *out, int nrhs);

/* Apply an operator (see lqcd_op) to nrhs fields.  With LQCD_LAYOUT_LEX,
 * in/out are complex128 LEX fields and the stencil runs in precision prec
 * (inputs rounded to prec, outputs widened to FP64).  With LQCD_LAYOUT_EO
 * they are internal-layout fields of precision prec.  in and out must not
 * overlap.  F16 / BF16 (op LQCD_OP_SCHUR with LQCD_LAYOUT_LEX only, else
 * EINVAL): the even half of the input is rounded to FP32 and stored in 16
 * bits with one FP32 scale per site (its largest |re| or |im|); the
 * stencil reads that storage and computes in FP32. */
lqcd_status wilson_apply(lqcd_ctx *ctx, lqcd_op op, lqcd_prec prec, lqcd_layout layout,
                         const void *in, void *out, int nrhs);

/* Deflated restarted GMRES (Sec. 7: GMRES-DR(m,k) for the first noise vector
 * solved to super-convergence, GMRES-Proj for the rest; Sec. 5.4 for the
 * hermitian system).
 * op = LQCD_OP_SCHUR: solves M x = b through the even/odd reduced system;
 *      x is the full solution.
 * op = LQCD_OP_MG5:   solves M' x = b on the full lattice (hermitian).
 * b, x: device complex128 LEX [nrhs][12V]; x is output only (zero start).
 * defl_inout: if *defl_inout is NULL the first right-hand side is solved by
 *   GMRES-DR and its deflation space (V_{k+1}, Hbar_k with A V_k =
 *   V_{k+1} Hbar_k) is returned in *defl_inout (free with lqcd_defl_free);
 *   every other right-hand side is solved by GMRES-Proj over that space.
 * stats: host array [nrhs] or NULL.
 * ENOCONV if any right-hand side misses tol within max_cycles, and when the
 * first right-hand side's GMRES-DR / MINRES-DR reaches max_cycles before
 * its own targets (tol_super, and eig_tol when set).  x then holds the
 * iterates and stats the counts; a deflation space built by the call is
 * still returned in *defl_inout. */
lqcd_status gmresdr_solve(lqcd_ctx *ctx, lqcd_op op, const lqcd_solve_params *params,
                          const void *b, void *x, int nrhs, lqcd_defl **defl_inout,
                          lqcd_solve_stats *stats);

/* Eigenpairs held by a deflation space of the hermitian operator M'
 * (op LQCD_OP_MG5): Rayleigh-Ritz in V_k (Sec. 5.4), the Q of smallest
 * |lambda'|.  lambda_host: host double [Q]; resid_host: host double [Q]
 * (|M' e - lambda' e|) or NULL. */
lqcd_status lqcd_defl_eigpairs(lqcd_ctx *ctx, lqcd_defl *defl, int Q, double *lambda_host,
                               double *resid_host);
/* Harmonic Ritz values of a deflation space: host complex128 [k]. */
lqcd_status lqcd_defl_ritz(const lqcd_defl *defl, double *theta_host, int *k_out);
void lqcd_defl_free(lqcd_defl *defl);

/* Hermitian-forced deflation (Sec. 5.4 Eqs. (66)-(68); Sec. 5.5 Eqs. (69)-(72)).
 * With (lambda'_q, e'_q) the Q lowest eigenpairs of M' in defl (op MG5) and
 * weights w_q = 1/lambda'_q (mode HFES) or w_q = 1/lambda'_q - 1/xi'_q
 * (mode EIGPOLY, 1/xi'_q = e'_q^+ g5 p(kappa P) e'_q, p(z) = sum_j
 * coeffs[j] z^j, coeffs_host complex128 [ncoeff]), accumulates
 *   xt[n] += g5 sum_q w_q e'_q (e'_q^+ eta[n])                (device LEX)
 *   trace_corr[th][t] += sum_q w_q sum_{x in t} e'_q(x)^+ Theta g5 e'_q(x)
 * (host complex128 [ntheta][Lt], Theta codes from thetas_host).  HFES is
 * xt = 0 plus this; HFPS / HFPOLY are PS / POLY output plus this.
 * xi_inv_host: optional host complex128 [Q] receiving 1/xi'_q.
 * Mode ES (Sec. 5.3, eigenvalue subtraction) takes the even/odd deflation
 * space instead (op SCHUR): with the Q eigenvalues lambda_q of M of
 * smallest |lambda| and biorthonormal right / left eigenvectors r_q, l_q
 * reconstructed from the Ritz pairs of Mhat (lambda = 1 - sqrt(1 -
 * lambda_hat); odd halves kappa / (1 - lambda) D_oe r_hat and
 * kappa / (1 - conj lambda) g5 D_oe g5 l_hat, l halved so that l^+ r = 1) it
 * accumulates xt[n] += sum_q r_q (l_q^+ eta[n]) / lambda_q and
 * trace_corr[th][t] += sum_q sum_{x in t} l_q(x)^+ Theta r_q(x) / lambda_q,
 * and xi_inv_host receives lambda_q.  EINVAL for a space of op MG5. */
lqcd_status deflate_project(lqcd_ctx *ctx, lqcd_defl *defl, int Q, lqcd_defl_mode mode,
                            const double *coeffs_host, int ncoeff, const int *thetas_host,
                            int ntheta, const void *eta, void *xt, int nrhs,
                            double *trace_corr_host, double *xi_inv_host);

/* Several hermitian-forced projections of the same noise at once (modes
 * HFES and EIGPOLY of deflate_project; Sec. 5.4 Eqs. (66)-(68), Sec. 5.5
 * Eqs. (69)-(72)): variant v is deflate_project with
 * mode modes[v], coefficients coeffs_list[v] (ncoeffs[v] complex128; read
 * for EIGPOLY only), xt = xt_list[v] and trace_corr_host = corr_list[v]
 * (corr_list NULL or an entry NULL: no correction), and its results equal
 * that call's bit for bit; the overlaps e'_q^+ eta[n] are formed once for
 * all variants.  EINVAL unless 1 <= nvar <= 4 and every mode is HFES or
 * EIGPOLY. */
lqcd_status deflate_project_multi(lqcd_ctx *ctx, lqcd_defl *defl, int Q, int nvar, const int *modes,
                                  const double *const *coeffs_list, const int *ncoeffs, const int *thetas_host,
                                  int ntheta, const void *eta, void *const *xt_list, int nrhs,
                                  double *const *corr_list);

/* Perturbative subtraction (Sec. 5.1, Eqs. (28)-(35)): xt[n] =
 * sum_{j=0}^{order} (kappa P)^j eta[n] (device LEX), and the exact trace
 * correction Tr_t(Theta sum_j (kappa P)^j) per timeslice (host complex128
 * [ntheta][Lt]; may be NULL), for any operator code.  Only closed paths
 * contribute to the correction (point-split: paths closed by the
 * operator's own hop, Sec. 5.1); order <= 7. */
lqcd_status pert_subtract(lqcd_ctx *ctx, int order, const int *thetas_host, int ntheta,
                          const void *eta, void *xt, int nrhs, double *trace_corr_host);

/* Polynomial subtraction (Sec. 5.2, Eqs. (40)-(50)).  If b is not NULL the
 * Min-Res coefficients for the noise vector b (device LEX, one field) are
 * computed first: minimise |b - M sum_{j=0}^{d} c_j (kappa P)^j b|
 * (the minimiser of the normal equations (v^+ v) a = v^+ b of Eq. (44),
 * written in the kappa P basis); coeffs_host (complex128 [degree+1]) is
 * written.  If b is NULL, coeffs_host is read instead.  Then
 * xt[n] = sum_j c_j (kappa P)^j eta[n] and the exact per-timeslice trace
 * correction Tr_t(Theta sum_j c_j (kappa P)^j).  a_host: optional
 * complex128 [degree+1] receiving the M-basis coefficients a_k of
 * Eq. (42).  degree <= 7. */
lqcd_status poly_subtract(lqcd_ctx *ctx, int degree, const void *b, double *coeffs_host,
                          double *a_host, const int *thetas_host, int ntheta,
                          const void *eta, void *xt, int nrhs, double *trace_corr_host);

/* Several polynomial subtraction vectors of the same noise at once (the
 * vectors of pert_subtract, whose coefficients are all 1, and of
 * poly_subtract; Sec. 5.1 Eq. (31), Sec. 5.2 Eq. (40)):
 *   xt_list[a][n] = sum_{j=0}^{degree} coeffs[a][j] (kappa P)^j eta[n],
 * with the powers (kappa P)^j eta formed once for all a and summed in order
 * of j (the single-polynomial calls use Horner's rule, so the vectors agree
 * with theirs to rounding).  coeffs_host: complex128 [npoly][degree+1] (a
 * polynomial of lower degree pads with zeros); eta: device LEX [nrhs];
 * xt_list: host array [npoly] of device LEX pointers [nrhs], written.  The
 * trace corrections are those of pert_subtract / poly_subtract (once per
 * configuration).  Workspace: degree+1 full FP64 fields per block of 16
 * right-hand sides.  EINVAL unless 1 <= npoly <= 4 and 0 <= degree <= 7. */
lqcd_status poly_subtract_multi(lqcd_ctx *ctx, int npoly, int degree, const double *coeffs_host,
                                const void *eta, void *const *xt_list, int nrhs);

/* Operator codes (thetas_host arrays): 0 = scalar (Theta = 1), 1..4 = local
 * vector g_1..g_4 (Table 2), 5..8 = point-split vector in direction mu =
 * 0..3 (Table 2): Theta(mu) psi(x) = kappa [ (1 + g_mu) U_mu(x - mu)^+
 * psi(x - mu) - (1 - g_mu) U_mu(x) psi(x + mu) ], with the context's kappa;
 * a term belongs to the timeslice of its row site x.  pert_subtract,
 * poly_subtract, deflate_project and loop_estimate accept all nine codes;
 * loop_gradient the local ones (0..4). */

/* The subtracted estimator (Sec. 5 Eq. (23); Sec. 6 Eq. (73)):
 *   t_n[th][t] = sum_{x in timeslice t} eta_n(x)^+ Theta (x_n - xt_n)(x),
 *   est[th][t] = (1/N) sum_n t_n[th][t] + trace_corr[th][t],
 * with entry t = Lt the whole-lattice sum.  eta, x: device LEX [nrhs];
 * xt: device LEX [nrhs] or NULL (no subtraction); trace_corr_host:
 * host complex128 [ntheta][Lt] or NULL.  Outputs (host): est complex128
 * [ntheta][Lt+1]; stderr_host double [ntheta][Lt+1][2] = standard errors
 * s / sqrt(N) of the real and imaginary parts (unbiased variance; 0 if
 * N = 1); samples_host optional complex128 [nrhs][ntheta][Lt+1].
 * The physical <psibar Theta psi> is -est (Eq. (73)). */
lqcd_status loop_estimate(lqcd_ctx *ctx, const int *thetas_host, int ntheta, const void *eta,
                          const void *x, const void *xt, int nrhs,
                          const double *trace_corr_host, double *est_host,
                          double *stderr_host, double *samples_host);

/* Several subtracted estimates of one set of solutions at once (Sec. 5
 * Eq. (23) for each of the subtraction methods of Secs. 5.1-5.5 on the same
 * noise): variant v is loop_estimate with xt = xt_list[v] and
 * trace_corr_host = corr_list[v], and its results equal that call's bit for
 * bit, while eta and x are read once for all variants.
 * xt_list: host array [nvar] of device LEX pointers [nrhs] (an entry NULL:
 * no subtraction); corr_list: host array [nvar] of host complex128
 * [ntheta][Lt] pointers (an entry NULL: no correction), or NULL for none.
 * Outputs (host): est complex128 [nvar][ntheta][Lt+1]; stderr_host double
 * [nvar][ntheta][Lt+1][2]; samples_host optional complex128
 * [nvar][nrhs][ntheta][Lt+1].  EINVAL unless 1 <= nvar <= 6. */
lqcd_status loop_estimate_multi(lqcd_ctx *ctx, const int *thetas_host, int ntheta, const void *eta,
                                const void *x, const void *const *xt_list, int nvar, int nrhs,
                                const double *const *corr_list, double *est_host, double *stderr_host,
                                double *samples_host);

/* Allocation-free form of loop_estimate, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, results and
 * errors, with the per-workgroup partial sums in a fixed device array of
 * 4 MiB per GPU, held by the library until the process ends, instead of a
 * context workspace that grows on first use.  It calls no hipMalloc or
 * hipFree.  EINVAL when nrhs * 10 * Lt * 2 partial sums exceed 2^19 (e.g.
 * nrhs > 819 at Lt = 32).  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other streams or host threads) race. */
lqcd_status loop_estimate_noalloc(lqcd_ctx *ctx, const int *thetas_host, int ntheta, const void *eta,
                                  const void *x, const void *xt, int nrhs, const double *trace_corr_host,
                                  double *est_host, double *stderr_host, double *samples_host);

/* Derivatives of the trace estimate (differentiation of Eq. (23) with
 * M = 1 - kappa P of Sec. 5.1 Eqs. (24)-(25); the adjoint uses the
 * g5-hermiticity of Sec. 5.4).  For the fixed-noise estimate
 *   T = (1/N) sum_n eta_n^+ Theta_w M^{-1} eta_n,
 *   Theta_w = sum_a w[a][t(x)] Theta_{thetas[a]}  (a site-diagonal weighting,
 *   t(x) the timeslice of x),
 * computes exactly (up to the solver tolerance)
 *   dkappa_host = dT/dkappa = (1/N) sum_n y_n^+ P x_n,
 *   dlinks[x][mu][a] = dT/dw^a for U_mu(x) -> exp(i w^a T^a) U_mu(x),
 *   T^a = lambda^a / 2 (Gell-Mann), = (kappa/N) sum_n y_n^+ (dP/dw^a) x_n,
 * with x_n = M^{-1} eta_n and y_n = g5 M^{-1} g5 Theta_w^+ eta_n.
 * thetas_host: int [ntheta] codes 0..4; weights_host: complex128
 * [ntheta][Lt] or NULL (all 1: the whole-lattice Tr(Theta M^{-1}) summed
 * over the codes).  eta: device LEX [nrhs]; x: device LEX [nrhs] solutions
 * of M x = eta, or NULL to solve for them in the same batched call.
 * The adjoint (and, if x is NULL, forward) systems are solved by
 * gmresdr_solve with op LQCD_OP_SCHUR, params, and *defl_inout as there
 * (NULL: the first right-hand side builds the deflation space and it is
 * returned).  dkappa_host: host complex128 [1]; dlinks: device complex128
 * LEX [V][4][8] or NULL (only the kappa derivative); stats: host [nrhs]
 * statistics of the adjoint solves, or NULL.  Its scratch (the stacked
 * right-hand sides and solutions) lives in context workspaces that grow
 * on first use and are kept.  ENOCONV as gmresdr_solve. */
lqcd_status loop_gradient(lqcd_ctx *ctx, const int *thetas_host, const double *weights_host,
                          int ntheta, const lqcd_solve_params *params, lqcd_defl **defl_inout,
                          const void *eta, const void *x, int nrhs, double *dkappa_host,
                          void *dlinks, lqcd_solve_stats *stats);

/* ------------------------------------------------------------------ batching
 * Several lattices solved together (one configuration per context; the
 * paper solves one configuration at a time).  All contexts must live on one
 * device and share one stream. */
typedef struct lqcd_batch lqcd_batch;
lqcd_status lqcd_batch_create(lqcd_ctx *const *ctxs, int nlat, lqcd_batch **out);
lqcd_status lqcd_batch_destroy(lqcd_batch *batch);
/* Workgroups of the persistent batched stencil launch (default 8192). */
lqcd_status lqcd_batch_set_grid(lqcd_batch *batch, int workgroups);
/* Form of the batched stencil: 0 (default) = one persistent launch over the
 * slot table (every slot reads its own links); 16, 32 or 64 = the
 * link-tiled stencil with tiles of that many sites, one launch per run of
 * consecutive slots that hold one lattice (its links staged once per tile
 * for all of them; the captured cycle is recorded again when a refill of
 * the slots changes these runs).  EINVAL for other values. */
lqcd_status lqcd_batch_set_tile(lqcd_batch *batch, int tile_sites);

/* Deflated GMRES-Proj solves (Sec. 7) of every lattice's right-hand sides
 * with FP32 inner solves in FP64 refinement (params->inner must be
 * LQCD_F32), all lattices in lockstep: right-hand sides are taken
 * params->rhs_block at a time from one queue over the lattices (uneven
 * counts and sizes mix in a block); each inner operator application is
 * one persistent launch over all of them or one link-tiled launch per
 * lattice among them (lqcd_batch_set_tile), the Gram-Schmidt and
 * projection kernels are batched over all of them, and with use_graph != 0
 * each GMRES(m - k) cycle (or proj_m) runs as a captured hipGraph.  b[l], x[l]: device
 * complex128 LEX [nrhs[l]][12 V_l]; defl[l]: deflation space of lattice l's
 * even/odd system (gmresdr_solve with LQCD_OP_SCHUR on that context).
 * stats: host array over all right-hand sides in lattice order, or NULL.
 * Stopping rule, tolerances and ENOCONV as gmresdr_solve. */
lqcd_status batch_solve(lqcd_batch *batch, const lqcd_solve_params *params, const void *const *b,
                        void *const *x, const int *nrhs, lqcd_defl *const *defl, int use_graph,
                        lqcd_solve_stats *stats);

/* Autotuner: times trial batch_solve runs (captured cycles) for rhs_block
 * in {4, 8, 16, 32} and the stencil forms of lqcd_batch_set_tile {0, 16,
 * 32, 64}, each on one block of right-hand sides drawn evenly from the
 * lattices, and returns the fastest pair (best_tile as for
 * lqcd_batch_set_tile).  rate_host: optional host double [16] receiving
 * the trial rates (right-hand sides per second, order: rhs_block major,
 * tile minor; 0 for skipped pairs).  The batch's tile setting is left
 * unchanged. */
lqcd_status batch_autotune(lqcd_batch *batch, const lqcd_solve_params *params, const void *const *b,
                           const int *nrhs, lqcd_defl *const *defl, int *best_rhs_block,
                           int *best_tile, double *rate_host);

/* The even/odd operator Mhat (Sec. 7) in FP32 on every right-hand side of
 * every lattice in one persistent launch per half hop: in[l], out[l] device
 * complex128 LEX [nrhs[l]][12 V_l] (even sites of out hold Mhat x_e, odd
 * sites zero), as wilson_apply with LQCD_OP_SCHUR and LQCD_F32. */
lqcd_status batch_wilson_apply(lqcd_batch *batch, const void *const *in, void *const *out,
                               const int *nrhs);

/* Kernel timing (measurement aid).  When enabled, the library brackets
 * every launch of the classes below with HIP events on the context stream
 * and accumulates, per class, the summed kernel duration, the number of
 * launches and the algorithmic bytes those launches must move (each
 * field, link or basis vector counted once per launch).  Enabling resets
 * the counters.  Reading synchronises the stream. */
typedef enum {
  LQCD_KC_HOP64 = 0,   /* stencil (Wilson hop + epilogue), FP64 */
  LQCD_KC_HOP32 = 1,   /* stencil, FP32 */
  LQCD_KC_DOT = 2,     /* Gram-Schmidt block dot products (first stage) */
  LQCD_KC_AXPY = 3,    /* Gram-Schmidt block updates (with norms) */
  LQCD_KC_GEMM = 4,    /* deflation projections V^+ X and V C, basis recombination */
  LQCD_KC_FORCE = 5,   /* link derivative of the trace (loop_gradient) */
  LQCD_KC_COUNT = 6
} lqcd_kernel_class;
lqcd_status lqcd_timer_enable(lqcd_ctx *ctx, int on);
lqcd_status lqcd_timer_read(lqcd_ctx *ctx, int kclass, double *ms, double *bytes,
                            int64_t *launches);

/* Launch-shape tuning.  LQCD_TUNE_HOP_NB64 / LQCD_TUNE_HOP_NB32: the
 * largest number of right-hand sides (1, 2, 4 or 8) that the stencil maps
 * onto adjacent lanes to share link loads, per precision (defaults 2 and
 * 1).  LQCD_TUNE_HOP_TILE64 / LQCD_TUNE_HOP_TILE32: 1 (default) lets
 * launches with at least 8 (FP64) or 4 (FP32) right-hand sides use the
 * link-tiled stencil (links staged in LDS per tile of sites and reused by
 * every right-hand side), 0 keeps the lane-grouped form.
 * LQCD_TUNE_HOP_ORDER: workgroup order of the lane-grouped form, 0
 * (default) = right-hand-side groups of a site block back to back, 1 =
 * site blocks of a right-hand side back to back.
 * LQCD_TUNE_HOP_TBLOCK64 / LQCD_TUNE_HOP_TBLOCK32: tile order of the
 * link-tiled stencil, 0 = tiles of consecutive sites in index order, n > 0
 * = tiles within one (z, t) plane, ordered by blocks of n timeslices, z
 * within a block, t fastest (up to 1024); -1 (default) = planes with
 * ceil(Lt / 8) timeslices per block when a plane (Lx / 2 * Ly sites) splits
 * into whole tiles and Lt >= 8, else index order.  LQCD_TUNE_HOP_TSITES32 /
 * LQCD_TUNE_HOP_TSITES64: sites per tile, FP32 16, 32 (default) or 64, FP64
 * 16 or 32 (default); a tile of T sites takes 256 / T right-hand sides per
 * pass, and launches with fewer use the next larger tile.  Smaller tiles
 * keep fewer sites in flight per XCD, so the neighbour planes' spinors stay
 * in its L2.  LQCD_TUNE_HOP_RGROUP: the
 * tiled stencil splits launches with more right-hand sides than this into
 * groups of this many, the group index slowest across the XCDs (each XCD's
 * L2 then holds one group's spinors; links are read once per group);
 * 0 = one group.  LQCD_TUNE_HOP_RNEST (plane order only): groups of this many
 * right-hand sides are swept in turn within each XCD's block of timeslices
 * (its L2 then holds one group's planes at a time; the block's links are
 * read once per group); 0 = off, -1 (default) = automatic: groups of 8 in
 * FP64, off in FP32; a nonzero group size takes precedence over
 * LQCD_TUNE_HOP_RGROUP.  LQCD_TUNE_GEMM_MFMA: 1 (default) runs the deflation
 * and eigenvector products V C whose columns share one basis (J <= 64
 * vectors, two or more columns) on the matrix cores; 0 uses the FMA
 * kernel.  LQCD_TUNE_CYCLE_REORTH: 0 (default) runs the second
 * Gram-Schmidt pass of the GMRES-Proj cycles only where the first pass
 * cancelled more than one digit (in the s-step form: where that test or
 * the conditioning of the block asks; the other blocks store their basis
 * vectors from the first update pass); 1 runs it on every step (a check
 * of that pass; slower).  LQCD_TUNE_KEPT_PERIOD: MINRES-DR tests its basis against
 * the kept vectors of the last restart on every this-many-th step of a cycle
 * and on its last step (1..64, default 16).  LQCD_TUNE_ARNOLDI_STEPS: 1 to
 * 6 (default 4) Arnoldi steps per pass over the basis in the GMRES-Proj
 * cycles with a 16-bit basis (s > 1: the s powers (Mhat - 1)^k v_j,
 * k = 1..s, are orthogonalised together, reading the basis once for all
 * of them; same Krylov space).  LQCD_TUNE_SSTEP_Z16: 0 (default) keeps
 * those powers in FP32; 1 stores them in the basis's 16-bit form when the
 * basis is FP16 (half the bytes for the stencil and the Gram-Schmidt passes
 * that read them; the Arnoldi relation then carries their rounding; a BF16
 * basis keeps them in FP32).  LQCD_TUNE_RECOMBINE_REGS: 1 (default) runs
 * the restart recombination V_{k+1} = V_{m+1} P with its outputs in
 * registers (up to 48 of them, P in LDS); 0 uses the LDS-tiled form.
 * Values are per context; EINVAL for other values. */
typedef enum {
  LQCD_TUNE_HOP_NB64 = 0,
  LQCD_TUNE_HOP_NB32 = 1,
  LQCD_TUNE_HOP_TILE64 = 2,
  LQCD_TUNE_HOP_TILE32 = 3,
  LQCD_TUNE_HOP_ORDER = 4,
  LQCD_TUNE_HOP_TBLOCK64 = 5,
  LQCD_TUNE_HOP_TBLOCK32 = 6,
  LQCD_TUNE_HOP_TSITES32 = 7,
  LQCD_TUNE_HOP_RGROUP = 8,
  LQCD_TUNE_HOP_TSITES64 = 9,
  LQCD_TUNE_GEMM_MFMA = 10,
  LQCD_TUNE_HOP_RNEST = 11,
  LQCD_TUNE_CYCLE_REORTH = 12,
  LQCD_TUNE_KEPT_PERIOD = 13,
  LQCD_TUNE_ARNOLDI_STEPS = 14,
  LQCD_TUNE_SSTEP_Z16 = 15,
  LQCD_TUNE_RECOMBINE_REGS = 16
} lqcd_tune_param;
lqcd_status lqcd_tune_set(lqcd_ctx *ctx, lqcd_tune_param param, int value);

/* Thread-local description of the last non-OK status. */
const char *lqcd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LQCD_H */
