/*
 * ces.h -- C interface of the MI355X (gfx950) implementation of the spectral
 * Kohn-Sham hot path: applying the discretised Hamiltonian H to a block of
 * orbitals in the spherical-Bessel x spherical-harmonic basis on a ball, and
 * Chebyshev-filtered subspace iteration around it.
 *
 * Method: A. S. Banerjee, R. S. Elliott, R. D. James, "A spectral scheme for
 * Kohn-Sham density functional theory of clusters" (J. Comput. Phys.).
 *
 * Conventions shared by every call
 * --------------------------------
 *  Basis.  F_lmn = R_ln(r) S_lm(theta, phi), 0 <= l < L (L = lmax + 1),
 *    -l <= m <= l, 0 <= n < N, with R_ln the Dirichlet spherical-Bessel radial
 *    functions of Section 2.2.1 (eq. spherical_bessel_1) and S_lm the REAL
 *    orthonormal harmonics
 *        S_lm     = sqrt2 c_lm P_l^m(cos theta) cos(m phi)   (m > 0)
 *        S_l0     =       c_l0 P_l(cos theta)
 *        S_{l,-m} = sqrt2 c_lm P_l^m(cos theta) sin(m phi)   (m > 0)
 *    without the Condon-Shortley phase (Section 2.2.1).  This basis is a
 *    unitary recombination of the paper's complex Y_l^m within each (l, n):
 *    s_m = (f_m + f_{-m})/sqrt2, s_{-m} = i (f_m - f_{-m})/sqrt2; eigenvalues,
 *    densities and residual norms are the same in both.
 *  Index.  Coefficient alpha = (l*l + l + m) * N + n (0-based form of the
 *    paper's indexing map, Section 2.2.3).  d = L*L*N.  A basis built with a
 *    kinetic-energy cutoff (ces_basis_create_ke) keeps N_l <= N radial
 *    functions for each l; then alpha = off_l + (l + m) * N_l + n with
 *    off_l = sum_{l' < l} (2l' + 1) N_l', and d = sum_l (2l + 1) N_l.
 *  Blocks.  Orbitals are columns; column-major; leading dimension ld >= d.
 *    All values crossing this interface are FP64.  A block has k >= 1
 *    columns and n_r * n_theta * ceil(k16 / 32) < 2^31, k16 = k rounded up to
 *    a multiple of 16 (the angular kernels' grid); otherwise, or with
 *    ld < d or a null block, the call returns CES_ERR_INVALID_ARG.
 *  Grid.  n_r radial nodes (ascending r) x n_theta Gauss-Legendre nodes in
 *    cos(theta) (ascending theta) x n_phi uniform phi_p = 2 pi p / n_phi
 *    (Section 2.2.2).  Grid arrays are C-order [r][theta][phi].
 *  Pointers.  d_* are device pointers, h_* host pointers.  The caller owns
 *    every buffer, the workspace and the stream; handles own their tables.
 *  Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  Calls are asynchronous on it unless stated otherwise.
 *  Workspace.  Calls that take (d_work, work_bytes) use only that device
 *    memory for scratch and allocate no device or host memory; query the size
 *    with ces_workspace_size.  The Hamiltonian's pinned host buffer for
 *    read-backs is allocated by ces_ham_create, sized for the largest block
 *    Rayleigh-Ritz accepts (k <= min(d, 32768)).  Calls that
 *    run concurrently on different streams need distinct workspaces.
 *  Threads.  Apart from ces_ham_set_veff, calls do not change what a basis
 *    or Hamiltonian handle represents, and calls on one handle may run from
 *    several host threads at once (each on its own stream, with its own
 *    workspace).  The handle's internal state (the one-time upload of the
 *    basis tables, the rocBLAS handle, its workspace-size cache and the
 *    pinned buffer for read-backs) is guarded by locks: Rayleigh-Ritz (also
 *    inside ces_chefsi and ces_scf) and ces_lanczos_bound on one handle run
 *    one at a time; H X, the filter and the density do not lock.
 *    ces_ham_set_veff must not overlap other calls on its handle, and calls
 *    on one ces_mlp handle must be serialised by the caller.
 *  Errors.  Every call returns a ces_status; arguments are validated on the
 *    host before any launch.  Device faults surface as CES_ERR_DEVICE at the
 *    next synchronising call.  ces_last_error() gives a thread-local detail.
 */
#ifndef CES_H
#define CES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CES_OK = 0,
  CES_ERR_INVALID_ARG = 1,
  CES_ERR_DEVICE = 2,
  CES_ERR_ALLOC = 3,
  CES_ERR_WORKSPACE = 4,
  CES_ERR_NOT_POSITIVE_DEFINITE = 5,
  CES_ERR_EIGENSOLVER = 6
} ces_status;

/* FP64: every stage in double.  MIXED: the transforms, kinetic term,
 * projector GEMMs and Chebyshev recurrence in FP32 with FP32 accumulation
 * (converted from/to FP64 once per call); orthonormalisation and
 * Rayleigh-Ritz stay FP64. */
typedef enum { CES_PREC_FP64 = 0, CES_PREC_MIXED = 1 } ces_precision;

/* Radial rule: Gauss-Jacobi nodes for the weight r^2 on [0,R] (the paper's
 * choice, Section 2.2.2) or Gauss-Legendre nodes with r^2 in the weights. */
typedef enum {
  CES_RADIAL_GAUSS_JACOBI_R2 = 0,
  CES_RADIAL_GAUSS_LEGENDRE = 1
} ces_radial_rule;

typedef struct ces_basis_s* ces_basis;
typedef struct ces_ham_s* ces_ham;

/* ------------------------------------------------------------------ basis */

/* Build the basis tables (Section 2.2.1-2.2.2): Bessel zeros b_ln by Halley
 * iteration, Lambda_ln = (b_ln/R)^2, radial and angular Gauss nodes and
 * weights by Golub-Welsch, R_ln(r_k), normalised P_l^m(t_j), and their FP32
 * copies, uploaded to the current device.  Synchronous.
 * lmax >= 0, n_rad >= 1, R > 0, n_r >= 1, n_theta >= 1, n_phi >= 2*lmax+1;
 * kernel tile limits: lmax <= 95, n_rad <= 192, n_r <= 256, n_phi <= 2048
 * (CES_ERR_INVALID_ARG beyond them). */
ces_status ces_basis_create(int lmax, int n_rad, double R, int n_r, int n_theta,
                            int n_phi, int radial_rule, ces_basis* out);
/* The non-uniform basis of the footnote in Section 2.2.1: the spherical
 * waves of the uniform basis above whose kinetic energy Lambda_ln / 2 =
 * b_ln^2 / (2 R^2) is at most e_cut (Hartree), i.e. N_l = #{n < n_rad :
 * Lambda_ln / 2 <= e_cut} radial functions for each l (n = 0 .. N_l - 1;
 * N_l does not grow with l), with the coefficient layout given under
 * "Index".  The grid, tables and limits are those of ces_basis_create; every
 * call works on either kind of basis.  e_cut must be finite and > 0 and keep
 * at least one l = 0 function (CES_ERR_INVALID_ARG). */
ces_status ces_basis_create_ke(int lmax, int n_rad, double R, int n_r, int n_theta, int n_phi,
                               int radial_rule, double e_cut, ces_basis* out);
/* h_nl[L] = N_l, the radial functions kept for each l (n_rad for a basis
 * without a cutoff). */
ces_status ces_basis_radial_counts(ces_basis b, int* h_nl);
ces_status ces_basis_destroy(ces_basis b);
/* d (L*L*N, or sum (2l+1) N_l with a cutoff) and n_grid = n_r*n_theta*n_phi. */
ces_status ces_basis_info(ces_basis b, int64_t* d, int64_t* n_grid);
/* Host copies of the grid: h_r[n_r], h_wr[n_r] (weights include r^2),
 * h_theta[n_theta], h_wtheta[n_theta] (Gauss weights in cos theta),
 * h_phi[n_phi].  Any pointer may be NULL. */
ces_status ces_basis_grid(ces_basis b, double* h_r, double* h_wr, double* h_theta,
                          double* h_wtheta, double* h_phi);
/* Host copies of the setup tables, for checking: h_zeros[L*N] = b_ln
 * (row l), h_radial[L*n_r*N] = R_ln(r_k) at [l][k][n], h_legendre
 * [n_theta*L*(L+1)/2] = c_lm P_l^m(t_j) at [j][l(l+1)/2 + m] (m >= 0, no
 * sqrt2 factor).  Any pointer may be NULL. */
ces_status ces_basis_tables(ces_basis b, double* h_zeros, double* h_radial,
                            double* h_legendre);

/* Coefficients in the paper's complex basis R_ln Y_l^m (Section 2.2.1,
 * without the Condon-Shortley phase; same index alpha) to the real basis of
 * this interface, and back.  For each (l, n) and mu = |m| > 0:
 *   complex -> real  s_{l,mu}  = (f_{l,mu} + f_{l,-mu}) / sqrt2
 *                    s_{l,-mu} = i (f_{l,mu} - f_{l,-mu}) / sqrt2
 *   real -> complex  f_{l,mu}  = (s_{l,mu} - i s_{l,-mu}) / sqrt2
 *                    f_{l,-mu} = (s_{l,mu} + i s_{l,-mu}) / sqrt2
 * and s_{l,0} = f_{l,0}; the map is unitary, so norms and inner products
 * carry over.  Both blocks are d x k column-major of interleaved complex
 * doubles (re, im), leading dimension >= d in complex entries, 16-byte
 * aligned, device memory, and must not overlap (CES_ERR_INVALID_ARG).  A
 * real function has f_{l,-mu} = conj(f_{l,mu}) and real s (zero imaginary
 * parts up to rounding).  Asynchronous on `stream`. */
ces_status ces_coeffs_complex_to_real(ces_basis b, int k, const double* d_f, int64_t ldf,
                                      double* d_s, int64_t lds, void* stream);
ces_status ces_coeffs_real_to_complex(ces_basis b, int k, const double* d_s, int64_t lds,
                                      double* d_f, int64_t ldf, void* stream);

/* ------------------------------------------------------------ hamiltonian */

/* H = 1/2 diag(Lambda) + B^T W diag(V_eff) B [+ P diag(h) P^T]
 * (Section 2.2.4, eq. matvec_final; Section 2.3.2 for the projector term).
 * d_veff: n_grid doubles, [r][theta][phi], copied.  d_proj: d x n_proj
 * column-major (ld = d) real-layout projector coefficients, or NULL with
 * n_proj = 0; copied in FP64 and FP32.  h_proj_energy: n_proj host doubles.
 * Synchronous on `stream`. */
ces_status ces_ham_create(ces_basis b, const double* d_veff, int n_proj,
                          const double* d_proj, const double* h_proj_energy,
                          void* stream, ces_ham* out);
/* Replace V_eff (same layout); asynchronous on `stream`. */
ces_status ces_ham_set_veff(ces_ham h, const double* d_veff, void* stream);

/* Model options of the handle's SCF calls (default 0, 0, 0): correlation = 1
 * adds the Perdew-Zunger LDA correlation potential (ces_pz_correlation) to
 * ces_ks_potential's V_eff, and so to ces_scf's; smearing_kT > 0 (Hartree)
 * makes ces_scf occupy all k states by Fermi-Dirac (ces_fermi_dirac, 2 n_occ
 * electrons) from each step's Ritz values instead of filling n_occ states;
 * mix_density = 1 makes ces_scf Anderson-mix the electron density (history
 * of rho_in, rho_out - rho_in; V_in = ks_potential(rho_in)) instead of the
 * potential (Section 3.4.1 allows either).  correlation or mix_density not
 * 0 or 1, or a negative or non-finite kT, is CES_ERR_INVALID_ARG.  Like
 * ces_ham_set_veff, must not overlap other calls on the handle. */
ces_status ces_ham_set_model(ces_ham h, int correlation, double smearing_kT, int mix_density);
ces_status ces_ham_destroy(ces_ham h);

/* Device bytes that any call below with k columns and precision `prec`
 * needs in d_work.  A CES_PREC_MIXED workspace holds the transform
 * intermediates of the FP32 product (about half the FP64 product's); FP64
 * products on it (ces_apply_H, ces_cheb_filter and ces_chefsi with
 * CES_PREC_FP64, Rayleigh-Ritz's H X, ces_to_grid, ces_from_grid) run in
 * column chunks of about k / 2, with the same results. */
ces_status ces_workspace_size(ces_ham h, int k, int prec, size_t* bytes);

/* Y = H X for a d x k block (eq. matvec_final): inverse radial sum
 * (eq. G_lmr), inverse Legendre sums, phi synthesis, V_eff, phi analysis,
 * Legendre quadrature (eq. Ar_lm), radial quadrature (eq. Arlm_to_coeff),
 * plus 1/2 Lambda X and the projector term.  X and Y must not overlap. */
ces_status ces_apply_H(ces_ham h, int k, const double* d_X, int64_t ldx, double* d_Y,
                       int64_t ldy, int prec, void* d_work, size_t work_bytes,
                       void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): Y = H X exactly as ces_apply_H
 * computes it, with no workspace argument.  Its scratch is a fixed device
 * array of CES_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 * from the first call on that GPU until the process ends; the call itself
 * allocates nothing.  A block whose product needs more scratch than that
 * returns CES_ERR_WORKSPACE before any launch (k = 32 on a basis of
 * L_max = 30, N = 60 with a 90 x 62 x 124 grid fits in both precisions).
 * Every call on one GPU uses the same array: calls that overlap in time on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller.  Arguments and errors as ces_apply_H; asynchronous on `stream`. */
#define CES_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ces_status ces_apply_H_noalloc(ces_ham h, int k, const double* d_X, int64_t ldx, double* d_Y,
                               int64_t ldy, int prec, void* stream);

/* X <- p_m(H) X in place, p_m(t) = T_m((t-c)/e) / T_m((a0-c)/e), e = (b-a)/2,
 * c = (b+a)/2 (the scaled Chebyshev filter of Section 3.2), by the three-term
 * recurrence with per-step scaling.  Requires degree >= 1, a < b, a0 < a. */
ces_status ces_cheb_filter(ces_ham h, int k, double* d_X, int64_t ldx, int degree,
                           double a, double b, double a0, int prec, void* d_work,
                           size_t work_bytes, void* stream);

/* Cholesky-QR with column scaling (Section 3.1.1, 3.2), then Rayleigh-Ritz
 * (Section 3.2), all FP64: Q = X D R^{-1}; theta, S = eig(Q^T H Q) ascending;
 * X <- Q S; HX <- (H Q) S; r_i = ||H x_i - theta_i x_i||.  d_HX (d x k, ld =
 * ldx) may be NULL.  d_eval[k], d_resnorm[k] device doubles; h_eval[k] (host,
 * may be NULL) receives a copy of the eigenvalues.  hx_prec selects
 * the precision of the H*Q product.  If factorising the scaled Gram matrix
 * D S D (unit diagonal) meets a pivot not above 2 k eps (a numerically
 * dependent column) or a non-positive one, X is left as it was and one
 * shifted Cholesky-QR pass followed by two plain passes (shifted
 * CholeskyQR3) orthonormalises it; CES_ERR_NOT_POSITIVE_DEFINITE if one of
 * these passes fails too (X then holds the output of the last pass that
 * succeeded).  *h_orth_path (host, may be NULL) receives which ran: 0 the
 * plain pass, 1 the shifted CholeskyQR3 fallback.  The k x k eigenproblem is
 * solved by a one-workgroup Jacobi method for k <= 60, by rocSOLVER syevd
 * above; CES_ERR_EIGENSOLVER if it does not converge.  1 <= k <= min(d,
 * 32768).  Synchronises `stream`. */
ces_status ces_rayleigh_ritz(ces_ham h, int k, double* d_X, int64_t ldx, double* d_HX,
                             double* d_eval, double* d_resnorm, double* h_eval,
                             int* h_orth_path, int hx_prec, void* d_work, size_t work_bytes,
                             void* stream);

/* Upper bound of the spectrum of H: `steps` Lanczos steps from the start
 * vector d_v0 (d doubles, not modified); bound = (largest Ritz value +
 * final residual norm) * 1.01 (1/1.01 if negative).  Synchronous. */
ces_status ces_lanczos_bound(ces_ham h, const double* d_v0, int steps, double* h_bound,
                             void* d_work, size_t work_bytes, void* stream);

/* Chebyshev-filtered subspace iteration from the block in d_X (Section 3.2,
 * started from random vectors): Rayleigh-Ritz; then repeat filter(prec, a =
 * theta_k, a0 = theta_1, b) + Rayleigh-Ritz (FP64 H*X) until, for i <
 * n_check, r_i <= res_tol*max(1,|theta_i|) and |delta theta_i| < dtheta_tol,
 * or max_iter; fixed_iter > 0 runs exactly that many iterations.  On return
 * d_X holds the Ritz vectors, d_eval/d_resnorm their values and residuals,
 * *h_iters the outer iterations.  Synchronous. */
ces_status ces_chefsi(ces_ham h, int k, double* d_X, int64_t ldx, int degree, double b,
                      int n_check, int max_iter, int fixed_iter, double res_tol,
                      double dtheta_tol, int prec, double* d_eval, double* d_resnorm,
                      int* h_iters, void* d_work, size_t work_bytes, void* stream);

/* Lowest eigenpairs of H by block LOBPCG (Section 3.1, following the
 * published method of Knyazev et al. that the paper adopts) from the block in
 * d_X: column-scaled Cholesky orthonormalisation of every search block;
 * soft locking (a column whose residual r_i = ||H x_i - theta_i x_i|| <=
 * res_tol * max(1, |theta_i|) leaves the residual and conjugate-direction
 * blocks; its Ritz vector still takes part in the Rayleigh-Ritz step); hard
 * locking against the n_lock orthonormal constraint columns d_Y (d x n_lock,
 * ld ldy; may be NULL with n_lock = 0): the start block and every residual
 * block are projected against them; on a failed factorisation of the
 * conjugate directions or of the projected pencil the iteration goes on
 * without them, and on a failed factorisation of the residual block it
 * restarts from the current Ritz vectors.  With precondition = 1 each
 * residual y is multiplied coefficient-wise by the Teter-Payne-Allan factor
 * (Section 3.1.2) T(g) = (27 + 18g + 12g^2 + 8g^3) / (27 + 18g + 12g^2 + 8g^3
 * + 16g^4), g = g_scale * Lambda_alpha / KE(y), KE(y) = (1/2) sum Lambda |y|^2
 * / sum |y|^2 (g_scale = 1 is the printed formula read per unit norm of y;
 * 0.5 is Teter, Payne and Allan's own variable).  H W runs in `prec`; the
 * Gram products, factorisations and updates in FP64.  Stops when the first
 * n_check columns have converged or after max_iter iterations.  On return
 * d_X holds the Ritz vectors after a final FP64 Rayleigh-Ritz, d_eval /
 * d_resnorm (k device doubles) their values and residual norms, *h_iters the
 * iterations, *h_restarts (may be NULL) the restarts.  Requires 3k + n_lock
 * <= d, k <= 32768, 1 <= n_check <= k, res_tol > 0, g_scale > 0.
 * Workspace: ces_lobpcg_workspace_size.  Synchronous. */
ces_status ces_lobpcg_workspace_size(ces_ham h, int k, int n_lock, int prec, size_t* bytes);
ces_status ces_lobpcg(ces_ham h, int k, double* d_X, int64_t ldx, int n_lock, const double* d_Y,
                      int64_t ldy, int n_check, int max_iter, double res_tol, double g_scale,
                      int precondition, int prec, double* d_eval, double* d_resnorm, int* h_iters,
                      int* h_restarts, void* d_work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------- density */

/* rho(x_g) = 2 sum_i f_i psi_i(x_g)^2 with psi_i the inverse transform of
 * column i (Section 2.2.5); d_occ[k] device doubles f_i; d_rho_grid[n_grid]
 * ([r][theta][phi]); d_rho_coef[d] (may be NULL) = forward transform of rho
 * (same basis, the dualing choice of Section 2.2.5).  prec CES_PREC_FP64, or
 * CES_PREC_MIXED: psi formed in FP32, its squares weighted and summed over
 * the orbitals in FP64; rho and its coefficients are FP64 either way.
 * Workspace: ces_workspace_size(h, k, prec). */
ces_status ces_density(ces_ham h, int k, const double* d_X, int64_t ldx,
                       const double* d_occ, double* d_rho_grid, double* d_rho_coef,
                       int prec, void* d_work, size_t work_bytes, void* stream);

/* Inverse transform of k columns to the grid: d_f[n_grid * k], column i at
 * offset i*n_grid, each [r][theta][phi] (Section 2.2.2, eq. G_lmr). */
ces_status ces_to_grid(ces_ham h, int k, const double* d_X, int64_t ldx, double* d_f,
                       void* d_work, size_t work_bytes, void* stream);
/* Forward transform of k grid functions (eqs. Ar_lm, Arlm_to_coeff). */
ces_status ces_from_grid(ces_ham h, int k, const double* d_f, double* d_X, int64_t ldx,
                         void* d_work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------ SCF extras */
/* The self-consistent cluster model: V_eff = V_ext + V_H[rho - rho_ion] +
 * V_x[rho] (Section 2.1 with LDA exchange only), rho_ion a caller-given
 * positive background (e.g. Gaussian ion charges) that makes the cluster
 * neutral.  Grid arrays are n_grid FP64 values [r][theta][phi].  Calls that
 * take (d_work, work_bytes) need at least ces_workspace_size(h, 1, FP64)
 * bytes unless stated otherwise. */

/* Hartree potential of the density sum_lmn tau_lmn F_lmn (Section 2.3.1,
 * eqs. Laplace_expansion, hartree_calc1, zeta_definition):
 *   V_H(x) = sum_lmn tau_lmn (4 pi / (2l+1)) zeta_ln(r) S_lm(x/|x|),
 * with the radial integral zeta_ln in closed form: the free-space potential
 * (decaying as Q/r outside the ball), not a Dirichlet solve.  d_tau[d]
 * coefficients in the real layout; d_vh[n_grid] output. */
ces_status ces_hartree(ces_ham h, const double* d_tau, double* d_vh, void* d_work,
                       size_t work_bytes, void* stream);

/* Perdew-Zunger (1981) LDA correlation of the unpolarised electron gas (the
 * parametrisation Section 2.1 adopts), elementwise over n grid values, with
 * r_s = (3 / (4 pi rho))^(1/3):
 *   r_s >= 1: eps_c = -0.1423 / (1 + 1.0529 sqrt(r_s) + 0.3334 r_s)
 *   r_s < 1:  eps_c = 0.0311 ln r_s - 0.048 + 0.0020 r_s ln r_s - 0.0116 r_s
 * d_vc = v_c = d(rho eps_c)/d rho; d_ec (may be NULL) = eps_c, the energy
 * per electron.  rho <= 0 gives 0 for both.  d_vc may equal d_rho; d_ec must
 * alias neither (CES_ERR_INVALID_ARG).  n = 0 does nothing.  Asynchronous. */
ces_status ces_pz_correlation(int64_t n, const double* d_rho, double* d_vc, double* d_ec,
                              void* stream);

/* Fermi-Dirac occupations (Section 3.4.1, eq. Fermi_constraint), on the
 * host: h_occ[i] = 1 / (1 + exp((h_eval[i] - eF) / kT)) for the k given
 * eigenvalues (any order), with the Fermi level eF such that
 * sum_i h_occ[i] = n_electrons / 2 (spin-unpolarised, every orbital doubly
 * occupied), found by Brent's method to about machine precision in eF.  The
 * sum runs over all k states.  kT (Hartree) > 0 and 0 < n_electrons / 2 < k,
 * finite eigenvalues, else CES_ERR_INVALID_ARG.  h_occ feeds ces_density's
 * d_occ.  Host pointers; no device work. */
ces_status ces_fermi_dirac(int k, const double* h_eval, double n_electrons, double kT,
                           double* h_occ, double* h_eF);

/* Slater (LDA) exchange potential, elementwise over n grid values:
 * d_vx = -(3 rho_+ / pi)^(1/3), rho_+ = max(d_rho, 0) (Section 2.1's V_x in
 * its exchange-only local form).  d_vx may equal d_rho.  n = 0 does nothing;
 * n < 0 or a null pointer is CES_ERR_INVALID_ARG.  Asynchronous. */
ces_status ces_slater_x(int64_t n, const double* d_rho, double* d_vx, void* stream);

/* Eigensolver of the handle's ces_scf: mode 0 (default) Chebyshev-filtered
 * subspace iteration in every step, started with Rayleigh-Ritz and
 * first_iters filters; mode 1 LOBPCG (ces_lobpcg with the preconditioner,
 * all k states to res_tol, at most max_iter iterations) in the first SCF
 * step and the filter afterwards (the paper's strategy for large systems,
 * Section 3.2); mode 2 LOBPCG in every step (its strategy for small ones,
 * Section 3.1).  Workspace sizes queried afterwards include LOBPCG's.  Like
 * ces_ham_set_veff, must not overlap other calls on the handle. */
ces_status ces_ham_set_scf_eigensolver(ces_ham h, int mode, double res_tol, int max_iter);

/* Non-dualing density (Section 2.2.5): the density of orbitals with
 * l <= lmax holds angular degrees up to 2 lmax, so the paper lets it be
 * expanded in a larger basis than the orbitals.  After this call the
 * handle's ces_ks_potential (and so ces_scf) expands rho - rho_ion in the
 * basis `rho_basis` for the Hartree potential; NULL restores the orbitals'
 * own basis (the dualing choice).  rho_basis must use the orbitals' grid
 * (same R, n_r, n_theta, n_phi and radial rule) and lmax_rho >= lmax;
 * lmax_rho = 2 lmax holds the density exactly in angle, and the grid
 * integrates the density against it exactly in angle when 2 n_theta - 1 >=
 * 2 lmax + lmax_rho and n_phi > 2 lmax + lmax_rho (with lmax_rho = 2 lmax:
 * n_theta >= 2 lmax + 1, n_phi >= 4 lmax + 1; the n_theta = 2L, n_phi = 4L
 * grids qualify).  The handle borrows rho_basis: keep it alive while set.
 * Workspace sizes queried afterwards include the density basis; like
 * ces_ham_set_veff, must not overlap other calls on the handle. */
ces_status ces_ham_set_density_basis(ces_ham h, ces_basis rho_basis);

/* d_v = V_ext + V_H[rho - rho_ion] + V_x[rho], V_x = -(3 rho_+ / pi)^(1/3),
 * rho_+ = max(rho, 0).  V_H uses the forward transform of rho - rho_ion in
 * the orbital basis (the dualing choice, Section 2.2.5), or in the density
 * basis set by ces_ham_set_density_basis, and the Hartree closed form of
 * ces_hartree on that basis.  d_tau (may be NULL) receives those
 * coefficients: d doubles of that basis.  d_v must not alias an input
 * (CES_ERR_INVALID_ARG). */
ces_status ces_ks_potential(ces_ham h, const double* d_rho, const double* d_rho_ion,
                            const double* d_vext, double* d_v, double* d_tau, void* d_work,
                            size_t work_bytes, void* stream);

/* Anderson mixing of potentials (Section 3.4.1).  d_V, d_F: n x m history
 * (column-major, leading dimension ld >= n, 1 <= m <= 64) of input
 * potentials V_i and residuals F_i = V_out(V_i) - V_i; column `oldest` is the
 * oldest pair and ages increase cyclically from it.  Writes
 *   d_out = sum_i c_i (V_i + beta F_i),
 * c minimising ||sum_i c_i F_i||_2 subject to sum_i c_i = 1 (the same V and F
 * averages as the difference form of the method; one pair gives V + beta F).
 * If that system is numerically singular the oldest pairs are left out
 * (c_i = 0) until it is not.  h_coef[m] (may be NULL) receives c.
 * Workspace: ces_anderson_workspace_size(n, m).  Each output element is
 * written after its history row is read, so d_out may alias a V column.
 * Synchronous. */
ces_status ces_anderson_workspace_size(int64_t n, int m, size_t* bytes);
ces_status ces_anderson_mix(int64_t n, int m, const double* d_V, const double* d_F, int64_t ld,
                            int oldest, double beta, double* d_out, double* h_coef,
                            void* d_work, size_t work_bytes, void* stream);

/* Superposition of atomic densities (Section 3.2): d_rho(x_g) = sum_a
 * rho_at(|x_g - a|), with the spherical atomic density
 *   rho_at(r) = S_00 sum_n tau00[n] R_0n(r)  (r < R; 0 for r >= R),
 * tau00[N_0] the l = 0 coefficients (alpha = n) of one atom's density in this
 * basis (from ces_ks_potential's d_tau or ces_density of a one-atom SCF).
 * h_atoms[3 n_atoms] host xyz (bohr); tau00 holds N_0 values (n_rad for a
 * basis without a cutoff).  Synchronous. */
ces_status ces_sad_density(ces_ham h, int n_atoms, const double* h_atoms,
                           const double* h_tau00, double* d_rho, void* d_work,
                           size_t work_bytes, void* stream);

/* Self-consistent field loop on the handle's basis (Sections 3.2, 3.4.1);
 * the handle's V_eff is overwritten.  The n_occ lowest orbitals are doubly
 * occupied (f_i = 1 in ces_density); the other k - n_occ are guard states.
 *   V_in = ks_potential(d_rho0); then per step:
 *   V_eff = V_in; b = ces_lanczos_bound(d_v0, 20 steps);
 *   step 1: Rayleigh-Ritz of d_X, then first_iters x (filter + RR);
 *   later steps: one filter (degree, prec; a = theta_k, a0 = theta_1) + RR
 *   (Rayleigh-Ritz always with FP64 H*X); or LOBPCG in the first or in
 *   every step (ces_ham_set_scf_eigensolver);
 *   rho = density of d_X; V_out = ks_potential(rho);
 *   stop when max_{i < n_occ} |theta_i - theta_i(previous step)| < tol;
 *   else V_in = ces_anderson_mix over the last `hist` pairs (V_in, V_out - V_in).
 * Outputs: d_X (Ritz vectors), d_eval[k], d_rho[n_grid] (last density),
 * *h_steps (steps taken, <= max_steps), h_dtheta[max_steps] (may be NULL:
 * per-step max change, +inf at step 1).  The caller checks convergence from
 * h_dtheta.  Workspace: ces_scf_workspace_size (includes 2 hist grid arrays
 * of history).  Synchronous. */
ces_status ces_scf_workspace_size(ces_ham h, int k, int prec, int hist, size_t* bytes);
ces_status ces_scf(ces_ham h, int k, double* d_X, int64_t ldx, int n_occ, const double* d_vext,
                   const double* d_rho_ion, const double* d_rho0, const double* d_v0, int degree,
                   double beta, int hist, double tol, int max_steps, int first_iters, int prec,
                   double* d_eval, double* d_rho, int* h_steps, double* h_dtheta, void* d_work,
                   size_t work_bytes, void* stream);

/* ------------------------------------------------------ learned start */
/* Not part of the paper's method: a learned correction to the SAD start
 * density, so that the SCF (ces_scf) needs fewer steps; the converged
 * eigenvalues do not depend on the start.  The start density is
 *   rho_0(x) = rho_SAD(x) + sum_j sum_q c_jq Phi_q(x - a_j; u_j),
 * c_j = network(descriptors of atom j), with the CES_MLP_CHANNELS functions
 *   q < 5:  (2 pi s^2)^(-3/2) exp(-r^2 / (2 s^2)),        s = 0.6 0.9 1.3 1.9 2.8
 *   q >= 5: (2 pi s^2)^(-3/2) (d.u_j / s) exp(-r^2/(2s^2)), s = 0.9 1.4 2.2
 * (d = x - a_j, r = |d|, u_j the atom's unit environment direction), so
 * rho_0 rotates with the cluster and does not depend on the atom order. */
#define CES_MLP_FEATURES 24
#define CES_MLP_CHANNELS 8

/* Per-atom descriptors (host only, no device work).  h_atoms[3n] xyz
 * (bohr); h_desc[n * 24] (row per atom): 16 radial symmetry functions
 * sum_i exp(-2 (r_ij - mu)^2) fc(r_ij), mu = 2.0, 2.5, ..., 9.5; 4 angular
 * ones 2^(1-z) sum_{i<k} (1 + l cos theta_ijk)^z exp(-0.02 (r_ij^2 + r_ik^2))
 * fc fc for (z, l) = (1, 1), (1, -1), (4, 1), (4, -1); |a_j| / 8; n / 40;
 * sum_i exp(-r_ij^2 / 18) / 10; |u_j|.  fc(r) = (cos(pi r / 10) + 1) / 2
 * below 10 bohr, else 0.  u_j = sum_i exp(-r_ij^2 / 18) (a_i - a_j) / r_ij;
 * h_dirs[3n] = u_j / |u_j| (zero when |u_j| <= 1e-6). */
ces_status ces_atom_descriptors(int n_atoms, const double* h_atoms, float* h_desc,
                                double* h_dirs);

/* Gram matrix of the correction functions and a target on the grid:
 * column c < 8 n of F holds sqrt(W_g) Phi_c(x_g) (c = 8 j + q), the last
 * column sqrt(W_g) target(x_g) (zero if d_target is NULL); d_gram
 * ((8n+1)^2, FP64) = F^T F.  Its leading block is M, its last column p,
 * its corner t, so ||sum c Phi - target||_W^2 = c.M c - 2 p.c + t.
 * Workspace: ces_density_fit_workspace_size.  Synchronous. */
ces_status ces_density_fit_workspace_size(ces_ham h, int n_atoms, size_t* bytes);
ces_status ces_density_fit_gram(ces_ham h, int n_atoms, const double* h_atoms,
                                const double* h_dirs, const double* d_target, double* d_gram,
                                void* d_work, size_t work_bytes, void* stream);

/* d_rho[g] += sum_{j,q} d_coef[8 j + q] Phi_q(x_g - a_j; u_j) (d_coef FP32).
 * d_work: at least 48 n_atoms bytes.  Synchronous. */
ces_status ces_density_correction(ces_ham h, int n_atoms, const double* h_atoms,
                                  const double* h_dirs, const float* d_coef, double* d_rho,
                                  void* d_work, size_t work_bytes, void* stream);

/* Per-atom network: n_in -> depth hidden layers of `width` (SiLU) -> n_out
 * (linear), FP32 on the device, inputs standardised by a stored mean and
 * std.  Weights start N(0, 1/fan_in) from a splitmix64 stream seeded by
 * `seed`, biases 0, mean 0, std 1.  Parameter order (get/set): for each
 * layer W (n_in_l x n_out_l, row-major) then b.  The handle owns its device
 * memory (parameters, gradients, Adam moments). */
typedef struct ces_mlp_s* ces_mlp;
ces_status ces_mlp_create(int n_in, int width, int depth, int n_out, uint64_t seed, ces_mlp* out);
ces_status ces_mlp_destroy(ces_mlp m);
ces_status ces_mlp_num_params(ces_mlp m, int64_t* n);
/* Host copies; any pointer may be NULL (not copied).  Synchronous. */
ces_status ces_mlp_get_params(ces_mlp m, float* h_params, float* h_mean, float* h_std);
ces_status ces_mlp_set_params(ces_mlp m, const float* h_params, const float* h_mean,
                              const float* h_std);
ces_status ces_mlp_get_grads(ces_mlp m, float* h_grads);
/* Workspace for `rows` input rows: the activations that backward reuses. */
ces_status ces_mlp_workspace_size(ces_mlp m, int rows, size_t* bytes);
/* d_out[rows x n_out] = network(d_in[rows x n_in]) (row-major). */
ces_status ces_mlp_forward(ces_mlp m, int rows, const float* d_in, float* d_out, void* d_work,
                           size_t work_bytes, void* stream);
/* Gradients of sum(d_gout * out) for the last forward on the same
 * workspace, written (not accumulated) into the handle. */
ces_status ces_mlp_backward(ces_mlp m, int rows, const float* d_gout, void* d_work,
                            size_t work_bytes, void* stream);
/* Adam (Kingma and Ba) with bias correction for step >= 1. */
ces_status ces_mlp_adam_step(ces_mlp m, float lr, float beta1, float beta2, float eps, int step,
                             void* stream);

/* Batched quadratic loss of n_clusters clusters.  Cluster c owns network
 * output rows [d_row_off[c], d_row_off[c+1]) (n_c atoms, at most max_atoms
 * <= 2048), M_c (8 n_c x 8 n_c, symmetric, FP32) at d_M + d_m_off[c],
 * p_c (8 n_c) at d_p + 8 d_row_off[c] and t_c = d_t[c].  With c the
 * cluster's outputs flattened row-major:
 *   d_loss[c] = c.M c - 2 p.c + t,  d_gout (rows) = scale (2 M c - 2 p).
 * A cluster with more than max_atoms atoms gets loss NaN and no gradient. */
ces_status ces_cluster_quad_loss(int n_clusters, int max_atoms, const int64_t* d_row_off,
                                 const int64_t* d_m_off, const float* d_M, const float* d_p,
                                 const float* d_t, const float* d_out, float* d_gout,
                                 float* d_loss, float scale, void* stream);

/* -------------------------------------------------------------- profiling */

/* Stage timing with HIP events recorded around each launch of the H*X
 * kernels on the caller's stream.  Stage ids: 0 radial inverse (eq. G_lmr),
 * 1 Legendre synthesis, 2 phi stage with V_eff, 3 Legendre quadrature
 * (eq. Ar_lm), 4 radial quadrature with the kinetic / projector / Chebyshev
 * epilogue (eq. Arlm_to_coeff), 5 projector product C = diag(h) P^T Y,
 * 6 projector product P C; ids 7..13 are the same stages in FP64 (0..6 are
 * FP32).  ces_profile_enable(1, n) starts
 * recording into a pool of n event pairs (launches beyond the pool are not
 * recorded) and clears the totals; ces_profile_enable(0, 0) stops and frees
 * the pool.  Process-wide, not thread-safe; meant for benchmarking. */
ces_status ces_profile_enable(int on, int max_records);
/* Synchronise the recorded events and return, per stage s < n_stages (<= 14),
 * the summed milliseconds h_ms[s] and launch count h_count[s]. */
ces_status ces_profile_read(int n_stages, double* h_ms, int64_t* h_count);

/* ----------------------------------------------------------------- misc */
const char* ces_status_string(ces_status s);
const char* ces_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CES_H */
