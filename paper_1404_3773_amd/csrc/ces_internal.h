// Internal declarations of libces: handle structs, device table layouts and
// kernel launchers.  Device layouts (all row-major, innermost index last):
//   X blocks   [i][alpha]            column-major d x k, ld >= d
//   G, A       [r][lm][i]            per radial node and (l,m), i padded to kp
//   RiT        [l][N4][R16]          R_ln(r_k) at [l][n][r]
//   RfT        [l][R4][N16]          w_k R_ln(r_k) at [l][r][n]
//   Pm, PwT, RiT, RfT                zero-padded MFMA operand tables (shapes
//                                    in kernels_angular.hip / kernels_radial.hip)
//   ab         [r][j][2][S]          halved phi-Fourier cosine / sine sums of
//                                    V_eff at each (r, theta_j), S = 2L - 1
//   V          [r][j][p]
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ces.h"

typedef struct _rocblas_handle* rocblas_handle;

namespace ces {

constexpr int kColPad = 16;  // internal column padding of G/A and mixed blocks

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

template <typename T>
struct DevTables {
  T* RiT = nullptr;
  T* RfT = nullptr;
  T* lamh = nullptr;   // [l][n] Lambda_ln / 2
  T* wt = nullptr;     // [n_theta]
  T* Pm = nullptr;     // [m][L+4][J64]  c_lm P_l^m(t_j) (* sqrt2, m > 0); 0 for l < m
  T* PwT = nullptr;    // [m][J4][L16]   w_j * Pm[m][m + ll][j] at [m][j][ll]
};

struct Basis {
  int L = 0, N = 0, n_r = 0, n_theta = 0, n_phi = 0, rule = 0;
  double R = 0;
  int64_t d = 0, n_grid = 0;
  // Coefficient layout: N_l radial functions kept for each l (N for the
  // uniform basis; fewer under a kinetic-energy cutoff) and the first index
  // off_l of each l, so alpha(l, m, n) = off_l + (l + m) N_l + n.
  std::vector<int> Nl;
  std::vector<int64_t> off;
  double e_cut = 0.0;            // the cutoff (0: uniform basis)
  int* dev_lay = nullptr;        // [L][2] off_l, N_l (device)
  double* dev_lam = nullptr;     // [d] Lambda of each coefficient (device)
  std::vector<double> zeros, r, wr, theta, t, wt, phi;
  std::vector<double> radial;    // [l][k][n]
  std::vector<double> legendre;  // [j][l(l+1)/2 + m]
  int device = -1;
  double* dev_cs = nullptr;      // [2][n_phi] cos, sin(2 pi u / n_phi)
  double* dev_rnode = nullptr;   // [n_r] radial nodes
  double* dev_wr = nullptr;      // [n_r] radial weights (r^2 included)
  double* dev_cth = nullptr;     // [n_theta] cos(theta_j)
  double* dev_sth = nullptr;     // [n_theta] sin(theta_j)
  double* dev_hart = nullptr;    // [l][N4][R16] (4 pi / (2l+1)) zeta_ln(r_k), RiT layout
  DevTables<double> t64;
  DevTables<float> t32;
  void* dev_block = nullptr;     // single allocation holding all device tables
  std::mutex dev_mu;             // held while the device tables are uploaded
};

struct Ham {
  Basis* basis = nullptr;
  double* veff = nullptr;   // [n_grid]
  double* ab64 = nullptr;   // [n_r*n_theta*2*S]
  float* ab32 = nullptr;
  int n_proj = 0;
  double* proj64 = nullptr; // d x n_proj
  float* proj32 = nullptr;
  double* hproj64 = nullptr;
  float* hproj32 = nullptr;
  rocblas_handle blas = nullptr;
  int xc_correlation = 0;    // ces_ks_potential adds the Perdew-Zunger v_c
  double smear_kT = 0.0;     // ces_scf: Fermi-Dirac occupations at kT when > 0
  int mix_density = 0;       // ces_scf: Anderson-mix rho instead of V_eff
  Basis* rho_basis = nullptr;  // density basis on the same grid (non-dualing), or null
  int scf_solver = 0;         // ces_scf eigensolver: 0 CheFSI, 1 LOBPCG first step, 2 LOBPCG
  double lobpcg_tol = 1e-6;   // LOBPCG residual tolerance inside ces_scf
  int lobpcg_max_iter = 200;
  size_t solver_ws = 0;     // device bytes rocSOLVER needs for k = kmax_query
  int solver_ws_k = 0;
  void* dev_block = nullptr;
  double* host_stage = nullptr;   // pinned host buffer for results read back by a call
  size_t host_stage_n = 0;        // its length in doubles
  // Held by every call that uses the rocBLAS handle, the solver-size cache or
  // host_stage (workspace layout queries, Rayleigh-Ritz, the Lanczos bound),
  // so concurrent calls on one handle from several threads stay correct; the
  // H X, filter and density paths touch none of these and run unlocked.
  std::mutex mu;
};

// Pinned host staging of at least n doubles on h (grown as needed), so that a
// call's read-backs are DMA copies behind one synchronisation.
ces_status host_stage(Ham& h, size_t n);
// Copies `bytes` from device `src` into the stage at double offset `off`
// (asynchronous on s; read after synchronising s).
ces_status stage_read(Ham& h, size_t off, const void* src, size_t bytes, hipStream_t s);

// ------------------------------------------- shared by the C interface files

ces_status fail(ces_status s, const std::string& msg);   // sets the thread's last error

#define CES_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::ces::fail(CES_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CES_TRY(expr)                 \
  do {                                \
    ces_status s_ = (expr);           \
    if (s_ != CES_OK) return s_;      \
  } while (0)

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Byte offsets of the regions of a caller workspace for k columns.
struct Layout {
  size_t G = 0, A = 0, gbuf = 0, B1 = 0, B2 = 0, V3 = 0, F0 = 0, F1 = 0, C = 0, Cpart = 0,
         Zkb = 0, S1 = 0, S2 = 0, vec = 0, part = 0, info = 0, solver = 0, total = 0;
  size_t solver_bytes = 0;
  int64_t kp = 0;
  // columns of an FP64 product that G, A and gbuf hold: kp in an FP64
  // workspace; in a mixed one (regions sized for the FP32 product) about
  // half, and FP64 products run in column chunks of that size
  int64_t kc64 = 0;
};
Layout layout_for(Ham& h, int k, int prec);
ces_status check_work(Ham& h, int k, int prec, void* work, size_t bytes, Layout& ly);
ces_status check_block(const Ham& h, int k, const void* X, int64_t ldx, const char* what);
// The regions one H*X uses (G, A, gbuf, F0/F1 in mixed precision, projector
// products), sized for the precision the product runs in.
Layout hx_layout(const Ham& h, int k, int prec);
// out = alpha (H Yin - c Yin) + beta Yold on the regions of ly in work.
template <typename T>
ces_status h_step(Ham& h, const Layout& ly, void* work, int k, const T* Yin, int64_t ldin,
                  const T* Yold, int64_t ldold, T* out, int64_t ldout, T alpha, T c, T beta,
                  hipStream_t s);
// Y = H X (FP64, or the mixed-precision conversions around an FP32 product).
ces_status apply_H_impl(Ham& h, const Layout& ly, void* work, int k, const double* X,
                        int64_t ldx, double* Y, int64_t ldy, int prec, hipStream_t s);

// Cholesky-QR + Rayleigh-Ritz on the block (see ces_rayleigh_ritz); h_eval /
// h_res (host, may be null) receive the eigenvalues / residual norms, *h_path
// (may be null) 0 for the plain pass, 1 for the shifted CholeskyQR3 fallback.
ces_status rr_impl(Ham& h, const Layout& ly, void* work, int k, double* X, int64_t ldx,
                   double* HX, int64_t ldhx, double* eval, double* res, int hx_prec,
                   hipStream_t s, double* h_eval, double* h_res, int* h_path);
// rr_impl for a caller that already holds h.mu.
ces_status rr_locked(Ham& h, const Layout& ly, void* work, int k, double* X, int64_t ldx,
                     double* HX, int64_t ldhx, double* eval, double* res, int hx_prec,
                     hipStream_t s, double* h_eval, double* h_res, int* h_path);
// Workspace bytes of ces_lobpcg for k columns (takes h.mu).
size_t lobpcg_workspace_bytes(Ham& h, int k, int n_lock, int prec);
// Device bytes rocSOLVER needs for potrf/trtri/syevd of order k (cached per
// handle; takes h.mu).
size_t solver_bytes_for(Ham& h, int k);

template <typename T>
struct Ptr {
  static T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }
};

// ---------------------------------------------------------------- launchers
// All launchers are asynchronous on `s` and assume validated arguments.

template <typename T>
void launch_radial_inverse(const Basis& b, const DevTables<T>& tb, const T* X, int64_t ldx,
                           T* G, int k, int kp, hipStream_t s);

// out = alpha * (Z + lamh o Yin + KB - c * Yin) + beta * Yold, with
// Z = Rfwd^T A (per lm) (+ Zkb, the projector term: column-major d x k, ld d,
// or null).  Yold may be null when beta == 0.
template <typename T>
void launch_radial_forward(const Basis& b, const DevTables<T>& tb, const T* A, const T* Yin,
                           int64_t ldin, const T* Yold, int64_t ldold, T* out, int64_t ldout,
                           T alpha, T cshift, T beta, bool kinetic, const T* Zkb, int k, int kp,
                           hipStream_t s);

// Angular stage on MFMA: G -> gbuf (n_r x n_theta x S x kp) -> gh (in place)
// -> A, as three launches.
template <typename T>
void launch_legendre_synth(const Basis& b, const DevTables<T>& tb, const T* G, T* gbuf, int kp,
                           hipStream_t s);
template <typename T>
void launch_phi_stage(const Basis& b, const T* ab, T* gbuf, int kp, hipStream_t s);
template <typename T>
void launch_legendre_analysis(const Basis& b, const DevTables<T>& tb, const T* gbuf, T* A,
                              int kp, hipStream_t s);


// C (k x k, column-major, ld k) = A^T B for d x k blocks, or its symmetric
// part (A^T B + B^T A) / 2 with sym, split over rows with partial sums in
// `part` (gram_chunks(rows, k) * k * k doubles).
int gram_chunks(int64_t rows, int k);
void launch_gram(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                 double* part, int64_t rows, int k, hipStream_t s, bool sym = false);

void launch_veff_fourier(const Basis& b, const double* V, double* ab64, float* ab32,
                         hipStream_t s);

template <typename Tin, typename Tout>
void launch_convert(const Tin* src, int64_t lds, Tout* dst, int64_t ldd, int64_t rows,
                    int cols, hipStream_t s);

// C[q][i] *= h[q] for q < rows, i < ld.
// Leading dimension of the library's FP32 blocks of d-vectors (the mixed
// precision's copies of X and H X, and the FP32 projectors): d rounded up to
// 32, so every column starts on a 128-byte line and a 32-float segment of it
// (one staged step of the projector products) is one line.
inline int64_t f32_ld(int64_t d) { return (d + 31) / 32 * 32; }
// C[q][i] = h_q sum_alpha P[q][alpha] Y[alpha][i] (projector product; P n_proj x d
// row-major with row stride ldp, Y column-major d x k, C row-major n_proj x kp
// with zeros for i >= k); part: kb_partial_bytes(n_proj, k, d) bytes of scratch.
size_t kb_partial_bytes(int n_proj, int k, int64_t d);
template <typename T>
void launch_kb_gemm(const T* P, int64_t d, int64_t ldp, const T* Y, int64_t ldy, const T* h,
                    T* C, T* part, int n_proj, int k, int kp, hipStream_t s);
// part[c][q][i] (row-major k x kp per chunk c of the rows) = the chunk's share
// of (A^T B)[q][i] for column-major rows x k blocks A, B, on FP64 MFMA with
// the projector product's kernel; at most part_cap doubles of part are used.
// Returns the number of chunks.
int launch_atb_partial(const double* A, int64_t lda, const double* B, int64_t ldb, double* part,
                       int64_t part_cap, int64_t rows, int k, int kp, hipStream_t s);
// Z[alpha][i] = sum_q P[q][alpha] C[q][i] (P row stride ldp; Z column-major d x k,
// ld d).
template <typename T>
void launch_kb_apply(const T* P, int64_t d, int64_t ldp, const T* C, T* Z, int n_proj, int k,
                     int kp, hipStream_t s);

// Phi transforms of k grid functions (column i at f + i ldf, [r][j][p]) to /
// from the Legendre stages' layout g[r][j][s][c] with kp columns (columns k ..
// kp-1 of the analysis output zeroed).
void launch_phi_synthesis_cols(const Basis& b, const double* g, int k, int kp, double* f,
                               int64_t ldf, hipStream_t s);
void launch_phi_analysis_cols(const Basis& b, const double* f, int64_t ldf, int k, int kp,
                              double* gh, hipStream_t s);
// rho[r][j][p] = 2 sum_i occ_i psi_i(r, j, p)^2 from the Legendre-synthesis
// output gbuf (n_r x n_theta x S x kp), accumulated in FP64.
template <typename T>
void launch_density_phi(const Basis& b, const T* gbuf, const double* occ, double* rho, int k,
                        int kp, hipStream_t s);
// gh[r][j][s][c] (16 columns, c > 0 zero) = phi analysis of one grid
// function f[r][j][p], the input of launch_legendre_analysis with kp = 16.
void launch_phi_analysis_one(const Basis& b, const double* f, double* gh, hipStream_t s);
// f[r][j][p] = phi synthesis of column 0 of g (Legendre-synthesis output with
// kp = 16): one grid function.
void launch_phi_synthesis_one(const Basis& b, const double* g, double* f, hipStream_t s);

// Self-consistent field extras (kernels_scf.hip).
void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s);
// v = vext + v + V_x(rho) [+ v_c(rho) when corr], v holding V_H on entry.
void launch_ks_finish(const double* vext, const double* rho, double* v, int64_t n, int corr,
                      hipStream_t s);
// Perdew-Zunger LDA correlation: vc (and ec when not null) elementwise.
void launch_pz_correlation(const double* rho, double* vc, double* ec, int64_t n, hipStream_t s);
// vx = -(3 rho_+ / pi)^(1/3) elementwise (vx may be rho).
void launch_slater_x(const double* rho, double* vx, int64_t n, hipStream_t s);
// Complex <-> real harmonic coefficients (kernels.hip), d x k interleaved
// complex blocks with leading dimensions in complex entries.
void launch_coeffs_c2r(const Basis& b, const double* f, int64_t ldf, double* sr, int64_t lds,
                       int k, hipStream_t s);
void launch_coeffs_r2c(const Basis& b, const double* sr, int64_t lds, double* f, int64_t ldf,
                       int k, hipStream_t s);
// out = sum_i c_i (V_i + beta F_i) over m columns of ld-strided history.
void launch_anderson_combine(const double* V, const double* F, int64_t ld, const double* c,
                             int m, double beta, double* out, int64_t n, hipStream_t s);
// rho on the grid = sum over atoms of sum_n cn[n] j0(n' pi |x - a| / R), n' = n + 1.
void launch_sad_density(const Basis& b, const double* atoms, int n_atoms, const double* cn,
                        double* rho, hipStream_t s);

// Learned start density (kernels_mlp.hip).  Row-major FP32 GEMM:
// C = alpha op(A) op(B) + beta C, op(A) = A^T if ta (A stored K x M).
void launch_gemm_f32(bool ta, bool tb, const float* A, int lda, const float* B, int ldb, float* C,
                     int ldc, int M, int N, int K, float alpha, float beta, hipStream_t s);
void launch_standardize(const float* X, const float* mean, const float* sd, float* H,
                        int64_t rows, int cols, hipStream_t s);
void launch_bias_act(float* Z, const float* b, float* H, int64_t rows, int cols, bool act,
                     hipStream_t s);
void launch_act_grad(float* G, const float* Z, int64_t n, hipStream_t s);
void launch_colsum(const float* G, float* db, int64_t rows, int cols, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s);
// F: n_grid x (8 n_atoms + 1) column-major, sqrt(W) Phi and sqrt(W) target.
void launch_fit_columns(const Basis& b, const double* atoms, const double* dirs, int n_atoms,
                        const double* target, double* F, hipStream_t s);
void launch_density_correction(const Basis& b, const double* atoms, const double* dirs,
                               int n_atoms, const float* coef, double* rho, hipStream_t s);
void launch_cluster_quad_loss(int n_clusters, const int64_t* row_off, const int64_t* m_off,
                              const float* M, const float* p, const float* t, const float* out,
                              float* gout, float* loss, float scale, int max_nq, hipStream_t s);

// Small blocks (k <= kJacobiMax): the k x k matrices that rotate a block are
// written with leading dimension small_ld(k) = k rounded up to 16, zero
// outside k x k (buffers hold small_ld(k)^2 doubles).
constexpr int kJacobiMax = 60;
int small_ld(int k);
// Eigenpairs of a symmetric k x k matrix S (column-major, ld k) in one
// workgroup: eigenvectors overwrite S (ld small_ld(k)), eigenvalues ascending
// in evals; *info = 0 on convergence.
void launch_jacobi_eig(double* S, int k, double* evals, int* info, hipStream_t s);
// From the Gram matrix S (ld k): D = diag(S)^{-1/2} into dinv, D S D + shift I
// = R^T R, S <- D R^{-1} (ld small_ld(k), zero-padded); *info = 0 or the
// 1-based index of the first pivot not above 2 k eps.
void launch_chol_inv(double* S, int k, double shift, double* dinv, int* info, hipStream_t s);
// X <- X W in place (W ld small_ld(k), zero-padded); rows are written only
// where flags[0] and flags[1] are zero.
void launch_block_apply(double* X, int64_t ldx, const double* W, int k, int64_t rows,
                        const int* flags, hipStream_t s);
// X <- X W and Y <- Y W in place (W dense, ld small_ld(k), zero-padded) and
// res_j = || (Y W)_j - theta_j (X W)_j ||; X and Y are written only where
// flags[0] and flags[1] are zero.
void launch_block_rotate(double* X, int64_t ldx, double* Y, int64_t ldy, const double* W, int k,
                         int64_t rows, const int* flags, const double* theta, double* res,
                         double* part, int64_t part_cap, hipStream_t s);
// LOBPCG (kernels_lobpcg.hip).  W[:, j] = AX[:, act[j]] - theta[act[j]] X[:, act[j]]
// for j < na, and ke[j] = the kinetic energy per unit norm of W[:, j]
// (sum (Lambda/2) w^2 / sum w^2, lamh the [l][N] table of Lambda / 2); part:
// 2 * 64 * na doubles of scratch.
void launch_active_residual(const double* X, int64_t ldx, const double* AX, int64_t ldax,
                            const double* theta, const int* act, int na, double* W, int64_t ldw,
                            const double* lam, int64_t rows, double* part, double* ke,
                            hipStream_t s);
// W[alpha, j] *= T(g_scale Lambda_alpha / ke[j]) (Teter-Payne-Allan factor);
// lam[alpha] = Lambda_alpha.
void launch_tpa_scale(double* W, int64_t ldw, int na, const double* ke, const double* lam,
                      double g_scale, int64_t rows, hipStream_t s);
// dst[:, j] = src[:, list[j]] for j < n.
void launch_gather_cols(const double* src, int64_t lds, const int* list, int n, double* dst,
                        int64_t ldd, int64_t rows, hipStream_t s);

// Largest block Rayleigh-Ritz accepts (its pinned read-back stage is sized
// for it when the Hamiltonian is created).
constexpr int kRRMax = 32768;
// After potrf of the unit-diagonal D S D (upper factor R, ld k): if info[0]
// is still 0 and some R_jj^2 <= 2 k eps, info[0] = j + 1 for the first such j.
void launch_check_pivots(const double* R, int k, int* info, hipStream_t s);
// S(i, j) *= dinv[i], k x k column-major.
void launch_scale_rows_k(double* S, int k, const double* dinv, hipStream_t s);
// dst <- src unless flags[0] or flags[1] is nonzero (checked on the device).
void launch_copy2d_if(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                      int cols, const int* flags, hipStream_t s);

// Small FP64 helpers for Cholesky-QR / Rayleigh-Ritz / Lanczos.
void launch_scale_gram(double* S, int k, double* dinv, hipStream_t s);
void launch_scale_cols(double* X, int64_t ldx, int64_t rows, int k, const double* dinv,
                       hipStream_t s);
void launch_symmetrize(double* S, int k, hipStream_t s);
void launch_add_diag(double* S, int k, double shift, hipStream_t s);
void launch_zero_lower(double* S, int k, hipStream_t s);
void launch_residuals(const double* HX, int64_t ldh, const double* X, int64_t ldx,
                      const double* theta, double* res, int64_t rows, int k, double* part,
                      int64_t part_cap, hipStream_t s);
void launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                   int cols, hipStream_t s);
// *out = x . y; part: kDotBlocks doubles of scratch.
constexpr int kDotBlocks = 64;
void launch_dot(const double* x, const double* y, int64_t n, double* out, double* part,
                hipStream_t s);
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);

}  // namespace ces

struct ces_basis_s {
  ces::Basis b;
};
struct ces_ham_s {
  ces::Ham h;
};

namespace ces {
ces_status check_ham(ces_ham hh);   // non-null and on the current device
ces_status ensure_device(Basis& b);  // uploads the basis tables once (current device)
}  // namespace ces
