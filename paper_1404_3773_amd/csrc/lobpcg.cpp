// Block LOBPCG with soft and hard locking and the Teter-Payne-Allan
// preconditioner (Section 3.1, 3.1.2): the paper's other eigensolver, used
// for the first SCF step.  Host sequencing of device work: H*W through the
// H*X kernels, FP64 Gram products on the split-row / split-K MFMA kernels,
// column-scaled Cholesky factorisations, the projected pencil by rocSOLVER
// sygvd, and the block updates.  One host synchronisation per decision
// (active set, factorisation status, pencil status).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ces_internal.h"

namespace ces {
namespace {

#define CES_BLAS(call)                                                                  \
  do {                                                                                  \
    rocblas_status e_ = (call);                                                         \
    if (e_ != rocblas_status_success)                                                   \
      return fail(CES_ERR_DEVICE, std::string(#call) + ": " + rocblas_status_to_string(e_)); \
  } while (0)

// Workspace of one LOBPCG call: the regions of the Rayleigh-Ritz / H*X layout
// for k columns, then the LOBPCG blocks.
struct LobLayout {
  Layout base;
  size_t S = 0, AS = 0, P = 0, AP = 0, T = 0, gA = 0, gB = 0, evm = 0, ework = 0, M1 = 0,
         act = 0, rpart = 0, ke = 0, info = 0, gpart = 0, kbpart = 0, solver = 0, total = 0;
  size_t solver_bytes = 0;
  size_t gcap = 0;   // doubles in gpart
  int m = 0;         // largest projected order, 3k
};

size_t lob_solver_bytes(Ham& h, int k, int m) {
  size_t sz = 0;
  std::lock_guard<std::mutex> lock(h.mu);
  if (rocblas_start_device_memory_size_query(h.blas) == rocblas_status_success) {
    if (rocblas_is_device_memory_size_query(h.blas)) {
      double* fake = reinterpret_cast<double*>(uintptr_t(4096));
      rocblas_int* ifake = reinterpret_cast<rocblas_int*>(uintptr_t(4096));
      (void)rocsolver_dsygvd(h.blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper,
                             m, fake, m, fake, m, fake, fake, ifake);
      (void)rocsolver_dpotrf(h.blas, rocblas_fill_upper, k, fake, k, ifake);
      (void)rocsolver_dtrtri(h.blas, rocblas_fill_upper, rocblas_diagonal_non_unit, k, fake, k,
                             ifake);
    }
    (void)rocblas_stop_device_memory_size_query(h.blas, &sz);
  }
  return align256(sz) + (16u << 20);
}

LobLayout lob_layout(Ham& h, int k, int n_lock, int prec) {
  LobLayout L;
  L.base = layout_for(h, k, prec);
  const int64_t d = h.basis->d;
  L.m = 3 * k;
  const size_t m = size_t(L.m);
  size_t off = L.base.total;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t at = off;
    off += bytes + 4096;
    return at;
  };
  const size_t blk = size_t(d) * sizeof(double);
  L.S = take(3 * size_t(k) * blk);
  L.AS = take(3 * size_t(k) * blk);
  L.P = take(size_t(k) * blk);
  L.AP = take(size_t(k) * blk);
  L.T = take(size_t(k) * blk);
  L.gA = take(m * m * sizeof(double));
  L.gB = take(m * m * sizeof(double));
  L.evm = take(m * sizeof(double));
  L.ework = take(m * sizeof(double));
  L.M1 = take(std::max(size_t(small_ld(k)) * small_ld(k), size_t(std::max(n_lock, 1)) * k) *
              sizeof(double));
  L.act = take(size_t(k) * sizeof(int));
  L.rpart = take(size_t(2 * 64) * k * sizeof(double));
  L.ke = take(size_t(k) * sizeof(double));
  L.info = take(8 * sizeof(int));
  // Gram partial sums for any order n <= m (the chunk count falls as n grows)
  size_t gp = 0;
  for (int n = 1; n <= L.m; ++n) gp = std::max(gp, size_t(gram_chunks(d, n)) * n * n);
  L.gcap = gp;
  L.gpart = take(gp * sizeof(double));
  // projector-product partial sums for H*W on any number of active columns
  L.kbpart = take(kb_partial_bytes(h.n_proj, k, d));
  L.solver_bytes = lob_solver_bytes(h, k, L.m);
  L.solver = take(L.solver_bytes);
  L.total = align256(off);
  return L;
}

struct Lob {
  Ham& h;
  const LobLayout& ly;
  void* work;
  hipStream_t s;
  int64_t d;
  int* info;
  double* gpart;
  int64_t gcap;
  double* T;

  template <typename U>
  U* at(size_t off) const { return Ptr<U>::at(work, off); }

  ces_status set_solver_workspace() {
    CES_BLAS(rocblas_set_stream(h.blas, s));
    CES_BLAS(rocblas_set_workspace(h.blas, at<char>(ly.solver), ly.solver_bytes));
    return CES_OK;
  }

  // Reads `n` status ints from the device (after the work queued so far).
  ces_status read_ints(const int* src, int n, int* out) {
    CES_HIP(hipGetLastError());
    CES_TRY(stage_read(h, 0, src, size_t(n) * sizeof(int), s));
    CES_HIP(hipStreamSynchronize(s));
    std::memcpy(out, h.host_stage, size_t(n) * sizeof(int));
    return CES_OK;
  }

  // V <- V - Y (Y^T V) for the n_lock orthonormal constraint columns Y.
  ces_status project_out(double* V, int n, const double* Y, int64_t ldy, int n_lock) {
    if (n_lock == 0) return CES_OK;
    const double one = 1.0, zero = 0.0, mone = -1.0;
    double* C = at<double>(ly.M1);
    CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_transpose, rocblas_operation_none, n_lock, n,
                           static_cast<int>(d), &one, Y, static_cast<int>(ldy), V,
                           static_cast<int>(d), &zero, C, n_lock));
    CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                           static_cast<int>(d), n, n_lock, &mone, Y, static_cast<int>(ldy), C,
                           n_lock, &one, V, static_cast<int>(d)));
    return CES_OK;
  }

  // Column-scaled Cholesky-QR factor of V (d x n, ld d): M = D R^{-1}, then
  // V <- V M and AV <- AV M (AV may be null).  Status in flags[0..1] (both 0
  // on success; on failure V and AV are left as they were).
  ces_status cholqr(double* V, double* AV, int n, int* flags) {
    double* M = at<double>(ly.M1);
    double* dinv = at<double>(ly.ke);   // free at this point of an iteration
    launch_gram(V, d, V, d, M, gpart, d, n, s, true);
    if (n <= kJacobiMax) {
      launch_chol_inv(M, n, 0.0, dinv, flags, s);
      launch_block_apply(V, d, M, n, d, flags, s);
      if (AV) launch_block_apply(AV, d, M, n, d, flags, s);
      return CES_OK;
    }
    launch_scale_gram(M, n, dinv, s);
    CES_BLAS(rocsolver_dpotrf(h.blas, rocblas_fill_upper, n, M, n, flags));
    launch_check_pivots(M, n, flags, s);
    launch_zero_lower(M, n, s);
    CES_BLAS(rocsolver_dtrtri(h.blas, rocblas_fill_upper, rocblas_diagonal_non_unit, n, M, n,
                              flags + 1));
    launch_scale_rows_k(M, n, dinv, s);
    const double one = 1.0, zero = 0.0;
    for (double* B : {V, AV}) {
      if (!B) continue;
      CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                             static_cast<int>(d), n, n, &one, B, static_cast<int>(d), M, n, &zero,
                             T, static_cast<int>(d)));
      launch_copy2d_if(T, d, B, d, d, n, flags, s);
    }
    return CES_OK;
  }
};

}  // namespace

size_t lobpcg_workspace_bytes(Ham& h, int k, int n_lock, int prec) {
  return lob_layout(h, k, n_lock, prec).total;
}

}  // namespace ces

using namespace ces;

extern "C" {

ces_status ces_lobpcg_workspace_size(ces_ham hh, int k, int n_lock, int prec, size_t* bytes) {
  if (!hh || !bytes) return fail(CES_ERR_INVALID_ARG, "null argument");
  if (k < 1 || n_lock < 0) return fail(CES_ERR_INVALID_ARG, "bad block sizes");
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  *bytes = lob_layout(hh->h, k, n_lock, prec).total;
  return CES_OK;
}

ces_status ces_lobpcg(ces_ham hh, int k, double* d_X, int64_t ldx, int n_lock, const double* d_Y,
                      int64_t ldy, int n_check, int max_iter, double res_tol, double g_scale,
                      int precondition, int prec, double* d_eval, double* d_resnorm, int* h_iters,
                      int* h_restarts, void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  const Basis& b = *h.basis;
  const int64_t d = b.d;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_eval || !d_resnorm || !h_iters) return fail(CES_ERR_INVALID_ARG, "null output");
  if (n_lock < 0 || (n_lock > 0 && (!d_Y || ldy < d)))
    return fail(CES_ERR_INVALID_ARG, "bad constraint block");
  if (3 * int64_t(k) + n_lock > d || k > kRRMax)
    return fail(CES_ERR_INVALID_ARG, "3 k + n_lock must not exceed d (and k <= 32768)");
  if (n_check < 1 || n_check > k || max_iter < 0 || !(res_tol > 0) || !(g_scale > 0))
    return fail(CES_ERR_INVALID_ARG, "bad iteration parameters");
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  if (!d_work) return fail(CES_ERR_WORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(CES_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const LobLayout ly = lob_layout(h, k, n_lock, prec);   // before taking h.mu
  if (work_bytes < ly.total)
    return fail(CES_ERR_WORKSPACE, "workspace too small: need " + std::to_string(ly.total) +
                                       " bytes, got " + std::to_string(work_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(h.mu);   // rocBLAS handle and host_stage
  Lob L{h, ly, d_work, s, d, Ptr<int>::at(d_work, ly.info), Ptr<double>::at(d_work, ly.gpart),
        int64_t(ly.gcap), Ptr<double>::at(d_work, ly.T)};
  double* S = L.at<double>(ly.S);
  double* AS = L.at<double>(ly.AS);
  double* P = L.at<double>(ly.P);
  double* AP = L.at<double>(ly.AP);
  double* gA = L.at<double>(ly.gA);
  double* gB = L.at<double>(ly.gB);
  double* evm = L.at<double>(ly.evm);
  int* act_d = L.at<int>(ly.act);
  std::vector<double> theta(k), res(k);
  int restarts = 0;

  // Rayleigh-Ritz of the block in S[:, :k] (orthonormalises it), AX in AS.
  auto ritz = [&]() -> ces_status {
    CES_TRY(rr_locked(h, ly.base, d_work, k, S, d, AS, d, evm, d_resnorm, CES_PREC_FP64, s,
                      theta.data(), res.data(), nullptr));
    return L.set_solver_workspace();
  };
  // H * V for n columns of V (ld d) into AV (ld d), in the call's precision,
  // on the H*X regions with the column padding of n columns
  auto apply = [&](const double* V, double* AV, int n) -> ces_status {
    Layout lw = ly.base;
    lw.kp = round_up(n, kColPad);
    lw.Cpart = ly.kbpart;
    if (prec == CES_PREC_FP64)
      return h_step<double>(h, lw, d_work, n, V, d, nullptr, 0, AV, d, 1.0, 0.0, 0.0, s);
    float* F0 = Ptr<float>::at(d_work, lw.F0);
    float* F1 = Ptr<float>::at(d_work, lw.F1);
    const int64_t ldf = f32_ld(d);
    launch_convert<double, float>(V, d, F0, ldf, d, n, s);
    CES_TRY(h_step<float>(h, lw, d_work, n, F0, ldf, nullptr, 0, F1, ldf, 1.0f, 0.0f, 0.0f, s));
    launch_convert<float, double>(F1, ldf, AV, d, d, n, s);
    return CES_OK;
  };

  // start: deflate against the constraints, then Rayleigh-Ritz
  launch_copy2d(d_X, ldx, S, d, d, k, s);
  CES_TRY(L.set_solver_workspace());
  CES_TRY(L.project_out(S, k, d_Y, ldy, n_lock));
  CES_TRY(ritz());
  bool have_p = false;
  int it = 0;
  while (true) {
    std::vector<int> act;
    bool done = true;
    for (int i = 0; i < k; ++i) {
      const bool conv = res[i] <= res_tol * std::max(1.0, std::fabs(theta[i]));
      if (!conv) {
        act.push_back(i);
        if (i < n_check) done = false;
      }
    }
    if (done || it >= max_iter) break;
    ++it;
    const int na = static_cast<int>(act.size());
    // active list to the device through the pinned stage
    std::memcpy(h.host_stage, act.data(), size_t(na) * sizeof(int));
    CES_HIP(hipMemcpyAsync(act_d, h.host_stage, size_t(na) * sizeof(int),
                           hipMemcpyHostToDevice, s));
    CES_HIP(hipMemsetAsync(L.info, 0, 8 * sizeof(int), s));
    double* W = S + int64_t(k) * d;
    double* AW = AS + int64_t(k) * d;
    launch_active_residual(S, d, AS, d, evm, act_d, na, W, d, b.dev_lam, d,
                           L.at<double>(ly.rpart), L.at<double>(ly.ke), s);
    if (precondition) launch_tpa_scale(W, d, na, L.at<double>(ly.ke), b.dev_lam, g_scale, d, s);
    CES_TRY(L.project_out(W, na, d_Y, ldy, n_lock));
    CES_TRY(L.cholqr(W, nullptr, na, L.info));
    bool use_p = have_p;
    if (use_p) {
      double* Pa = S + int64_t(k + na) * d;
      double* APa = AS + int64_t(k + na) * d;
      launch_gather_cols(P, d, act_d, na, Pa, d, d, s);
      launch_gather_cols(AP, d, act_d, na, APa, d, d, s);
      CES_TRY(L.cholqr(Pa, APa, na, L.info + 2));
    }
    int flags[4];
    CES_TRY(L.read_ints(L.info, 4, flags));
    bool restart = flags[0] != 0 || flags[1] != 0;
    if (!restart && use_p && (flags[2] != 0 || flags[3] != 0)) {
      use_p = false;   // conjugate directions degenerate: go on without them
      ++restarts;
    }
    bool solved = false;
    int m = 0;
    if (!restart) {
      CES_TRY(apply(W, AW, na));
      // Rayleigh-Ritz on span[X, W, P]; without P if the pencil fails
      while (true) {
        m = k + na + (use_p ? na : 0);
        launch_gram(S, d, S, d, gB, L.gpart, d, m, s, true);
        launch_gram(S, d, AS, d, gA, L.gpart, d, m, s, true);
        CES_BLAS(rocsolver_dsygvd(h.blas, rocblas_eform_ax, rocblas_evect_original,
                                  rocblas_fill_upper, m, gA, m, gB, m, evm,
                                  L.at<double>(ly.ework), L.info + 4));
        int st = 0;
        CES_TRY(L.read_ints(L.info + 4, 1, &st));
        if (st == 0) {
          solved = true;
          break;
        }
        if (!use_p) break;
        use_p = false;
        ++restarts;
      }
    }
    if (!solved) {
      // restart from the current Ritz vectors without W and P (Section 3.1)
      ++restarts;
      have_p = false;
      CES_TRY(ritz());
      continue;
    }
    // P = [W, P_a] C_r, AP likewise; X = X C_x + P, AX = AX C_x + AP
    const double one = 1.0, zero = 0.0;
    const int nr = m - k;
    CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                           static_cast<int>(d), k, nr, &one, W, static_cast<int>(d), gA + k, m,
                           &zero, P, static_cast<int>(d)));
    CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                           static_cast<int>(d), k, nr, &one, AW, static_cast<int>(d), gA + k, m,
                           &zero, AP, static_cast<int>(d)));
    for (int pass = 0; pass < 2; ++pass) {
      double* B = pass == 0 ? S : AS;
      double* Q = pass == 0 ? P : AP;
      CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                             static_cast<int>(d), k, k, &one, B, static_cast<int>(d), gA, m,
                             &zero, L.T, static_cast<int>(d)));
      launch_axpby(1.0, Q, 1.0, L.T, d * k, s);
      launch_copy2d(L.T, d, B, d, d, k, s);
    }
    have_p = true;
    launch_residuals(AS, d, S, d, evm, d_resnorm, d, k, L.gpart, L.gcap, s);
    CES_HIP(hipGetLastError());
    CES_TRY(stage_read(h, 2, evm, size_t(k) * 8, s));
    CES_TRY(stage_read(h, 2 + size_t(k), d_resnorm, size_t(k) * 8, s));
    CES_HIP(hipStreamSynchronize(s));
    std::memcpy(theta.data(), h.host_stage + 2, size_t(k) * 8);
    std::memcpy(res.data(), h.host_stage + 2 + k, size_t(k) * 8);
  }
  // the final Ritz vectors into the caller's block, with one more FP64
  // Rayleigh-Ritz (orthonormal to rounding, eigenvalues and residuals of it)
  launch_copy2d(S, d, d_X, ldx, d, k, s);
  CES_TRY(rr_locked(h, ly.base, d_work, k, d_X, ldx, nullptr, ldx, d_eval, d_resnorm,
                    CES_PREC_FP64, s, nullptr, nullptr, nullptr));
  *h_iters = it;
  if (h_restarts) *h_restarts = restarts;
  return CES_OK;
}

}  // extern "C"
