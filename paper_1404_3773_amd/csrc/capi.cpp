// C interface of libces (declared in include/ces.h): handle lifecycle,
// argument validation, workspace carving and the host-side sequencing of the
// device kernels for H*X, the Chebyshev filter, Cholesky-QR + Rayleigh-Ritz,
// Lanczos bounds, the CheFSI driver, density and grid transforms.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ces_internal.h"
#include "setup_tables.h"


namespace ces {

thread_local std::string g_err;

ces_status fail(ces_status s, const std::string& msg) {
  g_err = msg;
  return s;
}


#define CES_BLAS(call)                                                             \
  do {                                                                             \
    rocblas_status e_ = (call);                                                    \
    if (e_ != rocblas_status_success)                                              \
      return fail(CES_ERR_DEVICE, std::string(#call) + ": " + rocblas_status_to_string(e_)); \
  } while (0)


// Stage timing (ces_profile_enable / ces_profile_read): stage ids 0..6 for
// FP32 launches, 7..13 for FP64 launches.
enum { ST_RADIAL_INV = 0, ST_LEG_SYNTH, ST_PHI, ST_LEG_ANALYSIS, ST_RADIAL_FWD, ST_KB_C, ST_KB_Z,
       ST_PER_PREC };
constexpr int kStages = 2 * ST_PER_PREC;
template <typename T>
constexpr int stage_id(int st) { return st + (sizeof(T) == 8 ? ST_PER_PREC : 0); }
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> ev;     // 2 per record
  std::vector<int> stage;         // stage of each used record
  double ms[kStages] = {};
  int64_t count[kStages] = {};
};
Profiler g_prof;

struct StageTimer {
  int rec = -1;
  hipStream_t s;
  StageTimer(int st, hipStream_t stream) : s(stream) {
    if (!g_prof.on) return;
    const size_t used = g_prof.stage.size();
    if (2 * used + 2 > g_prof.ev.size()) return;
    rec = static_cast<int>(used);
    g_prof.stage.push_back(st);
    (void)hipEventRecord(g_prof.ev[2 * rec], s);
  }
  ~StageTimer() {
    if (rec >= 0) (void)hipEventRecord(g_prof.ev[2 * rec + 1], s);
  }
};

// Host tables of the basis (Section 2.2.1-2.2.2).
void build_host_tables(Basis& b) {
  const int L = b.L, N = b.N;
  b.zeros = bessel_zeros(L, N);
  std::vector<double> x, w;
  if (b.rule == CES_RADIAL_GAUSS_JACOBI_R2) {
    gauss_jacobi(b.n_r, 0.0, 2.0, x, w);  // weight (1+x)^2 on [-1,1]
    b.r.resize(b.n_r);
    b.wr.resize(b.n_r);
    for (int i = 0; i < b.n_r; ++i) {
      b.r[i] = b.R * (1.0 + x[i]) / 2.0;
      b.wr[i] = w[i] * std::pow(b.R / 2.0, 3);
    }
  } else {
    gauss_jacobi(b.n_r, 0.0, 0.0, x, w);
    b.r.resize(b.n_r);
    b.wr.resize(b.n_r);
    for (int i = 0; i < b.n_r; ++i) {
      b.r[i] = b.R * (1.0 + x[i]) / 2.0;
      b.wr[i] = w[i] * (b.R / 2.0) * b.r[i] * b.r[i];
    }
  }
  gauss_jacobi(b.n_theta, 0.0, 0.0, x, w);  // ascending t
  b.t.resize(b.n_theta);
  b.wt.resize(b.n_theta);
  b.theta.resize(b.n_theta);
  for (int j = 0; j < b.n_theta; ++j) {  // order by increasing theta
    b.t[j] = x[b.n_theta - 1 - j];
    b.wt[j] = w[b.n_theta - 1 - j];
    b.theta[j] = std::acos(b.t[j]);
  }
  // exact symmetry t_{n-1-j} = -t_j (the kernels rely on it)
  for (int j = 0; j < b.n_theta / 2; ++j) {
    const int jn = b.n_theta - 1 - j;
    const double tt = 0.5 * (b.t[j] - b.t[jn]);
    const double ww = 0.5 * (b.wt[j] + b.wt[jn]);
    b.t[j] = tt;
    b.t[jn] = -tt;
    b.wt[j] = b.wt[jn] = ww;
    b.theta[j] = std::acos(tt);
    b.theta[jn] = std::acos(-tt);
  }
  if (b.n_theta % 2 == 1) {
    b.t[b.n_theta / 2] = 0.0;
    b.theta[b.n_theta / 2] = M_PI / 2;
  }
  b.phi.resize(b.n_phi);
  for (int p = 0; p < b.n_phi; ++p) b.phi[p] = 2.0 * M_PI * p / b.n_phi;
  // R_ln(r_k) = sqrt(2/R^3) j_l(b_ln r_k / R) / j_{l+1}(b_ln)
  b.radial.assign(static_cast<size_t>(L) * b.n_r * N, 0.0);
  const double c0 = std::sqrt(2.0 / (b.R * b.R * b.R));
  for (int l = 0; l < L; ++l)
    for (int n = 0; n < N; ++n) {
      const double z = b.zeros[static_cast<size_t>(l) * N + n];
      const double den = sph_bessel_j(l + 1, z);
      for (int kk = 0; kk < b.n_r; ++kk)
        b.radial[(static_cast<size_t>(l) * b.n_r + kk) * N + n] =
            c0 * sph_bessel_j(l, z * b.r[kk] / b.R) / den;
    }
  const int LP = L * (L + 1) / 2;
  b.legendre.assign(static_cast<size_t>(b.n_theta) * LP, 0.0);
  for (int j = 0; j < b.n_theta; ++j) legendre_normalized(L, b.t[j], &b.legendre[size_t(j) * LP]);
}

template <typename T>
void fill_tables(const Basis& b, std::vector<T>& Rinv, std::vector<T>& Rfwd,
                 std::vector<T>& lamh, std::vector<T>& wt, std::vector<T>& Pm,
                 std::vector<T>& PwT) {
  const int L = b.L, N = b.N, LP = L * (L + 1) / 2;
  // zero-padded MFMA operand tables (see kernels_radial.hip)
  const int N4 = int(round_up(N, 4)), R16 = int(round_up(b.n_r, 16));
  const int R4 = int(round_up(b.n_r, 4)), N16 = int(round_up(N, 16));
  Rinv.assign(static_cast<size_t>(L) * N4 * R16, T(0));   // [l][n][r]
  Rfwd.assign(static_cast<size_t>(L) * R4 * N16, T(0));   // [l][r][n]
  for (int l = 0; l < L; ++l)
    for (int kk = 0; kk < b.n_r; ++kk)
      for (int n = 0; n < N; ++n) {
        const double v = b.radial[(static_cast<size_t>(l) * b.n_r + kk) * N + n];
        Rinv[(static_cast<size_t>(l) * N4 + n) * R16 + kk] = static_cast<T>(v);
        Rfwd[(static_cast<size_t>(l) * R4 + kk) * N16 + n] = static_cast<T>(b.wr[kk] * v);
      }
  lamh.resize(static_cast<size_t>(L) * N);
  for (int l = 0; l < L; ++l)
    for (int n = 0; n < N; ++n) {
      const double k = b.zeros[size_t(l) * N + n] / b.R;
      lamh[size_t(l) * N + n] = static_cast<T>(0.5 * k * k);
    }
  wt.resize(b.n_theta);
  for (int j = 0; j < b.n_theta; ++j) wt[j] = static_cast<T>(b.wt[j]);
  const int nt = b.n_theta;
  const int J64 = int(round_up(nt, 64)), J4 = int(round_up(nt, 4)), L16 = int(round_up(L, 16));
  Pm.assign(static_cast<size_t>(L) * (L + 4) * J64, T(0));   // [m][l][j]
  PwT.assign(static_cast<size_t>(L) * J4 * L16, T(0));       // [m][j][l - m]
  for (int m = 0; m < L; ++m)
    for (int l = m; l < L; ++l)
      for (int j = 0; j < nt; ++j) {
        const double v = b.legendre[size_t(j) * LP + l * (l + 1) / 2 + m] * (m > 0 ? std::sqrt(2.0) : 1.0);
        Pm[(size_t(m) * (L + 4) + l) * J64 + j] = static_cast<T>(v);
        PwT[(size_t(m) * J4 + j) * L16 + (l - m)] = static_cast<T>(b.wt[j] * v);
      }
}

// Upload device tables once (on the device current at first use).
ces_status ensure_device(Basis& b) {
  std::lock_guard<std::mutex> lock(b.dev_mu);
  int dev = 0;
  CES_HIP(hipGetDevice(&dev));
  if (b.dev_block) {
    if (dev != b.device) return fail(CES_ERR_INVALID_ARG, "basis tables live on another device");
    return CES_OK;
  }
  std::vector<double> R64, F64, l64, w64, M64, W64;
  std::vector<float> R32, F32, l32, w32, M32, W32;
  fill_tables(b, R64, F64, l64, w64, M64, W64);
  fill_tables(b, R32, F32, l32, w32, M32, W32);
  std::vector<double> cs(2 * static_cast<size_t>(b.n_phi));
  for (int u = 0; u < b.n_phi; ++u) {
    cs[u] = std::cos(2.0 * M_PI * u / b.n_phi);
    cs[b.n_phi + u] = std::sin(2.0 * M_PI * u / b.n_phi);
  }
  // Hartree radial table (Section 2.3.1): the Laplace-expansion radial
  // integral zeta_ln(r) of R_ln in closed form, with k = b_ln / R,
  //   (4 pi / (2l+1)) zeta_ln(r) = (4 pi / k^2) R_ln(r)
  //                              + (4 pi / (2l+1)) sqrt(2/R^3) R (r/R)^l / k,
  // the Dirichlet Poisson solution plus the harmonic term that continues it
  // as the free-space potential outside the ball.
  const int N4 = int(round_up(b.N, 4)), R16 = int(round_up(b.n_r, 16));
  std::vector<double> hart(static_cast<size_t>(b.L) * N4 * R16, 0.0);
  const double c0 = std::sqrt(2.0 / (b.R * b.R * b.R));
  for (int l = 0; l < b.L; ++l)
    for (int n = 0; n < b.N; ++n) {
      const double k = b.zeros[size_t(l) * b.N + n] / b.R;
      for (int kk = 0; kk < b.n_r; ++kk) {
        const double rad = b.radial[(size_t(l) * b.n_r + kk) * b.N + n];
        hart[(size_t(l) * N4 + n) * R16 + kk] =
            4.0 * M_PI / (k * k) * rad +
            4.0 * M_PI / (2 * l + 1) * c0 * b.R * std::pow(b.r[kk] / b.R, l) / k;
      }
    }
  std::vector<int> lay(2 * size_t(b.L));
  std::vector<double> lam(b.d);
  for (int l = 0; l < b.L; ++l) {
    lay[2 * l] = static_cast<int>(b.off[l]);
    lay[2 * l + 1] = b.Nl[l];
    for (int mm = 0; mm < 2 * l + 1; ++mm)
      for (int n = 0; n < b.Nl[l]; ++n) {
        const double kk = b.zeros[size_t(l) * b.N + n] / b.R;
        lam[b.off[l] + int64_t(mm) * b.Nl[l] + n] = kk * kk;
      }
  }
  std::vector<double> cth(b.n_theta), sth(b.n_theta);
  for (int j = 0; j < b.n_theta; ++j) {
    cth[j] = b.t[j];
    sth[j] = std::sin(b.theta[j]);
  }
  struct Piece {
    const void* src;
    size_t bytes;
    void** dst;
  };
  std::vector<Piece> pieces = {
      {R64.data(), R64.size() * 8, (void**)&b.t64.RiT}, {F64.data(), F64.size() * 8, (void**)&b.t64.RfT},
      {l64.data(), l64.size() * 8, (void**)&b.t64.lamh}, {w64.data(), w64.size() * 8, (void**)&b.t64.wt},
      {R32.data(), R32.size() * 4, (void**)&b.t32.RiT}, {F32.data(), F32.size() * 4, (void**)&b.t32.RfT},
      {l32.data(), l32.size() * 4, (void**)&b.t32.lamh}, {w32.data(), w32.size() * 4, (void**)&b.t32.wt},
      {M64.data(), M64.size() * 8, (void**)&b.t64.Pm},   {W64.data(), W64.size() * 8, (void**)&b.t64.PwT},
      {M32.data(), M32.size() * 4, (void**)&b.t32.Pm},   {W32.data(), W32.size() * 4, (void**)&b.t32.PwT},
      {cs.data(), cs.size() * 8, (void**)&b.dev_cs},
      {hart.data(), hart.size() * 8, (void**)&b.dev_hart},
      {b.r.data(), b.r.size() * 8, (void**)&b.dev_rnode},
      {b.wr.data(), b.wr.size() * 8, (void**)&b.dev_wr},
      {cth.data(), cth.size() * 8, (void**)&b.dev_cth},
      {sth.data(), sth.size() * 8, (void**)&b.dev_sth},
      {lay.data(), lay.size() * sizeof(int), (void**)&b.dev_lay},
      {lam.data(), lam.size() * 8, (void**)&b.dev_lam}};
  size_t total = 0;
  for (auto& p : pieces) total += align256(p.bytes);
  void* blk = nullptr;
  if (hipMalloc(&blk, total) != hipSuccess) return fail(CES_ERR_ALLOC, "hipMalloc of basis tables failed");
  size_t off = 0;
  for (auto& p : pieces) {
    *p.dst = static_cast<char*>(blk) + off;
    if (hipMemcpy(*p.dst, p.src, p.bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(blk);
      return fail(CES_ERR_DEVICE, "upload of basis tables failed");
    }
    off += align256(p.bytes);
  }
  b.dev_block = blk;
  b.device = dev;
  return CES_OK;
}

// ------------------------------------------------------------- workspace


size_t solver_bytes_for(Ham& h, int k) {
  std::lock_guard<std::mutex> lock(h.mu);
  if (h.solver_ws_k == k) return h.solver_ws;
  size_t sz = 0;
  // Size query: no kernel runs while the handle is in query mode; the
  // functions only need non-null placeholders to pass argument checks.
  if (rocblas_start_device_memory_size_query(h.blas) == rocblas_status_success) {
    if (rocblas_is_device_memory_size_query(h.blas)) {
      double* fake = reinterpret_cast<double*>(uintptr_t(4096));
      rocblas_int* ifake = reinterpret_cast<rocblas_int*>(uintptr_t(4096));
      (void)rocsolver_dpotrf(h.blas, rocblas_fill_upper, k, fake, k, ifake);
      (void)rocsolver_dtrtri(h.blas, rocblas_fill_upper, rocblas_diagonal_non_unit, k, fake, k,
                             ifake);
      (void)rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_upper, k, fake, k,
                             fake, fake, ifake);
    }
    (void)rocblas_stop_device_memory_size_query(h.blas, &sz);
  }
  h.solver_ws = align256(sz) + (16u << 20);  // margin for the BLAS-3 calls
  h.solver_ws_k = k;
  return h.solver_ws;
}

// The pinned read-back stage is allocated once, by ces_ham_create, for the
// largest block a Rayleigh-Ritz call accepts; later calls only check that
// what they read back fits.
ces_status host_stage(Ham& h, size_t n) {
  if (h.host_stage_n >= n) return CES_OK;
  if (h.host_stage)
    return fail(CES_ERR_INVALID_ARG, "read-back of " + std::to_string(n) +
                                         " doubles exceeds the handle's pinned stage");
  const size_t want = std::max<size_t>(n, 1024);
  CES_HIP(hipHostMalloc(reinterpret_cast<void**>(&h.host_stage), want * sizeof(double),
                        hipHostMallocDefault));
  h.host_stage_n = want;
  return CES_OK;
}

ces_status stage_read(Ham& h, size_t off, const void* src, size_t bytes, hipStream_t s) {
  CES_TRY(host_stage(h, off + (bytes + 7) / 8));
  CES_HIP(hipMemcpyAsync(h.host_stage + off, src, bytes, hipMemcpyDeviceToHost, s));
  return CES_OK;
}

Layout layout_for(Ham& h, int k, int prec) {
  const Basis& b = *h.basis;
  Layout L;
  L.kp = round_up(k, kColPad);
  const size_t LL = size_t(b.L) * b.L;
  // G, A and gbuf: the FP32 product's kp columns in mixed precision (FP64
  // products, e.g. Rayleigh-Ritz's H X, then run in chunks of kc64 columns),
  // the FP64 product's kp columns otherwise
  size_t ecols;
  if (prec == CES_PREC_MIXED) {
    // half the columns (rounded up to 16), so an FP64 product takes two chunks
    L.kc64 = round_up((L.kp + 1) / 2, kColPad);
    ecols = std::max(size_t(L.kp) * sizeof(float), size_t(L.kc64) * sizeof(double));
  } else {
    L.kc64 = L.kp;
    ecols = size_t(L.kp) * sizeof(double);
  }
  size_t gbytes = size_t(b.n_r) * LL * ecols;
  size_t gbuf = size_t(b.n_r) * b.n_theta * (2 * size_t(b.L) - 1) * ecols;
  size_t v3 = size_t(b.d) * 3 * sizeof(double);
  if (const Basis* bd = h.rho_basis) {   // one-column transforms on the density basis
    gbytes = std::max(gbytes, size_t(bd->n_r) * bd->L * bd->L * kColPad * sizeof(double));
    gbuf = std::max(gbuf, size_t(bd->n_r) * bd->n_theta * (2 * size_t(bd->L) - 1) * kColPad *
                              sizeof(double));
    v3 = std::max(v3, size_t(bd->d) * sizeof(double));
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t at = off;
    off += bytes + 4096;   // slack past every region
    return at;
  };
  L.G = take(gbytes);
  L.A = take(gbytes);
  L.gbuf = take(gbuf);
  L.B1 = take(size_t(b.d) * k * sizeof(double));
  L.B2 = take(size_t(b.d) * k * sizeof(double));
  L.V3 = take(v3);
  if (prec == CES_PREC_MIXED) {
    L.F0 = take(size_t(f32_ld(b.d)) * L.kp * sizeof(float));
    L.F1 = take(size_t(f32_ld(b.d)) * L.kp * sizeof(float));
  }
  L.C = take(size_t(std::max(h.n_proj, 1)) * L.kp * sizeof(double));
  L.Cpart = take(kb_partial_bytes(h.n_proj, k, b.d));
  L.Zkb = take(h.n_proj > 0 ? size_t(b.d) * L.kp * sizeof(double) : 0);
  const size_t kk = std::max<size_t>(size_t(k) * k, size_t(small_ld(k)) * small_ld(k));
  L.S1 = take(kk * sizeof(double));
  L.S2 = take(kk * sizeof(double));
  L.vec = take(size_t(8) * std::max(k, 64) * sizeof(double));
  L.part = take(size_t(gram_chunks(b.d, k)) * k * k * sizeof(double));
  L.info = take(256);
  L.solver_bytes = solver_bytes_for(h, k);
  L.solver = take(L.solver_bytes);
  L.total = align256(off);
  return L;
}

// Regions one H*X needs and nothing else (G, A, gbuf, the FP32 copies in
// mixed precision, the projector products), each sized for the precision the
// product runs in.
Layout hx_layout(const Ham& h, int k, int prec) {
  const Basis& b = *h.basis;
  const size_t e = prec == CES_PREC_MIXED ? sizeof(float) : sizeof(double);
  Layout L;
  L.kp = round_up(k, kColPad);
  const size_t LL = size_t(b.L) * b.L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align256(off);
    const size_t at = off;
    off += bytes + 4096;
    return at;
  };
  L.kc64 = prec == CES_PREC_MIXED ? 0 : L.kp;   // an FP32 product only in mixed precision
  L.G = take(size_t(b.n_r) * LL * L.kp * e);
  L.A = take(size_t(b.n_r) * LL * L.kp * e);
  L.gbuf = take(size_t(b.n_r) * b.n_theta * (2 * size_t(b.L) - 1) * L.kp * e);
  if (prec == CES_PREC_MIXED) {
    L.F0 = take(size_t(f32_ld(b.d)) * L.kp * sizeof(float));
    L.F1 = take(size_t(f32_ld(b.d)) * L.kp * sizeof(float));
  }
  L.C = take(size_t(std::max(h.n_proj, 1)) * L.kp * e);
  L.Cpart = take(kb_partial_bytes(h.n_proj, k, b.d));
  L.Zkb = take(h.n_proj > 0 ? size_t(b.d) * L.kp * e : 0);
  L.total = align256(off);
  return L;
}

// -------------------------------------------------------------- one H step

template <typename T>
const DevTables<T>& tables(const Basis& b);
template <>
const DevTables<double>& tables<double>(const Basis& b) { return b.t64; }
template <>
const DevTables<float>& tables<float>(const Basis& b) { return b.t32; }

template <typename T>
const T* ab_of(const Ham& h);
template <>
const double* ab_of<double>(const Ham& h) { return h.ab64; }
template <>
const float* ab_of<float>(const Ham& h) { return h.ab32; }


// out = alpha * (H Yin - c Yin) + beta * Yold  (kinetic and projector terms
// included) for k columns with kp = k rounded up to 16.  Uses the G, A, gbuf
// and projector regions of the workspace.
template <typename T>
ces_status h_step_block(Ham& h, const Layout& ly, void* work, int k, const T* Yin, int64_t ldin,
                        const T* Yold, int64_t ldold, T* out, int64_t ldout, T alpha, T c,
                        T beta, hipStream_t s) {
  const Basis& b = *h.basis;
  const DevTables<T>& tb = tables<T>(b);
  T* G = Ptr<T>::at(work, ly.G);
  T* A = Ptr<T>::at(work, ly.A);
  T* C = Ptr<T>::at(work, ly.C);
  const int kp = static_cast<int>(round_up(k, kColPad));
  T* Zkb = nullptr;
  if (h.n_proj > 0) {
    // C = diag(h) P^T Yin (n_proj x kp, row-major), then Zkb = P C (d x k)
    const T* Pd = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)h.proj64 : (const void*)h.proj32);
    const T* hd = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)h.hproj64 : (const void*)h.hproj32);
    const int64_t ldp = sizeof(T) == 8 ? b.d : f32_ld(b.d);   // P row stride
    {
      StageTimer t(stage_id<T>(ST_KB_C), s);
      launch_kb_gemm<T>(Pd, b.d, ldp, Yin, ldin, hd, C, Ptr<T>::at(work, ly.Cpart), h.n_proj, k,
                        kp, s);
    }
    Zkb = Ptr<T>::at(work, ly.Zkb);
    StageTimer t(stage_id<T>(ST_KB_Z), s);
    launch_kb_apply<T>(Pd, b.d, ldp, C, Zkb, h.n_proj, k, kp, s);
  }
  T* gbuf = Ptr<T>::at(work, ly.gbuf);
  {
    StageTimer t(stage_id<T>(ST_RADIAL_INV), s);
    launch_radial_inverse<T>(b, tb, Yin, ldin, G, k, kp, s);
  }
  {
    StageTimer t(stage_id<T>(ST_LEG_SYNTH), s);
    launch_legendre_synth<T>(b, tb, G, gbuf, kp, s);
  }
  {
    StageTimer t(stage_id<T>(ST_PHI), s);
    launch_phi_stage<T>(b, ab_of<T>(h), gbuf, kp, s);
  }
  {
    StageTimer t(stage_id<T>(ST_LEG_ANALYSIS), s);
    launch_legendre_analysis<T>(b, tb, gbuf, A, kp, s);
  }
  {
    StageTimer t(stage_id<T>(ST_RADIAL_FWD), s);
    launch_radial_forward<T>(b, tb, A, Yin, ldin, Yold, ldold, out, ldout, alpha, c, beta, true,
                             Zkb, k, kp, s);
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

// h_step_block over column chunks of at most the columns the layout's G, A
// and gbuf hold in this precision (one chunk unless an FP64 product runs in a
// mixed-precision workspace).
template <typename T>
ces_status h_step(Ham& h, const Layout& ly, void* work, int k, const T* Yin, int64_t ldin,
                  const T* Yold, int64_t ldold, T* out, int64_t ldout, T alpha, T c, T beta,
                  hipStream_t s) {
  const int64_t cap = sizeof(T) == 8 ? ly.kc64 : ly.kp;
  if (cap < kColPad) return fail(CES_ERR_WORKSPACE, "workspace holds no product of this precision");
  for (int64_t c0 = 0; c0 < k; c0 += cap) {
    const int kc = static_cast<int>(std::min<int64_t>(cap, k - c0));
    CES_TRY(h_step_block<T>(h, ly, work, kc, Yin + c0 * ldin, ldin,
                            Yold ? Yold + c0 * ldold : nullptr, ldold, out + c0 * ldout, ldout,
                            alpha, c, beta, s));
  }
  return CES_OK;
}

template ces_status h_step<double>(Ham&, const Layout&, void*, int, const double*, int64_t,
                                   const double*, int64_t, double*, int64_t, double, double,
                                   double, hipStream_t);
template ces_status h_step<float>(Ham&, const Layout&, void*, int, const float*, int64_t,
                                  const float*, int64_t, float*, int64_t, float, float, float,
                                  hipStream_t);

// Y = H X on the regions of `ly` in `work` (FP64, or FP32 with the
// conversions of the mixed precision).
ces_status apply_H_impl(Ham& h, const Layout& ly, void* work, int k, const double* X,
                        int64_t ldx, double* Y, int64_t ldy, int prec, hipStream_t s) {
  const int64_t d = h.basis->d;
  if (prec == CES_PREC_FP64)
    return h_step<double>(h, ly, work, k, X, ldx, nullptr, 0, Y, ldy, 1.0, 0.0, 0.0, s);
  float* F0 = Ptr<float>::at(work, ly.F0);
  float* F1 = Ptr<float>::at(work, ly.F1);
  const int64_t ldf = f32_ld(d);
  launch_convert<double, float>(X, ldx, F0, ldf, d, k, s);
  CES_TRY(h_step<float>(h, ly, work, k, F0, ldf, nullptr, 0, F1, ldf, 1.0f, 0.0f, 0.0f, s));
  launch_convert<float, double>(F1, ldf, Y, ldy, d, k, s);
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status check_ham(ces_ham hh) {
  if (!hh) return fail(CES_ERR_INVALID_ARG, "null ham");
  int dev = 0;
  CES_HIP(hipGetDevice(&dev));
  if (dev != hh->h.basis->device) return fail(CES_ERR_INVALID_ARG, "ham lives on another device");
  return CES_OK;
}

// Largest block: (radial node, theta node, 32-column group) work items and
// the angular kernels' grid sizes stay below 2^31.
bool k_fits(const Basis& b, int k) {
  return int64_t(b.n_r) * b.n_theta * ((round_up(k, kColPad) + 31) / 32) < (int64_t(1) << 31);
}

ces_status check_block(const Ham& h, int k, const void* X, int64_t ldx, const char* what) {
  if (k < 1) return fail(CES_ERR_INVALID_ARG, std::string(what) + ": k must be >= 1");
  if (!k_fits(*h.basis, k)) return fail(CES_ERR_INVALID_ARG, std::string(what) + ": k too large");
  if (!X) return fail(CES_ERR_INVALID_ARG, std::string(what) + ": null block");
  if (ldx < h.basis->d) return fail(CES_ERR_INVALID_ARG, std::string(what) + ": ld < d");
  return CES_OK;
}

ces_status check_work(Ham& h, int k, int prec, void* work, size_t bytes, Layout& ly) {
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  ly = layout_for(h, k, prec);
  if (!work) return fail(CES_ERR_WORKSPACE, "null workspace");
  if (bytes < ly.total)
    return fail(CES_ERR_WORKSPACE, "workspace too small: need " + std::to_string(ly.total) +
                                       " bytes, got " + std::to_string(bytes));
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0)
    return fail(CES_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return CES_OK;
}

// Layout for a call whose products run in FP64: the FP64 layout when the
// workspace holds it, else the mixed-precision layout of the same k (FP64
// products then run in column chunks), so a workspace sized for a mixed-
// precision filter also serves the FP64 Rayleigh-Ritz and transforms.
ces_status check_work_fp64(Ham& h, int k, void* work, size_t bytes, Layout& ly) {
  const Layout l64 = layout_for(h, k, CES_PREC_FP64);
  if (bytes >= l64.total) return check_work(h, k, CES_PREC_FP64, work, bytes, ly);
  const Layout lmx = layout_for(h, k, CES_PREC_MIXED);
  if (bytes >= lmx.total) return check_work(h, k, CES_PREC_MIXED, work, bytes, ly);
  return fail(CES_ERR_WORKSPACE, "workspace too small: need " +
                                     std::to_string(std::min(l64.total, lmx.total)) +
                                     " bytes, got " + std::to_string(bytes));
}

// The layout for a call whose products run in `prec`: check_work_fp64 for
// FP64, the mixed layout otherwise.
ces_status check_work_for(Ham& h, int k, int prec, void* work, size_t bytes, Layout& ly) {
  if (prec == CES_PREC_FP64) return check_work_fp64(h, k, work, bytes, ly);
  return check_work(h, k, prec, work, bytes, ly);
}

// Chebyshev filter on an internal block; Y0 (ld ld0) in place.
template <typename T>
ces_status cheb_run(Ham& h, const Layout& ly, void* work, int k, T* Y0, int64_t ld0, T* Yb,
                    int64_t ldb, int degree, double a, double bnd, double a0, hipStream_t s,
                    T** result, int64_t* ldres) {
  const double e = (bnd - a) / 2.0, c = (bnd + a) / 2.0;
  const double sigma1 = e / (a0 - c);
  // step 1: Yb = (sigma1/e) (H Y0 - c Y0)
  CES_TRY(h_step<T>(h, ly, work, k, Y0, ld0, nullptr, 0, Yb, ldb, T(sigma1 / e), T(c), T(0), s));
  T* cur = Yb;
  int64_t ldc = ldb;
  T* prev = Y0;
  int64_t ldp = ld0;
  double sigma = sigma1;
  for (int j = 2; j <= degree; ++j) {
    const double sn = 1.0 / (2.0 / sigma1 - sigma);
    // Y_j = (2 sn / e)(H Y_{j-1} - c Y_{j-1}) - sigma sn Y_{j-2}, written over Y_{j-2}
    CES_TRY(h_step<T>(h, ly, work, k, cur, ldc, prev, ldp, prev, ldp, T(2.0 * sn / e), T(c),
                      T(-sigma * sn), s));
    std::swap(cur, prev);
    std::swap(ldc, ldp);
    sigma = sn;
  }
  *result = cur;
  *ldres = ldc;
  return CES_OK;
}

// Largest eigenvalue of a symmetric tridiagonal matrix (Sturm bisection).
double tridiag_max(const std::vector<double>& a, const std::vector<double>& bb) {
  const int n = static_cast<int>(a.size());
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double rad = (i > 0 ? std::fabs(bb[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(bb[i]) : 0.0);
    lo = std::min(lo, a[i] - rad);
    hi = std::max(hi, a[i] + rad);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double dd = 1.0;
    for (int i = 0; i < n; ++i) {
      dd = (a[i] - x) - (i > 0 ? bb[i - 1] * bb[i - 1] / dd : 0.0);
      if (dd == 0.0) dd = -1e-300;
      if (dd < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

// h_eval / h_res (host, may be null) receive the eigenvalues / residual norms
// in the same synchronisation that checks the factorisation.
ces_status rr_impl(Ham& h, const Layout& ly, void* work, int k, double* X, int64_t ldx, double* HX,
                   int64_t ldhx, double* eval, double* res, int hx_prec, hipStream_t s,
                   double* h_eval, double* h_res, int* h_path) {
  std::lock_guard<std::mutex> lock(h.mu);   // rocBLAS handle and host_stage
  return rr_locked(h, ly, work, k, X, ldx, HX, ldhx, eval, res, hx_prec, s, h_eval, h_res,
                   h_path);
}

ces_status rr_locked(Ham& h, const Layout& ly, void* work, int k, double* X, int64_t ldx,
                     double* HX, int64_t ldhx, double* eval, double* res, int hx_prec,
                     hipStream_t s, double* h_eval, double* h_res, int* h_path) {
  const Basis& b = *h.basis;
  const int64_t d = b.d;
  double* S1 = Ptr<double>::at(work, ly.S1);
  double* vec = Ptr<double>::at(work, ly.vec);
  double* dinv = vec;
  double* evals = eval ? eval : vec + k;   // eigenvalues straight into the caller's array
  double* Ework = vec + 2 * k;
  // info[0]: factorisation, info[1]: triangular inverse, info[2]: eigensolver
  rocblas_int* info = Ptr<rocblas_int>::at(work, ly.info);
  double* B1 = Ptr<double>::at(work, ly.B1);
  double* T2 = Ptr<double>::at(work, ly.B2);
  CES_BLAS(rocblas_set_stream(h.blas, s));
  CES_BLAS(rocblas_set_workspace(h.blas, Ptr<char>::at(work, ly.solver), ly.solver_bytes));
  const double one = 1.0, zero = 0.0;
  double* part = Ptr<double>::at(work, ly.part);
  const int64_t part_cap = int64_t(gram_chunks(d, k)) * k * k;   // doubles in the region
  const bool small = k <= kJacobiMax;
  // the one-workgroup Cholesky writes flags 0 and 1 and Jacobi flag 2 on every
  // call; the library path clears them first
  if (!small) CES_HIP(hipMemsetAsync(info, 0, 4 * sizeof(rocblas_int), s));
  // One Cholesky-QR pass: S = X^T X, D = diag(S)^{-1/2}, R^T R = D S D (+ shift I),
  // X <- X D R^{-1} (column scaling before factorising follows Section 3.1.1).
  // X is written only if the factorisation succeeded (checked on the device),
  // so a failed pass leaves X as it was.
  auto pass = [&](double shift) -> ces_status {
    launch_gram(X, ldx, X, ldx, S1, part, d, k, s, true);
    if (small) {
      launch_chol_inv(S1, k, shift, dinv, info, s);     // S1 <- D R^{-1}
      launch_block_apply(X, ldx, S1, k, d, info, s);     // X <- X D R^{-1}
      return CES_OK;
    }
    launch_scale_gram(S1, k, dinv, s);
    if (shift > 0) launch_add_diag(S1, k, shift, s);
    CES_BLAS(rocsolver_dpotrf(h.blas, rocblas_fill_upper, k, S1, k, info));
    // the same failure test as the one-workgroup factorisation: a pivot of
    // the unit-diagonal D S D at rounding level marks a dependent column
    launch_check_pivots(S1, k, info, s);
    launch_zero_lower(S1, k, s);   // potrf leaves the Gram entries below the diagonal
    CES_BLAS(rocsolver_dtrtri(h.blas, rocblas_fill_upper, rocblas_diagonal_non_unit, k, S1, k,
                              info + 1));
    launch_scale_rows_k(S1, k, dinv, s);                // S1 <- D R^{-1}
    CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                           static_cast<int>(d), k, k, &one, X, static_cast<int>(ldx), S1, k, &zero,
                           T2, static_cast<int>(d)));
    launch_copy2d_if(T2, d, X, ldx, d, k, info, s);
    return CES_OK;
  };
  // read-backs go through the handle's pinned stage: info flags at offset 0,
  // eigenvalues at 2, residual norms at 2 + k, behind one synchronisation
  auto read_info = [&](rocblas_int* h3) -> ces_status {
    // a launch that never started leaves its status flag as an earlier call
    // wrote it: report it before the flags are trusted
    CES_HIP(hipGetLastError());
    CES_TRY(stage_read(h, 0, info, 3 * sizeof(rocblas_int), s));
    CES_HIP(hipStreamSynchronize(s));
    std::memcpy(h3, h.host_stage, 3 * sizeof(rocblas_int));
    return CES_OK;
  };
  // Rayleigh-Ritz on the (orthonormal) block; X and HX are written only if
  // the Cholesky-QR before it succeeded.
  auto rayleigh = [&]() -> ces_status {
    double* HQ = HX ? HX : B1;
    const int64_t ldhq = HX ? ldhx : d;
    if (hx_prec == CES_PREC_FP64) {
      CES_TRY(h_step<double>(h, ly, work, k, X, ldx, nullptr, 0, HQ, ldhq, 1.0, 0.0, 0.0, s));
    } else {
      float* F0 = Ptr<float>::at(work, ly.F0);
      float* F1 = Ptr<float>::at(work, ly.F1);
      const int64_t ldf = f32_ld(d);
      launch_convert<double, float>(X, ldx, F0, ldf, d, k, s);
      CES_TRY(h_step<float>(h, ly, work, k, F0, ldf, nullptr, 0, F1, ldf, 1.0f, 0.0f, 0.0f, s));
      launch_convert<float, double>(F1, ldf, HQ, ldhq, d, k, s);
    }
    // Hs = Q^T H Q, eigen-decomposition (ascending)
    launch_gram(X, ldx, HQ, ldhq, S1, part, d, k, s, true);
    if (small) {   // one-workgroup Jacobi, then X <- Q S, HQ <- HQ S in place
      launch_jacobi_eig(S1, k, evals, info + 2, s);
      launch_block_rotate(X, ldx, HQ, ldhq, S1, k, d, info, evals, res, part, part_cap, s);
    } else {
      CES_BLAS(rocsolver_dsyevd(h.blas, rocblas_evect_original, rocblas_fill_upper, k, S1, k,
                                evals, Ework, info + 2));
      // X <- Q S ; HQ <- HQ S through T2
      CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                             static_cast<int>(d), k, k, &one, X, static_cast<int>(ldx), S1, k,
                             &zero, T2, static_cast<int>(d)));
      launch_copy2d_if(T2, d, X, ldx, d, k, info, s);
      CES_BLAS(rocblas_dgemm(h.blas, rocblas_operation_none, rocblas_operation_none,
                             static_cast<int>(d), k, k, &one, HQ, static_cast<int>(ldhq), S1, k,
                             &zero, T2, static_cast<int>(d)));
      launch_copy2d_if(T2, d, HQ, ldhq, d, k, info, s);
      launch_residuals(HQ, ldhq, X, ldx, evals, res, d, k, part, part_cap, s);
    }
    return CES_OK;
  };
  auto finish = [&](rocblas_int* h3) -> ces_status {
    CES_TRY(host_stage(h, 2 + 2 * size_t(k)));
    if (h_eval) CES_TRY(stage_read(h, 2, evals, size_t(k) * 8, s));
    if (h_res) CES_TRY(stage_read(h, 2 + size_t(k), res, size_t(k) * 8, s));
    CES_TRY(read_info(h3));
    if (h_eval) std::memcpy(h_eval, h.host_stage + 2, size_t(k) * 8);
    if (h_res) std::memcpy(h_res, h.host_stage + 2 + k, size_t(k) * 8);
    return CES_OK;
  };
  if (h_path) *h_path = 0;
  CES_TRY(pass(0.0));
  CES_TRY(rayleigh());
  rocblas_int h3[3] = {0, 0, 0};
  CES_TRY(finish(h3));
  if (h3[0] != 0 || h3[1] != 0) {
    if (h_path) *h_path = 1;
    // The plain pass failed and X is unchanged: shifted Cholesky-QR (shift ~
    // 11 (d k + k(k+1)) u ||D S D||), then two plain passes restore
    // orthonormality (shifted CholeskyQR3); then Rayleigh-Ritz again.
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * (double(d) * k + double(k) * (k + 1)) * u * k;
    CES_HIP(hipMemsetAsync(info, 0, 4 * sizeof(rocblas_int), s));
    CES_TRY(pass(shift));
    CES_TRY(read_info(h3));
    if (h3[0] != 0 || h3[1] != 0) return fail(CES_ERR_NOT_POSITIVE_DEFINITE, "shifted Cholesky-QR failed");
    for (int rep = 0; rep < 2; ++rep) {
      CES_TRY(pass(0.0));
      CES_TRY(read_info(h3));
      if (h3[0] != 0 || h3[1] != 0)
        return fail(CES_ERR_NOT_POSITIVE_DEFINITE, "Cholesky-QR after the shifted pass failed");
    }
    CES_TRY(rayleigh());
    CES_TRY(finish(h3));
  }
  if (h3[2] != 0) return fail(CES_ERR_EIGENSOLVER, "projected eigenproblem did not converge");
  return CES_OK;
}

}  // namespace ces

using namespace ces;

extern "C" {

const char* ces_status_string(ces_status s) {
  switch (s) {
    case CES_OK: return "CES_OK";
    case CES_ERR_INVALID_ARG: return "CES_ERR_INVALID_ARG";
    case CES_ERR_DEVICE: return "CES_ERR_DEVICE";
    case CES_ERR_ALLOC: return "CES_ERR_ALLOC";
    case CES_ERR_WORKSPACE: return "CES_ERR_WORKSPACE";
    case CES_ERR_NOT_POSITIVE_DEFINITE: return "CES_ERR_NOT_POSITIVE_DEFINITE";
    case CES_ERR_EIGENSOLVER: return "CES_ERR_EIGENSOLVER";
  }
  return "unknown ces_status";
}

const char* ces_last_error(void) { return g_err.c_str(); }

ces_status ces_profile_enable(int on, int max_records) {
  for (auto& e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof = Profiler();
  if (!on) return CES_OK;
  if (max_records < 1 || max_records > (1 << 20))
    return fail(CES_ERR_INVALID_ARG, "max_records must be in [1, 2^20]");
  g_prof.ev.resize(2 * size_t(max_records));
  for (auto& e : g_prof.ev) CES_HIP(hipEventCreate(&e));
  g_prof.stage.reserve(max_records);
  g_prof.on = true;
  return CES_OK;
}

ces_status ces_profile_read(int n_stages, double* h_ms, int64_t* h_count) {
  if (n_stages < 0 || n_stages > kStages || (n_stages > 0 && (!h_ms || !h_count)))
    return fail(CES_ERR_INVALID_ARG, "bad profile_read arguments");
  for (size_t r = 0; r < g_prof.stage.size(); ++r) {
    CES_HIP(hipEventSynchronize(g_prof.ev[2 * r + 1]));
    float ms = 0.f;
    CES_HIP(hipEventElapsedTime(&ms, g_prof.ev[2 * r], g_prof.ev[2 * r + 1]));
    g_prof.ms[g_prof.stage[r]] += ms;
    g_prof.count[g_prof.stage[r]] += 1;
  }
  g_prof.stage.clear();
  for (int i = 0; i < n_stages; ++i) {
    h_ms[i] = g_prof.ms[i];
    h_count[i] = g_prof.count[i];
  }
  return CES_OK;
}

namespace {
// Shared by the uniform and the cutoff constructors; e_cut <= 0 keeps every
// radial function (N_l = N).
ces_status basis_create(int lmax, int n_rad, double R, int n_r, int n_theta, int n_phi,
                        int radial_rule, double e_cut, ces_basis* out) {
  if (!out) return fail(CES_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (lmax < 0 || n_rad < 1 || !(R > 0) || n_r < 1 || n_theta < 1)
    return fail(CES_ERR_INVALID_ARG, "basis sizes must be positive");
  if (n_phi < 2 * lmax + 1) return fail(CES_ERR_INVALID_ARG, "n_phi must be >= 2*lmax+1");
  if (radial_rule != CES_RADIAL_GAUSS_JACOBI_R2 && radial_rule != CES_RADIAL_GAUSS_LEGENDRE)
    return fail(CES_ERR_INVALID_ARG, "unknown radial rule");
  // kernel tile limits: L - m <= 96 and 2L-1 <= 192 (angular), N <= 192 and
  // n_r <= 256 (radial), n_phi <= 2048 (density synthesis)
  if (lmax > 95 || n_rad > 192 || n_r > 256 || n_theta > 4096 || n_phi > 2048)
    return fail(CES_ERR_INVALID_ARG, "basis sizes beyond supported limits "
                                     "(lmax <= 95, n_rad <= 192, n_r <= 256, n_phi <= 2048)");
  ces_basis_s* bb = new (std::nothrow) ces_basis_s();
  if (!bb) return fail(CES_ERR_ALLOC, "out of host memory");
  Basis& b = bb->b;
  b.L = lmax + 1;
  b.N = n_rad;
  b.R = R;
  b.n_r = n_r;
  b.n_theta = n_theta;
  b.n_phi = n_phi;
  b.rule = radial_rule;
  b.n_grid = int64_t(n_r) * n_theta * n_phi;
  try {
    build_host_tables(b);
  } catch (const std::exception& e) {
    delete bb;
    return fail(CES_ERR_INVALID_ARG, e.what());
  }
  // coefficient layout: N_l = #{n < N : Lambda_ln / 2 <= e_cut} (all N without
  // a cutoff); Lambda grows with n, so the kept functions are n < N_l
  b.e_cut = e_cut > 0 ? e_cut : 0.0;
  b.Nl.assign(b.L, b.N);
  b.off.assign(b.L, 0);
  int64_t d = 0;
  for (int l = 0; l < b.L; ++l) {
    if (e_cut > 0) {
      int cnt = 0;
      for (int n = 0; n < b.N; ++n) {
        const double kk = b.zeros[size_t(l) * b.N + n] / b.R;
        if (0.5 * kk * kk <= e_cut) ++cnt;
      }
      b.Nl[l] = cnt;
    }
    b.off[l] = d;
    d += int64_t(2 * l + 1) * b.Nl[l];
  }
  if (b.Nl[0] < 1) {
    delete bb;
    return fail(CES_ERR_INVALID_ARG, "the kinetic-energy cutoff keeps no radial function");
  }
  b.d = d;
  *out = bb;
  return CES_OK;
}
}  // namespace

ces_status ces_basis_create(int lmax, int n_rad, double R, int n_r, int n_theta, int n_phi,
                            int radial_rule, ces_basis* out) {
  return basis_create(lmax, n_rad, R, n_r, n_theta, n_phi, radial_rule, 0.0, out);
}

ces_status ces_basis_create_ke(int lmax, int n_rad, double R, int n_r, int n_theta, int n_phi,
                               int radial_rule, double e_cut, ces_basis* out) {
  if (!(e_cut > 0) || !std::isfinite(e_cut))
    return fail(CES_ERR_INVALID_ARG, "the kinetic-energy cutoff must be finite and > 0");
  return basis_create(lmax, n_rad, R, n_r, n_theta, n_phi, radial_rule, e_cut, out);
}

ces_status ces_basis_radial_counts(ces_basis bb, int* h_nl) {
  if (!bb || !h_nl) return fail(CES_ERR_INVALID_ARG, "null argument");
  std::memcpy(h_nl, bb->b.Nl.data(), bb->b.Nl.size() * sizeof(int));
  return CES_OK;
}

ces_status ces_basis_destroy(ces_basis bb) {
  if (!bb) return CES_OK;
  if (bb->b.dev_block) (void)hipFree(bb->b.dev_block);
  delete bb;
  return CES_OK;
}

ces_status ces_basis_info(ces_basis bb, int64_t* d, int64_t* n_grid) {
  if (!bb) return fail(CES_ERR_INVALID_ARG, "null basis");
  if (d) *d = bb->b.d;
  if (n_grid) *n_grid = bb->b.n_grid;
  return CES_OK;
}

namespace {
// Validation shared by the two coefficient maps: sizes, 16-byte alignment of
// the interleaved complex blocks, and no overlap between input and output.
ces_status check_coeff_map(ces_basis bb, int k, const double* in, int64_t ldi, const double* out,
                           int64_t ldo) {
  if (!bb) return fail(CES_ERR_INVALID_ARG, "null basis");
  const int64_t d = bb->b.d;
  if (k < 1) return fail(CES_ERR_INVALID_ARG, "k must be >= 1");
  if (!in || !out) return fail(CES_ERR_INVALID_ARG, "null coefficient block");
  if (ldi < d || ldo < d) return fail(CES_ERR_INVALID_ARG, "leading dimension below d");
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15)
    return fail(CES_ERR_INVALID_ARG, "complex blocks must be 16-byte aligned");
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(in), b0 = reinterpret_cast<uintptr_t>(out);
  const uintptr_t a1 = a0 + uintptr_t(16) * uintptr_t((k - 1) * ldi + d);
  const uintptr_t b1 = b0 + uintptr_t(16) * uintptr_t((k - 1) * ldo + d);
  if (a0 < b1 && b0 < a1) return fail(CES_ERR_INVALID_ARG, "input and output blocks overlap");
  return CES_OK;
}
}  // namespace

ces_status ces_coeffs_complex_to_real(ces_basis bb, int k, const double* d_f, int64_t ldf,
                                      double* d_s, int64_t lds, void* stream) {
  CES_TRY(check_coeff_map(bb, k, d_f, ldf, d_s, lds));
  CES_TRY(ensure_device(bb->b));   // the coefficient layout table
  launch_coeffs_c2r(bb->b, d_f, ldf, d_s, lds, k, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_coeffs_real_to_complex(ces_basis bb, int k, const double* d_s, int64_t lds,
                                      double* d_f, int64_t ldf, void* stream) {
  CES_TRY(check_coeff_map(bb, k, d_s, lds, d_f, ldf));
  CES_TRY(ensure_device(bb->b));   // the coefficient layout table
  launch_coeffs_r2c(bb->b, d_s, lds, d_f, ldf, k, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_basis_grid(ces_basis bb, double* h_r, double* h_wr, double* h_theta,
                          double* h_wtheta, double* h_phi) {
  if (!bb) return fail(CES_ERR_INVALID_ARG, "null basis");
  const Basis& b = bb->b;
  if (h_r) std::memcpy(h_r, b.r.data(), b.r.size() * 8);
  if (h_wr) std::memcpy(h_wr, b.wr.data(), b.wr.size() * 8);
  if (h_theta) std::memcpy(h_theta, b.theta.data(), b.theta.size() * 8);
  if (h_wtheta) std::memcpy(h_wtheta, b.wt.data(), b.wt.size() * 8);
  if (h_phi) std::memcpy(h_phi, b.phi.data(), b.phi.size() * 8);
  return CES_OK;
}

ces_status ces_basis_tables(ces_basis bb, double* h_zeros, double* h_radial, double* h_legendre) {
  if (!bb) return fail(CES_ERR_INVALID_ARG, "null basis");
  const Basis& b = bb->b;
  if (h_zeros) std::memcpy(h_zeros, b.zeros.data(), b.zeros.size() * 8);
  if (h_radial) std::memcpy(h_radial, b.radial.data(), b.radial.size() * 8);
  if (h_legendre) std::memcpy(h_legendre, b.legendre.data(), b.legendre.size() * 8);
  return CES_OK;
}

ces_status ces_ham_create(ces_basis bb, const double* d_veff, int n_proj, const double* d_proj,
                          const double* h_proj_energy, void* stream, ces_ham* out) {
  if (!out) return fail(CES_ERR_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!bb || !d_veff) return fail(CES_ERR_INVALID_ARG, "null basis or V_eff");
  if (n_proj < 0 || (n_proj > 0 && (!d_proj || !h_proj_energy)))
    return fail(CES_ERR_INVALID_ARG, "bad projector arguments");
  Basis& b = bb->b;
  CES_TRY(ensure_device(b));
  hipStream_t s = static_cast<hipStream_t>(stream);
  ces_ham_s* hh = new (std::nothrow) ces_ham_s();
  if (!hh) return fail(CES_ERR_ALLOC, "out of host memory");
  Ham& h = hh->h;
  h.basis = &b;
  h.n_proj = n_proj;
  const size_t S = 2 * size_t(b.L) - 1;
  const size_t nab = size_t(b.n_r) * b.n_theta * 2 * S;
  const size_t sz_v = align256(size_t(b.n_grid) * 8), sz_ab64 = align256(nab * 8),
               sz_ab32 = align256(nab * 4), sz_p64 = align256(size_t(b.d) * n_proj * 8),
               sz_p32 = align256(size_t(f32_ld(b.d)) * n_proj * 4), sz_h = align256(size_t(n_proj) * 8) + align256(size_t(n_proj) * 4);
  void* blk = nullptr;
  if (hipMalloc(&blk, sz_v + sz_ab64 + sz_ab32 + sz_p64 + sz_p32 + sz_h) != hipSuccess) {
    delete hh;
    return fail(CES_ERR_ALLOC, "hipMalloc of hamiltonian storage failed");
  }
  h.dev_block = blk;
  char* p = static_cast<char*>(blk);
  h.veff = reinterpret_cast<double*>(p);
  h.ab64 = reinterpret_cast<double*>(p + sz_v);
  h.ab32 = reinterpret_cast<float*>(p + sz_v + sz_ab64);
  char* pp = p + sz_v + sz_ab64 + sz_ab32;
  if (n_proj > 0) {
    h.proj64 = reinterpret_cast<double*>(pp);
    h.proj32 = reinterpret_cast<float*>(pp + sz_p64);
    h.hproj64 = reinterpret_cast<double*>(pp + sz_p64 + sz_p32);
    h.hproj32 = reinterpret_cast<float*>(pp + sz_p64 + sz_p32 + align256(size_t(n_proj) * 8));
  }
  auto cleanup = [&](ces_status st) {
    if (h.blas) rocblas_destroy_handle(h.blas);
    if (h.host_stage) (void)hipHostFree(h.host_stage);
    (void)hipFree(blk);
    delete hh;
    return st;
  };
  if (rocblas_create_handle(&h.blas) != rocblas_status_success)
    return cleanup(fail(CES_ERR_DEVICE, "rocblas_create_handle failed"));
  // the read-back buffer for every block size Rayleigh-Ritz accepts on this
  // basis (flags, eigenvalues and residual norms), so no later call allocates
  if (const ces_status st = host_stage(h, 2 + 2 * size_t(std::min<int64_t>(b.d, kRRMax)));
      st != CES_OK)
    return cleanup(st);
  if (hipMemcpyAsync(h.veff, d_veff, size_t(b.n_grid) * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return cleanup(fail(CES_ERR_DEVICE, "copy of V_eff failed"));
  launch_veff_fourier(b, h.veff, h.ab64, h.ab32, s);
  if (n_proj > 0) {
    if (hipMemcpyAsync(h.proj64, d_proj, size_t(b.d) * n_proj * 8, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return cleanup(fail(CES_ERR_DEVICE, "copy of projectors failed"));
    // FP32 rows padded to f32_ld(d) with zeros
    if (hipMemsetAsync(h.proj32, 0, size_t(f32_ld(b.d)) * n_proj * 4, s) != hipSuccess)
      return cleanup(fail(CES_ERR_DEVICE, "clearing the FP32 projectors failed"));
    launch_convert<double, float>(h.proj64, b.d, h.proj32, f32_ld(b.d), b.d, n_proj, s);
    std::vector<float> e32(n_proj);
    for (int q = 0; q < n_proj; ++q) e32[q] = static_cast<float>(h_proj_energy[q]);
    if (hipMemcpyAsync(h.hproj64, h_proj_energy, size_t(n_proj) * 8, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(h.hproj32, e32.data(), size_t(n_proj) * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess)
      return cleanup(fail(CES_ERR_DEVICE, "copy of projector energies failed"));
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return cleanup(fail(CES_ERR_DEVICE, "hamiltonian setup failed on the device"));
  *out = hh;
  return CES_OK;
}

ces_status ces_ham_set_veff(ces_ham hh, const double* d_veff, void* stream) {
  CES_TRY(check_ham(hh));
  if (!d_veff) return fail(CES_ERR_INVALID_ARG, "null V_eff");
  Ham& h = hh->h;
  hipStream_t s = static_cast<hipStream_t>(stream);
  CES_HIP(hipMemcpyAsync(h.veff, d_veff, size_t(h.basis->n_grid) * 8, hipMemcpyDeviceToDevice, s));
  launch_veff_fourier(*h.basis, h.veff, h.ab64, h.ab32, s);
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_ham_destroy(ces_ham hh) {
  if (!hh) return CES_OK;
  if (hh->h.blas) rocblas_destroy_handle(hh->h.blas);
  if (hh->h.dev_block) (void)hipFree(hh->h.dev_block);
  if (hh->h.host_stage) (void)hipHostFree(hh->h.host_stage);
  delete hh;
  return CES_OK;
}

ces_status ces_workspace_size(ces_ham hh, int k, int prec, size_t* bytes) {
  if (!hh || !bytes) return fail(CES_ERR_INVALID_ARG, "null argument");
  if (k < 1) return fail(CES_ERR_INVALID_ARG, "k must be >= 1");
  if (!k_fits(*hh->h.basis, k)) return fail(CES_ERR_INVALID_ARG, "k too large");
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  *bytes = layout_for(hh->h, k, prec).total;
  return CES_OK;
}

ces_status ces_apply_H(ces_ham hh, int k, const double* d_X, int64_t ldx, double* d_Y,
                       int64_t ldy, int prec, void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  CES_TRY(check_block(h, k, d_Y, ldy, "Y"));
  Layout ly;
  CES_TRY(check_work_for(h, k, prec, d_work, work_bytes, ly));
  return apply_H_impl(h, ly, d_work, k, d_X, ldx, d_Y, ldy, prec,
                      static_cast<hipStream_t>(stream));
}

ces_status ces_cheb_filter(ces_ham hh, int k, double* d_X, int64_t ldx, int degree, double a,
                           double b, double a0, int prec, void* d_work, size_t work_bytes,
                           void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (degree < 1) return fail(CES_ERR_INVALID_ARG, "degree must be >= 1");
  if (!(a < b) || !(a0 < a) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(a0))
    return fail(CES_ERR_INVALID_ARG, "filter bounds must satisfy a0 < a < b");
  Layout ly;
  CES_TRY(check_work_for(h, k, prec, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t d = h.basis->d;
  if (prec == CES_PREC_FP64) {
    double* B1 = Ptr<double>::at(d_work, ly.B1);
    double* res = nullptr;
    int64_t ldr = 0;
    CES_TRY(cheb_run<double>(h, ly, d_work, k, d_X, ldx, B1, d, degree, a, b, a0, s, &res, &ldr));
    if (res != d_X) launch_copy2d(res, ldr, d_X, ldx, d, k, s);
  } else {
    float* F0 = Ptr<float>::at(d_work, ly.F0);
    float* F1 = Ptr<float>::at(d_work, ly.F1);
    const int64_t ldf = f32_ld(d);
    launch_convert<double, float>(d_X, ldx, F0, ldf, d, k, s);
    float* res = nullptr;
    int64_t ldr = 0;
    CES_TRY(cheb_run<float>(h, ly, d_work, k, F0, ldf, F1, ldf, degree, a, b, a0, s, &res, &ldr));
    launch_convert<float, double>(res, ldr, d_X, ldx, d, k, s);
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_rayleigh_ritz(ces_ham hh, int k, double* d_X, int64_t ldx, double* d_HX,
                             double* d_eval, double* d_resnorm, double* h_eval,
                             int* h_orth_path, int hx_prec, void* d_work, size_t work_bytes,
                             void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_eval || !d_resnorm) return fail(CES_ERR_INVALID_ARG, "null eigenvalue/residual output");
  if (k > h.basis->d) return fail(CES_ERR_INVALID_ARG, "k exceeds the basis size");
  if (k > kRRMax) return fail(CES_ERR_INVALID_ARG, "k above the Rayleigh-Ritz limit");
  Layout ly;
  CES_TRY(check_work_for(h, k, hx_prec, d_work, work_bytes, ly));
  return rr_impl(h, ly, d_work, k, d_X, ldx, d_HX, ldx, d_eval, d_resnorm, hx_prec,
                 static_cast<hipStream_t>(stream), h_eval, nullptr, h_orth_path);
}

ces_status ces_lanczos_bound(ces_ham hh, const double* d_v0, int steps, double* h_bound,
                             void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  if (!d_v0 || !h_bound || steps < 1) return fail(CES_ERR_INVALID_ARG, "bad Lanczos arguments");
  const int64_t d = h.basis->d;
  if (steps > d) steps = static_cast<int>(d);
  Layout ly;
  CES_TRY(check_work(h, 1, CES_PREC_FP64, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* v = Ptr<double>::at(d_work, ly.V3);
  double* vp = v + d;
  double* w = v + 2 * d;
  double* sc = Ptr<double>::at(d_work, ly.vec);
  std::lock_guard<std::mutex> lock(h.mu);   // host_stage
  CES_HIP(hipMemsetAsync(vp, 0, size_t(d) * 8, s));
  launch_dot(d_v0, d_v0, d, sc, sc + 64, s);
  CES_TRY(stage_read(h, 0, sc, 8, s));
  CES_HIP(hipStreamSynchronize(s));
  const double nrm2 = h.host_stage[0];
  if (!(nrm2 > 0) || !std::isfinite(nrm2)) return fail(CES_ERR_INVALID_ARG, "bad Lanczos start vector");
  launch_axpby(1.0 / std::sqrt(nrm2), d_v0, 0.0, v, d, s);
  std::vector<double> al, be;
  double beta = 0.0;
  for (int j = 0; j < steps; ++j) {
    CES_TRY(h_step<double>(h, ly, d_work, 1, v, d, nullptr, 0, w, d, 1.0, 0.0, 0.0, s));
    launch_dot(v, w, d, sc, sc + 64, s);
    CES_TRY(stage_read(h, 0, sc, 8, s));
    CES_HIP(hipStreamSynchronize(s));
    const double alpha = h.host_stage[0];
    launch_axpby(-alpha, v, 1.0, w, d, s);
    if (j > 0) launch_axpby(-beta, vp, 1.0, w, d, s);
    launch_dot(w, w, d, sc, sc + 64, s);
    CES_TRY(stage_read(h, 0, sc, 8, s));
    CES_HIP(hipStreamSynchronize(s));
    const double b2 = h.host_stage[0];
    beta = std::sqrt(std::max(b2, 0.0));
    al.push_back(alpha);
    if (j + 1 < steps) {
      be.push_back(beta);
      if (!(beta > 0)) break;  // invariant subspace found
      launch_copy2d(v, d, vp, d, d, 1, s);
      launch_axpby(1.0 / beta, w, 0.0, v, d, s);
    }
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  const double ub = tridiag_max(al, be) + beta;
  *h_bound = ub > 0 ? ub * 1.01 : ub / 1.01;
  return CES_OK;
}

ces_status ces_chefsi(ces_ham hh, int k, double* d_X, int64_t ldx, int degree, double b,
                      int n_check, int max_iter, int fixed_iter, double res_tol,
                      double dtheta_tol, int prec, double* d_eval, double* d_resnorm,
                      int* h_iters, void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_eval || !d_resnorm || !h_iters) return fail(CES_ERR_INVALID_ARG, "null output");
  if (degree < 1 || n_check < 1 || n_check > k || max_iter < 1 || fixed_iter < 0)
    return fail(CES_ERR_INVALID_ARG, "bad iteration parameters");
  if (k > h.basis->d) return fail(CES_ERR_INVALID_ARG, "k exceeds the basis size");
  if (k > kRRMax) return fail(CES_ERR_INVALID_ARG, "k above the Rayleigh-Ritz limit");
  Layout ly;
  CES_TRY(check_work_for(h, k, prec, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t d = h.basis->d;
  std::vector<double> theta(k), theta_old(k), res(k);
  CES_TRY(rr_impl(h, ly, d_work, k, d_X, ldx, nullptr, ldx, d_eval, d_resnorm, CES_PREC_FP64, s,
                  theta.data(), res.data(), nullptr));
  int it = 0;
  while (true) {
    ++it;
    const double a0 = theta[0], a = theta[k - 1];
    if (!(a < b)) return fail(CES_ERR_INVALID_ARG, "upper bound b is below the Ritz values");
    const double a0u = (a0 < a) ? a0 : a - 1e-6 * std::max(1.0, std::fabs(a));
    if (prec == CES_PREC_FP64) {
      double* B1 = Ptr<double>::at(d_work, ly.B1);
      double* out = nullptr;
      int64_t ldr = 0;
      CES_TRY(cheb_run<double>(h, ly, d_work, k, d_X, ldx, B1, d, degree, a, b, a0u, s, &out, &ldr));
      if (out != d_X) launch_copy2d(out, ldr, d_X, ldx, d, k, s);
    } else {
      float* F0 = Ptr<float>::at(d_work, ly.F0);
      float* F1 = Ptr<float>::at(d_work, ly.F1);
      const int64_t ldf = f32_ld(d);
      launch_convert<double, float>(d_X, ldx, F0, ldf, d, k, s);
      float* out = nullptr;
      int64_t ldr = 0;
      CES_TRY(cheb_run<float>(h, ly, d_work, k, F0, ldf, F1, ldf, degree, a, b, a0u, s, &out,
                              &ldr));
      launch_convert<float, double>(out, ldr, d_X, ldx, d, k, s);
    }
    theta_old = theta;
    CES_TRY(rr_impl(h, ly, d_work, k, d_X, ldx, nullptr, ldx, d_eval, d_resnorm, CES_PREC_FP64, s,
                    theta.data(), res.data(), nullptr));
    if (fixed_iter > 0) {
      if (it >= fixed_iter) break;
      continue;
    }
    bool ok = true;
    for (int i = 0; i < n_check; ++i) {
      if (!(res[i] <= res_tol * std::max(1.0, std::fabs(theta[i])))) ok = false;
      if (!(std::fabs(theta[i] - theta_old[i]) < dtheta_tol)) ok = false;
    }
    if (ok || it >= max_iter) break;
  }
  *h_iters = it;
  return CES_OK;
}

ces_status ces_to_grid(ces_ham hh, int k, const double* d_X, int64_t ldx, double* d_f,
                       void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_f) return fail(CES_ERR_INVALID_ARG, "null grid output");
  Layout ly;
  CES_TRY(check_work_fp64(h, k, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Basis& b = *h.basis;
  double* G = Ptr<double>::at(d_work, ly.G);
  double* gbuf = Ptr<double>::at(d_work, ly.gbuf);
  for (int64_t c0 = 0; c0 < k; c0 += ly.kc64) {   // column chunks the regions hold
    const int kc = static_cast<int>(std::min<int64_t>(ly.kc64, k - c0));
    const int kp = static_cast<int>(round_up(kc, kColPad));
    launch_radial_inverse<double>(b, b.t64, d_X + c0 * ldx, ldx, G, kc, kp, s);
    launch_legendre_synth<double>(b, b.t64, G, gbuf, kp, s);
    launch_phi_synthesis_cols(b, gbuf, kc, kp, d_f + c0 * b.n_grid, b.n_grid, s);
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_from_grid(ces_ham hh, int k, const double* d_f, double* d_X, int64_t ldx,
                         void* d_work, size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_f) return fail(CES_ERR_INVALID_ARG, "null grid input");
  Layout ly;
  CES_TRY(check_work_fp64(h, k, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Basis& b = *h.basis;
  double* A = Ptr<double>::at(d_work, ly.A);
  double* gh = Ptr<double>::at(d_work, ly.gbuf);
  for (int64_t c0 = 0; c0 < k; c0 += ly.kc64) {   // column chunks the regions hold
    const int kc = static_cast<int>(std::min<int64_t>(ly.kc64, k - c0));
    const int kp = static_cast<int>(round_up(kc, kColPad));
    launch_phi_analysis_cols(b, d_f + c0 * b.n_grid, b.n_grid, kc, kp, gh, s);
    launch_legendre_analysis<double>(b, b.t64, gh, A, kp, s);
    launch_radial_forward<double>(b, b.t64, A, nullptr, 0, nullptr, 0, d_X + c0 * ldx, ldx, 1.0,
                                  0.0, 0.0, false, nullptr, kc, kp, s);
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_density(ces_ham hh, int k, const double* d_X, int64_t ldx, const double* d_occ,
                       double* d_rho_grid, double* d_rho_coef, int prec, void* d_work,
                       size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_occ || !d_rho_grid) return fail(CES_ERR_INVALID_ARG, "null occupations or density");
  Layout ly;
  CES_TRY(check_work(h, k, prec, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Basis& b = *h.basis;
  const int kp = static_cast<int>(ly.kp);
  // psi through the H*X transforms up to the Legendre synthesis, then the phi
  // synthesis with the squared, occupation-weighted sum over orbitals
  if (prec == CES_PREC_FP64) {
    double* G = Ptr<double>::at(d_work, ly.G);
    double* gbuf = Ptr<double>::at(d_work, ly.gbuf);
    launch_radial_inverse<double>(b, b.t64, d_X, ldx, G, k, kp, s);
    launch_legendre_synth<double>(b, b.t64, G, gbuf, kp, s);
    launch_density_phi<double>(b, gbuf, d_occ, d_rho_grid, k, kp, s);
  } else {
    float* F0 = Ptr<float>::at(d_work, ly.F0);
    float* G = Ptr<float>::at(d_work, ly.G);
    float* gbuf = Ptr<float>::at(d_work, ly.gbuf);
    launch_convert<double, float>(d_X, ldx, F0, f32_ld(b.d), b.d, k, s);
    launch_radial_inverse<float>(b, b.t32, F0, f32_ld(b.d), G, k, kp, s);
    launch_legendre_synth<float>(b, b.t32, G, gbuf, kp, s);
    launch_density_phi<float>(b, gbuf, d_occ, d_rho_grid, k, kp, s);
  }
  if (d_rho_coef) {   // tau: the forward transform of rho as one 16-column block
    double* gh = Ptr<double>::at(d_work, ly.gbuf);
    double* A = Ptr<double>::at(d_work, ly.A);
    launch_phi_analysis_one(b, d_rho_grid, gh, s);
    launch_legendre_analysis<double>(b, b.t64, gh, A, kColPad, s);
    launch_radial_forward<double>(b, b.t64, A, nullptr, 0, nullptr, 0, d_rho_coef, b.d, 1.0, 0.0,
                                  0.0, false, nullptr, 1, kColPad, s);
  }
  CES_HIP(hipGetLastError());
  return CES_OK;
}

}  // extern "C"
