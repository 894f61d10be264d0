// Radial stages of H*X on MFMA (gfx950).
//
// radial_inverse (eq. G_lmr):  G[r][lm][i] = sum_n R_ln(r) X[lm*N + n][i]
//   per (l, m): M = n_r, K = N, N = k.  The X tile (N x 32 columns) is
//   staged through LDS so that the global loads run down the contiguous
//   coefficient index n.  Index math is hoisted out of the K-loops: table
//   operands are zero-padded and streaming-operand addresses clamped.
// radial_forward (eq. Arlm_to_coeff with eq. matvec_final's kinetic term):
//   Z[n][i] = sum_r w_r R_ln(r) A[r][lm][i] (+ Zkb[lm*N+n][i], the projector term)
//   out = alpha (Z + (Lambda_ln/2 - c) Yin) + beta Yold
//   per (l, m): M = N, K = n_r, N = k; the last factor makes the kernel one
//   step of the scaled Chebyshev recurrence.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ces_internal.h"
#include "mfma.h"

namespace ces {
namespace {

__device__ __forceinline__ int isqrt_lm(int lm) {
  int l = static_cast<int>(sqrtf(static_cast<float>(lm)));
  while (l * l > lm) --l;
  while ((l + 1) * (l + 1) <= lm) ++l;
  return l;
}

constexpr int RI_NT = 2;   // 16-column tiles per workgroup (32 columns)

// Padded tables (zeros outside the valid range):
//   RiT [l][N4][R16]  R_ln(r_k) at [l][n][r];  N4 = N up to 4, R16 = n_r up to 16
//   RfT [l][R4][N16]  w_k R_ln(r_k) at [l][r][n]; R4 = n_r up to 4, N16 = N up to 16
__host__ __device__ inline int rup(int v, int m) { return (v + m - 1) / m * m; }

// Workgroup: one (l, m), 32 columns; M = n_r split over the 4 waves (MT
// 16-row tiles each; tiles past the last repeat it and are not stored).  The
// X tile (N rows x 32 columns, zero-padded to a multiple of 16 rows) is staged
// in LDS; the table operand is read in chunks of four k-steps, the next chunk
// in flight while the current one runs.  Column tile nt of lane l16 is column
// 2 l16 + nt of the 32: a lane reads both B values of a k-step with one
// 8-byte LDS read and writes both results of a row with one 8-byte store.
// FP64 is held to three waves per SIMD (309 atoms: 10.9 -> 10.4 ms; 147 atoms
// 1.76 -> 1.64 ms; no spills).
template <typename T, int MT, int CK, bool ONE, bool NTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 1, 8)))
void k_radial_inverse_mfma(const T* __restrict__ RiT,
                                                             const T* __restrict__ X,
                                                             int64_t ldx, T* __restrict__ G,
                                                             const int* __restrict__ lay,
                                                             int L, int N, int n_r, int k,
                                                             int kp) {
  typedef typename MF<T>::acc acc_t;
  static_assert(RI_NT == 2, "a lane holds the two columns 2 l16 and 2 l16 + 1");
  constexpr int CW = 16 * RI_NT, XW = CW + 2;   // even pitch: 8-byte aligned pairs
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Xs = reinterpret_cast<T*>(smem_raw);  // [N16][XW]  X[n][i]
  const int N4 = rup(N, 4), R16 = rup(n_r, 16);
  const int lm = blockIdx.y;
  const int l = isqrt_lm(lm);
  // this l's radial functions: N_l of them from coefficient off_l + (l + m) N_l
  const int Nl = lay[2 * l + 1];
  const int64_t xbase = lay[2 * l] + static_cast<int64_t>(lm - l * l) * Nl;
  const int N16l = rup(Nl, 16);
  const int i0 = blockIdx.x * CW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int nmt = R16 / 16;
  const T* Rl = RiT + static_cast<int64_t>(l) * N4 * R16 + l16;
  int mrow[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) mrow[u] = min(wave + 4 * u, nmt - 1) * 16;
  // a last tile past nmt repeats an earlier one and is not stored: in FP32
  // its MFMAs are skipped (wave-uniform; 309 atoms: inverse 6.1 -> 5.8 ms,
  // forward 8.6 -> 8.2 ms); FP64 keeps the plain loop (the branch costs the
  // forward kernel a wave per SIMD: 15.7 -> 20.2 ms)
  const bool skip_last = sizeof(T) == 4 && MT > 1 && wave + 4 * (MT - 1) >= nmt;
  // table operand in chunks of CK k-steps (4 CK rows n)
  auto load = [&](int chunk, T (*a)[MT]) {
#pragma unroll
    for (int t = 0; t < CK; ++t) {
      // rows past N4 read row N4 - 1 and are masked where used (a select
      // here would wait for each load)
      const int nc = min(chunk * 4 * CK + t * 4 + kk, N4 - 1);
#pragma unroll
      for (int u = 0; u < MT; ++u) a[t][u] = Rl[static_cast<int64_t>(nc) * R16 + mrow[u]];
    }
  };
  T ca[CK][MT];
  load(0, ca);   // the first chunk is in flight with the X tile below
  __builtin_amdgcn_sched_barrier(0);
  {
    // X tile: thread (column ii, rows n0 + 8 q), every load issued before the
    // LDS writes; N16 <= 4 CK rows in one chunk, N <= 192 otherwise
    constexpr int XQ = ONE ? CK / 2 : 24;
    // an l with no radial functions (N_l = 0) reads coefficient 0 and stores
    // only zeros
    const T* Xl = X + (Nl > 0 ? xbase : 0);
    const int ii = threadIdx.x >> 3, n0 = threadIdx.x & 7;
    const bool iok = i0 + ii < k;
    const T* xc = Xl + static_cast<int64_t>(min(i0 + ii, k - 1)) * ldx;
    const int nlast = max(Nl - 1, 0);
    T xv[XQ];
#pragma unroll
    for (int q = 0; q < XQ; ++q) xv[q] = xc[min(n0 + 8 * q, nlast)];
#pragma unroll
    for (int q = 0; q < XQ; ++q) {
      const int n = n0 + 8 * q;
      if (n < N16l) Xs[n * XW + ii] = (iok && n < Nl) ? xv[q] : T(0);
    }
  }
  __syncthreads();
  acc_t acc[MT][RI_NT];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  auto step = [&](int n, const T* a) {
    T b[RI_NT];
    load_vec<T, RI_NT>(Xs + n * XW + 2 * l16, b);
    const bool ok = n < N4;                       // table rows N..N4-1 are zero
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      if (u == MT - 1 && skip_last) break;
      const T av = ok ? a[u] : T(0);
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = MF<T>::mma(av, b[nt], acc[u][nt]);
    }
  };
  // the contraction runs over the N16l rows Xs holds (zero past N_l)
  if constexpr (ONE) {                            // whole contraction in one chunk (N16 <= 4 CK)
#pragma unroll
    for (int t = 0; t < CK; ++t) {
      if (4 * t >= N16l) break;
      step(t * 4 + kk, ca[t]);
    }
  } else {
    const int nch = (N16l + 4 * CK - 1) / (4 * CK);
    T na[CK][MT];
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) load(c + 1, na);
#pragma unroll
      for (int t = 0; t < CK; ++t) {
        if (c * 4 * CK + 4 * t >= N16l) break;
        step(c * 4 * CK + t * 4 + kk, ca[t]);
      }
#pragma unroll
      for (int t = 0; t < CK; ++t)
#pragma unroll
        for (int u = 0; u < MT; ++u) ca[t][u] = na[t][u];
    }
  }
  if (i0 + 2 * l16 >= kp) return;   // this lane's columns lie past the block
  const int64_t rstride = static_cast<int64_t>(L) * L * kp;
  T* Gb = G + static_cast<int64_t>(lm) * kp + i0 + 2 * l16;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = mt * 16 + MF<T>::row(lane, v);
      T pr[RI_NT];
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) pr[nt] = acc[u][nt][v];
      if (r < n_r) store_vec<T, RI_NT, NTS>(Gb + r * rstride, pr);
    }
  }
}

// Workgroup: one (l, m), 32 columns; M = N split over the 4 waves (MT tiles
// each, repeated past the last and not stored); K = n_r in chunks of four
// k-steps with the next chunk's operands in flight.  The projector term
// (column-major d x k, ld d) is added in the epilogue when Zkb is given.
// Column tile nt of lane l16 is column 2 l16 + nt of the 32 (one 8-byte load
// of the streamed operand per k-step), so result row q of tile nt is column
// 2 q + nt.
template <typename T, int MT, int CK, bool ONE>
__global__ __launch_bounds__(256) void k_radial_forward_mfma(
    const T* __restrict__ RfT, const T* __restrict__ A, const T* __restrict__ lamh,
    const T* __restrict__ Yin, int64_t ldin, const T* __restrict__ Yold, int64_t ldold,
    T* __restrict__ out, int64_t ldout, T alpha, T cshift, T beta, int kinetic,
    const T* __restrict__ Zkb, const int* __restrict__ lay, int64_t d, int L, int N, int n_r,
    int k, int kp) {
  typedef typename MF<T>::acc acc_t;
  const int R4 = rup(n_r, 4), N16 = rup(N, 16);
  const int lm = blockIdx.y;
  const int l = isqrt_lm(lm);
  // this l's radial functions: rows n < N_l at coefficient off_l + (l + m) N_l + n
  const int Nl = lay[2 * l + 1];
  if (Nl == 0) return;   // no coefficients for this l
  const int64_t obase = lay[2 * l] + static_cast<int64_t>(lm - l * l) * Nl;
  const int i0 = blockIdx.x * (16 * RI_NT);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int nmt = rup(Nl, 16) / 16;
  int mrow[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) mrow[u] = min(wave + 4 * u, nmt - 1) * 16;
  // a last tile past nmt repeats an earlier one and is not stored: in FP32
  // its MFMAs are skipped (wave-uniform; 309 atoms: inverse 6.1 -> 5.8 ms,
  // forward 8.6 -> 8.2 ms); FP64 keeps the plain loop (the branch costs the
  // forward kernel a wave per SIMD: 15.7 -> 20.2 ms)
  const bool skip_last = sizeof(T) == 4 && MT > 1 && wave + 4 * (MT - 1) >= nmt;
  // this lane's column pair, clamped into the block (a ragged last block's
  // lanes past it load the last pair; their columns are >= kp and not stored)
  const int cl = min(2 * l16, kp - i0 - 2);
  acc_t acc[MT][RI_NT];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  const T* Rl = RfT + static_cast<int64_t>(l) * R4 * N16 + l16;
  const T* Ab = A + static_cast<int64_t>(lm) * kp + i0 + cl;
  const int64_t rstride = static_cast<int64_t>(L) * L * kp;
  // operands in chunks of CK k-steps (4 CK radial nodes)
  auto load = [&](int chunk, T (*a)[MT], T (*b)[RI_NT]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < CK; ++t) {
      // rows past R4 read row R4 - 1 and are masked where used (a select
      // here would wait for each load)
      const int r = chunk * 4 * CK + t * 4 + kk;
      const int rt = min(r, R4 - 1);
      const int64_t roff = static_cast<int64_t>(min(r, n_r - 1)) * rstride;
#pragma unroll
      for (int u = 0; u < MT; ++u) a[t][u] = Rl[static_cast<int64_t>(rt) * N16 + mrow[u]];
      load_vec<T, RI_NT>(Ab + roff, b[t]);
    }
  };
  // transposed product Z^T = A^T Rf: the streamed A block is the MFMA A
  // operand and the table the B operand, so the result has lanes along n
  // and the epilogue reads and writes runs of n in each column i
  auto step = [&](int r, const T* a, const T* b) __attribute__((always_inline)) {
    const bool ok = r < R4;                         // table rows n_r..R4-1 are zero
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      if (u == MT - 1 && skip_last) break;
      const T av = ok ? a[u] : T(0);
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = MF<T>::mma(b[nt], av, acc[u][nt]);
    }
  };
  T ca[CK][MT], cb[CK][RI_NT];
  load(0, ca, cb);
  // epilogue operands (lanes along n, registers along i), indices clamped
  // into the block, invalid entries not stored: in the one-chunk form they
  // are loaded with the contraction's, so the epilogue waits for nothing new;
  // in the streamed FP32 form (with the projector term too) they are loaded
  // with the last chunk, in flight while its MFMAs run (in FP64 the registers
  // would cost a wave per SIMD, so there they are read in the epilogue)
  constexpr int EPR = (ONE || sizeof(T) == 4) ? 1 : 0;
  constexpr int ZP = (!ONE && sizeof(T) == 4) ? 1 : 0;
  T yin[MT][RI_NT][4 * EPR + 1 - EPR], yold[MT][RI_NT][4 * EPR + 1 - EPR];
  T zk[MT][RI_NT][4 * ZP + 1 - ZP];
  auto epi_load = [&](const T* Y, int64_t ld, T (*y)[RI_NT][4 * EPR + 1 - EPR])
      __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      const int64_t row = obase + min(mrow[u] + l16, Nl - 1);
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4 * EPR; ++v)
          y[u][nt][v] = Y[min(i0 + 2 * MF<T>::row(lane, v) + nt, k - 1) * ld + row];
    }
  };
  auto zkb_load = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      const int64_t row = obase + min(mrow[u] + l16, Nl - 1);
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4 * ZP; ++v)
          zk[u][nt][v] = Zkb[static_cast<int64_t>(min(i0 + 2 * MF<T>::row(lane, v) + nt, k - 1)) * d + row];
    }
  };
  if constexpr (ONE) {
    if (kinetic) epi_load(Yin, ldin, yin);
    if (beta != T(0)) epi_load(Yold, ldold, yold);
  }
  __builtin_amdgcn_sched_barrier(0);   // issue every load of the chunk before the first MFMA
  if constexpr (ONE) {      // whole contraction in one chunk (R4 <= 4 CK; rows past R4 are zero)
#pragma unroll
    for (int t = 0; t < CK; ++t) step(4 * t + kk, ca[t], cb[t]);
  } else {
    const int nch = (R4 + 4 * CK - 1) / (4 * CK);
    T na[CK][MT], nb[CK][RI_NT];
    // every chunk but the last is full
    for (int c = 0; c + 1 < nch; ++c) {
      load(c + 1, na, nb);
#pragma unroll
      for (int t = 0; t < CK; ++t) step(c * 4 * CK + 4 * t + kk, ca[t], cb[t]);
#pragma unroll
      for (int t = 0; t < CK; ++t) {
#pragma unroll
        for (int u = 0; u < MT; ++u) ca[t][u] = na[t][u];
#pragma unroll
        for (int nt = 0; nt < RI_NT; ++nt) cb[t][nt] = nb[t][nt];
      }
    }
    if constexpr (EPR) {
      if (kinetic) epi_load(Yin, ldin, yin);
      if (beta != T(0)) epi_load(Yold, ldold, yold);
      if (Zkb) zkb_load();
    }
    __builtin_amdgcn_sched_barrier(0);
    const int c = nch - 1;
#pragma unroll
    for (int t = 0; t < CK; ++t) {
      if (c * 4 * CK + 4 * t >= R4) break;
      step(c * 4 * CK + 4 * t + kk, ca[t], cb[t]);
    }
  }
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
    const int n = mt * 16 + l16;
    if (n >= Nl) continue;
    const int64_t row = obase + n;
    const T kin = kinetic ? lamh[static_cast<int64_t>(l) * N + n] - cshift : T(0);
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // columns past k (among them any clamped onto valid data) are skipped
        const int i = i0 + 2 * MF<T>::row(lane, v) + nt;
        if (i >= k) continue;
        T z = acc[u][nt][v];
        if (Zkb) z += ZP ? zk[u][nt][v * ZP] : Zkb[static_cast<int64_t>(i) * d + row];
        if (kinetic)
          z += kin * (EPR ? yin[u][nt][v * EPR] : Yin[static_cast<int64_t>(i) * ldin + row]);
        T val = alpha * z;
        if (beta != T(0))
          val += beta * (EPR ? yold[u][nt][v * EPR] : Yold[static_cast<int64_t>(i) * ldold + row]);
        out[static_cast<int64_t>(i) * ldout + row] = val;
      }
    }
  }
}

}  // namespace

// Short contractions (N <= 64 for the inverse, n_r <= 96 for the forward)
// load every operand fragment at once (ONE: one chunk of CK k-steps); longer
// ones stream chunks of kStreamCK k-steps with the next chunk in flight.
constexpr int kStreamCK = 4;
template <typename T, int CK, bool ONE>
void radial_inverse_ck(const Basis& b, const DevTables<T>& tb, const T* X, int64_t ldx, T* G,
                       int k, int kp, hipStream_t s) {
  dim3 grid((kp + 16 * RI_NT - 1) / (16 * RI_NT), b.L * b.L);
  const size_t lds = size_t(rup(b.N, 16)) * (16 * RI_NT + 2) * sizeof(T);
  const int mt = (rup(b.n_r, 16) / 16 + 3) / 4;   // n_r <= 256: at most 4 tiles per wave
  // streaming stores when G exceeds the last-level cache (see store_vec)
  const bool nts = size_t(b.n_r) * b.L * b.L * kp * sizeof(T) > kStreamStoreBytes;
  auto go = [&](auto nts_tag) {
    constexpr bool NTS = decltype(nts_tag)::value;
    switch (mt) {
      case 1: k_radial_inverse_mfma<T, 1, CK, ONE, NTS><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.dev_lay, b.L, b.N, b.n_r, k, kp); break;
      case 2: k_radial_inverse_mfma<T, 2, CK, ONE, NTS><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.dev_lay, b.L, b.N, b.n_r, k, kp); break;
      case 3: k_radial_inverse_mfma<T, 3, CK, ONE, NTS><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.dev_lay, b.L, b.N, b.n_r, k, kp); break;
      default: k_radial_inverse_mfma<T, 4, CK, ONE, NTS><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.dev_lay, b.L, b.N, b.n_r, k, kp); break;
    }
  };
  if (nts)
    go(std::true_type());
  else
    go(std::false_type());
}

template <typename T>
void launch_radial_inverse(const Basis& b, const DevTables<T>& tb, const T* X, int64_t ldx,
                           T* G, int k, int kp, hipStream_t s) {
  if (rup(b.N, 16) <= 64) return radial_inverse_ck<T, 16, true>(b, tb, X, ldx, G, k, kp, s);
  radial_inverse_ck<T, kStreamCK, false>(b, tb, X, ldx, G, k, kp, s);
}

template <typename T, int CK, bool ONE>
void radial_forward_ck(const Basis& b, const DevTables<T>& tb, const T* A, const T* Yin,
                       int64_t ldin, const T* Yold, int64_t ldold, T* out, int64_t ldout,
                       T alpha, T cshift, T beta, bool kinetic, const T* Zkb, int k, int kp,
                       hipStream_t s) {
  dim3 grid((k + 16 * RI_NT - 1) / (16 * RI_NT), b.L * b.L);
  const int mt = (rup(b.N, 16) / 16 + 3) / 4;   // N <= 192: at most 3 tiles per wave
  const int kin = kinetic ? 1 : 0;
  switch (mt) {
    case 1: k_radial_forward_mfma<T, 1, CK, ONE><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                    ldout, alpha, cshift, beta, kin, Zkb, b.dev_lay, b.d, b.L, b.N,
                                                    b.n_r, k, kp); break;
    case 2: k_radial_forward_mfma<T, 2, CK, ONE><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                    ldout, alpha, cshift, beta, kin, Zkb, b.dev_lay, b.d, b.L, b.N,
                                                    b.n_r, k, kp); break;
    default: k_radial_forward_mfma<T, 3, CK, ONE><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                     ldout, alpha, cshift, beta, kin, Zkb, b.dev_lay, b.d, b.L, b.N,
                                                     b.n_r, k, kp); break;
  }
}

template <typename T>
void launch_radial_forward(const Basis& b, const DevTables<T>& tb, const T* A, const T* Yin,
                           int64_t ldin, const T* Yold, int64_t ldold, T* out, int64_t ldout,
                           T alpha, T cshift, T beta, bool kinetic, const T* Zkb, int k, int kp,
                           hipStream_t s) {
  const int ks = rup(b.n_r, 4) / 4;   // k-steps of the contraction over r
  if (ks <= 8)
    return radial_forward_ck<T, 8, true>(b, tb, A, Yin, ldin, Yold, ldold, out, ldout, alpha, cshift,
                                   beta, kinetic, Zkb, k, kp, s);
  if (ks <= 16)
    return radial_forward_ck<T, 16, true>(b, tb, A, Yin, ldin, Yold, ldold, out, ldout, alpha, cshift,
                                    beta, kinetic, Zkb, k, kp, s);
  if (ks <= 24)
    return radial_forward_ck<T, 24, true>(b, tb, A, Yin, ldin, Yold, ldold, out, ldout, alpha, cshift,
                                    beta, kinetic, Zkb, k, kp, s);
  radial_forward_ck<T, kStreamCK, false>(b, tb, A, Yin, ldin, Yold, ldold, out, ldout, alpha, cshift, beta,
                          kinetic, Zkb, k, kp, s);
}

#define CES_INST(T)                                                                           \
  template void launch_radial_inverse<T>(const Basis&, const DevTables<T>&, const T*, int64_t, \
                                         T*, int, int, hipStream_t);                          \
  template void launch_radial_forward<T>(const Basis&, const DevTables<T>&, const T*, const T*, \
                                         int64_t, const T*, int64_t, T*, int64_t, T, T, T, bool, \
                                         const T*, int, int, hipStream_t);
CES_INST(float)
CES_INST(double)
#undef CES_INST

}  // namespace ces
