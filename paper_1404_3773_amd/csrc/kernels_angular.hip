// Angular stage of H*X on MFMA (gfx950), and the FP64 Gram product of
// Cholesky-QR / Rayleigh-Ritz.
//
// Per radial node r and orbital i the angular stage maps G(l,m) to A(l,m)
// (eqs. G_lmr -> Ar_lm of Section 2.2.2 with V_eff between them).  It runs as
// three batched contractions over the flattened column index c = r*kp + i:
//   legendre_synth     g[r][j][s][i]  = sum_l Pm[m][l][j] G[r][l,+-m][i]
//                      (per m-slot s: M = n_theta, K = L - m, N = n_r kp)
//   phi_stage          gh[r][j][.][i] = T_rj g[r][j][.][i]   (in place)
//                      (per (r, j): M = K = S = 2L-1, N = kp); T_rj is the
//                      exact phi synthesis / V_eff / phi analysis operator,
//                      a Toeplitz-plus-Hankel matrix in the a_q, b_q Fourier
//                      sums of V_eff at (r, theta_j), built per fragment
//   legendre_analysis  A[r][l,+-m][i]  = sum_j w_j Pm[m][l][j] gh[r][j][s][i]
//                      (per m-slot s: M = L - m, K = n_theta, N = n_r kp)
// MFMA 16x16x4 (FP32 or FP64), one wave per 16-row tile; A fragment of lane
// q is A[q%16][q/16], B fragment B[q/16][q%16]; the FP32 result of lane q,
// register v is D[4(q/16)+v][q%16], the FP64 result D[q/16+4v][q%16].
#include <hip/hip_runtime.h>

#include "ces_internal.h"
#include "mfma.h"

namespace ces {
namespace {

__device__ __forceinline__ void slot_to_m(int s, int L, int& m, int& sgn) {
  // slot s < L: cos(m phi), m = s, coefficient (l, +m); else sin, (l, -m)
  if (s < L) {
    m = s;
    sgn = 1;
  } else {
    m = s - L + 1;
    sgn = -1;
  }
}

// Padded table shapes (zeros outside the valid range, so K-loops need no
// predicates on the table operand):
//   Pm   [m][L + 4][J64]   J64 = n_theta rounded up to 64
//   PwT  [m][J4][L16]      J4 = n_theta rounded up to 4, L16 = L up to 16;
//                          entry [m][j][l - m] = w_j Pm[m][l][j]
//   S4 / S16             S rounded up to 4 / 16 (phi-stage tiles)
struct AngDims {
  int L, S, LL, n_theta, kp, J64, J4, L16, S4, S16;
};

__host__ __device__ inline int rup(int v, int m) { return (v + m - 1) / m * m; }

inline AngDims ang_dims(const Basis& b, int kp) {
  AngDims a;
  a.L = b.L;
  a.S = 2 * b.L - 1;
  a.LL = b.L * b.L;
  a.n_theta = b.n_theta;
  a.kp = kp;
  a.J64 = rup(b.n_theta, 64);
  a.J4 = rup(b.n_theta, 4);
  a.L16 = rup(b.L, 16);
  a.S4 = rup(a.S, 4);
  a.S16 = rup(a.S, 16);
  return a;
}

// ------------------------------------------------------- legendre_synth

constexpr int LS_NT = 4;  // 16-column tiles per workgroup (all waves share them)

// Workgroup: one m-slot, 64 theta nodes (one 16-row tile per wave), 64
// columns i of one radial node r.  g[r][j][s][i] = sum_l Pm[m][l][j] G[r][lm][i].
template <typename T>
__global__ __launch_bounds__(256) void k_legendre_synth(const T* __restrict__ Pm,
                                                        const T* __restrict__ G,
                                                        T* __restrict__ g, AngDims D,
                                                        int n_ic) {
  typedef typename MF<T>::acc acc_t;
  const int s = blockIdx.z;
  int m, sgn;
  slot_to_m(s, D.L, m, sgn);
  const int r = blockIdx.x / n_ic;
  const int i0 = (blockIdx.x - r * n_ic) * (16 * LS_NT);
  const int nt_valid = min(LS_NT, (D.kp - i0) / 16);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kk = lane >> 4;
  const int jt = blockIdx.y * 64 + wave * 16;
  const T* Pa = Pm + (static_cast<int64_t>(m) * (D.L + 4)) * D.J64 + jt + l16;
  const T* Gr = G + static_cast<int64_t>(r) * D.LL * D.kp + i0 + l16;
  acc_t acc[LS_NT];
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) acc[nt] = zero_acc<acc_t>();
  const int K = D.L - m;
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int l = m + k0 + kk;
    const T a = Pa[l * D.J64];                    // zero rows for l >= L
    const int lc = min(l, D.L - 1);
    const int off = (lc * lc + lc + sgn * m) * D.kp;
#pragma unroll
    for (int nt = 0; nt < LS_NT; ++nt)
      if (nt < nt_valid) acc[nt] = MF<T>::mma(a, Gr[off + nt * 16], acc[nt]);
  }
  T* gr = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp + i0 + l16;
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) {
    if (nt >= nt_valid) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = jt + MF<T>::row(lane, v);
      if (j < D.n_theta) gr[static_cast<int64_t>(j) * D.S * D.kp + nt * 16] = acc[nt][v];
    }
  }
}

// ------------------------------------------------------------ phi_stage

// Coupling of input slot s into output slot so of the phi stage: with
// ha = a/2, hb = b/2 and b_{-q} = -b_q,
//   cos <- cos  ha_|m-m'| + ha_{m+m'}      sin <- sin  ha_|m-m'| - ha_{m+m'}
//   cos <- sin  hb_{m+m'} + hb_{m-m'}      sin <- cos  hb_{m+m'} - hb_{m-m'}
template <typename T>
__device__ __forceinline__ T coupling(const T* ha, const T* hb, int L, int so, int s) {
  const bool so_sin = so >= L, s_sin = s >= L;
  const int mo = so_sin ? so - L + 1 : so;
  const int m = s_sin ? s - L + 1 : s;
  const int dm = m - mo;
  const int adm = dm < 0 ? -dm : dm;
  const T bd = dm >= 0 ? hb[adm] : -hb[adm];
  if (so_sin == s_sin) return so_sin ? ha[adm] - ha[m + mo] : ha[adm] + ha[m + mo];
  return so_sin ? hb[m + mo] - bd : hb[m + mo] + bd;
}

constexpr int PS_NT = 2;   // 16-column tiles per workgroup
constexpr int PS_MT = 3;   // M-tiles per wave (S16 <= 192)

// Workgroup: one (r, theta_j), 32 columns; gh = T_rj g in place.  The A
// fragments of T_rj are assembled from four LDS lookup tables of the
// halved Fourier sums (branch-free form of `coupling`):
//   D[q + L-1]          = ha_|q|           (q = m - m', same-type pairs)
//   D[q + L-1 + S]      = sign(q) hb_|q|   (mixed pairs)
//   E[sum]              = ha_sum,  E[sum + S] = hb_sum      (sum = m + m')
//   T = sd * D[...] + se * E[...], sd = -1 only for sin <- cos,
//   se = -1 only for sin <- sin.
template <typename T>
__global__ __launch_bounds__(256) void k_phi_stage(T* __restrict__ g, const T* __restrict__ ab,
                                                   AngDims D) {
  typedef typename MF<T>::acc acc_t;
  constexpr int GW = 16 * PS_NT + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int S = D.S, L = D.L;
  const int TW = 2 * S + 64;                   // table widths (padded)
  T* Dt = reinterpret_cast<T*>(smem_raw);      // [TW]
  T* Et = Dt + TW;                             // [TW]
  T* gs = Et + TW;                             // [S4][GW]
  const int64_t rj = blockIdx.x;
  const int i0 = blockIdx.y * (16 * PS_NT);
  const int nt_valid = min(PS_NT, (D.kp - i0) / 16);
  T* gr = g + rj * S * static_cast<int64_t>(D.kp) + i0;
  const T* abr = ab + rj * 2 * S;
  for (int e = threadIdx.x; e < TW; e += blockDim.x) {
    T dv = T(0), ev = T(0);
    if (e < S) {                         // same-type difference, sum tables
      const int q = e - (L - 1);
      dv = (q > -L && q < L) ? abr[q < 0 ? -q : q] : T(0);
      ev = abr[e];
    } else if (e < 2 * S) {              // mixed difference (odd in q), hb sums
      const int q = e - S - (L - 1);
      dv = (q > -L && q < L) ? (q < 0 ? -abr[S - q] : abr[S + q]) : T(0);
      ev = abr[S + e - S];
    }
    Dt[e] = dv;
    Et[e] = ev;
  }
  {
    const int ii = threadIdx.x & 31, s0 = threadIdx.x >> 5;
    for (int s = s0; s < D.S4; s += 8)
      gs[s * GW + ii] = (s < S && i0 + ii < D.kp) ? gr[s * D.kp + ii] : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kk = lane >> 4;
  const int nmt = D.S16 / 16;
  // lane-constant output-slot data per M-tile
  int mo[PS_MT];
  bool osin[PS_MT];
#pragma unroll
  for (int u = 0; u < PS_MT; ++u) {
    const int so = min((wave + 4 * u) * 16 + l16, S - 1);   // padded rows: any finite value
    osin[u] = so >= L;
    mo[u] = osin[u] ? so - L + 1 : so;
  }
  acc_t acc[PS_MT][PS_NT];
#pragma unroll
  for (int u = 0; u < PS_MT; ++u)
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
#pragma unroll 2
  for (int k0 = 0; k0 < D.S4; k0 += 4) {
    const int s = min(k0 + kk, S - 1);         // padded g rows are zero
    const bool ssin = s >= L;
    const int m = ssin ? s - L + 1 : s;
    T b[PS_NT];
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) b[nt] = gs[(k0 + kk) * GW + nt * 16 + l16];
#pragma unroll
    for (int u = 0; u < PS_MT; ++u) {
      const int mt = wave + 4 * u;
      if (mt >= nmt) break;
      const bool same = ssin == osin[u];
      const int di = m - mo[u] + (L - 1) + (same ? 0 : S);
      const int ei = m + mo[u] + (same ? 0 : S);
      const T dv = Dt[di], ev = Et[ei];
      const T a = (same || !osin[u] ? dv : -dv) + (same && osin[u] ? -ev : ev);
#pragma unroll
      for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
    }
  }
  // inputs came from the LDS copy: write gh in place
#pragma unroll
  for (int u = 0; u < PS_MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) {
      if (nt >= nt_valid) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = mt * 16 + MF<T>::row(lane, v);
        if (so < S) gr[so * D.kp + nt * 16 + l16] = acc[u][nt][v];
      }
    }
  }
}

// ---------------------------------------------------- legendre_analysis

constexpr int LA_NT = 2;   // 16-column tiles per wave (128 columns per workgroup)
constexpr int LA_MT = 6;   // M-tiles: L - m <= 96

// Workgroup: one m-slot, up to 128 columns of one radial node (32 per wave).
// A[r][lm][i] = sum_j w_j Pm[m][l][j] gh[r][j][s][i].
template <typename T>
__global__ __launch_bounds__(256) void k_legendre_analysis(const T* __restrict__ PwT,
                                                           const T* __restrict__ g,
                                                           T* __restrict__ A, AngDims D,
                                                           int n_ic) {
  typedef typename MF<T>::acc acc_t;
  const int s = blockIdx.y;
  int m, sgn;
  slot_to_m(s, D.L, m, sgn);
  const int r = blockIdx.x / n_ic;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kk = lane >> 4;
  const int i0 = (blockIdx.x - r * n_ic) * (64 * LA_NT) + wave * (16 * LA_NT);
  const int nt_valid = min(LA_NT, (D.kp - i0) / 16);
  if (nt_valid <= 0) return;
  const int M = D.L - m;
  const int nmt = (M + 15) / 16;
  const T* Pa = PwT + static_cast<int64_t>(m) * D.J4 * D.L16 + l16;
  const int64_t jstride = static_cast<int64_t>(D.S) * D.kp;
  const T* gb = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp + i0 + l16;
  acc_t acc[LA_MT][LA_NT];
#pragma unroll
  for (int u = 0; u < LA_MT; ++u)
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
#pragma unroll 4
  for (int k0 = 0; k0 < D.n_theta; k0 += 4) {
    const int j = k0 + kk;
    const int jc = min(j, D.n_theta - 1);          // padded A rows are zero
    T b[LA_NT];
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) b[nt] = (nt < nt_valid) ? gb[jc * jstride + nt * 16] : T(0);
#pragma unroll
    for (int u = 0; u < LA_MT; ++u) {
      if (u >= nmt) break;
      const T a = Pa[j * D.L16 + u * 16];
#pragma unroll
      for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
    }
  }
  T* Ar = A + static_cast<int64_t>(r) * D.LL * D.kp + i0 + l16;
#pragma unroll
  for (int nt = 0; nt < LA_NT; ++nt) {
    if (nt >= nt_valid) break;
#pragma unroll
    for (int u = 0; u < LA_MT; ++u) {
      if (u >= nmt) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int l = m + u * 16 + MF<T>::row(lane, v);
        if (l < D.L) Ar[(l * l + l + sgn * m) * D.kp + nt * 16] = acc[u][nt][v];
      }
    }
  }
}

// ------------------------------------------------------------ FP64 Gram

constexpr int GR_T = 64, GR_K = 16;

// part[chunk][j][i] = sum over rows of this chunk of A[row][i] B[row][j]
// (column-major A, B with leading dimensions lda, ldb); tiles of 64 x 64.
__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ Am, int64_t lda,
                                                      const double* __restrict__ Bm, int64_t ldb,
                                                      double* __restrict__ part, int64_t rows,
                                                      int k, int64_t chunk) {
  __shared__ double As[GR_K][GR_T + 1];
  __shared__ double Bs[GR_K][GR_T + 1];
  const int i0 = blockIdx.x * GR_T, j0 = blockIdx.y * GR_T;
  const int64_t r0 = static_cast<int64_t>(blockIdx.z) * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0;
  for (int64_t q0 = r0; q0 < r1; q0 += GR_K) {
    for (int e = tid; e < GR_K * GR_T; e += 256) {
      const int kk = e % GR_K, cc = e / GR_K;
      const int64_t row = q0 + kk;
      As[kk][cc] = (row < r1 && i0 + cc < k) ? Am[static_cast<int64_t>(i0 + cc) * lda + row] : 0.0;
      Bs[kk][cc] = (row < r1 && j0 + cc < k) ? Bm[static_cast<int64_t>(j0 + cc) * ldb + row] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GR_K; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tx + 16 * a];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][ty + 16 * c];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] += av[a] * bv[c];
    }
    __syncthreads();
  }
  double* P = part + static_cast<int64_t>(blockIdx.z) * k * k;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + tx + 16 * a;
    if (i >= k) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + ty + 16 * c;
      if (j < k) P[static_cast<int64_t>(j) * k + i] = acc[a][c];
    }
  }
}

// C[e] = sum_c part[c][e]: one wave per element, lanes stride the chunks.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part,
                                                     double* __restrict__ C, int k, int nchunk) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int lane = threadIdx.x & 63;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (e >= kk) return;
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += part[c * kk + e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) C[e] = s;
}

}  // namespace

template <typename T>
void launch_legendre_synth(const Basis& b, const DevTables<T>& tb, const T* G, T* gbuf, int kp,
                           hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  const int n_ic = (kp + 16 * LS_NT - 1) / (16 * LS_NT);
  dim3 grid(b.n_r * n_ic, (b.n_theta + 63) / 64, D.S);
  k_legendre_synth<T><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic);
}

template <typename T>
void launch_phi_stage(const Basis& b, const T* ab, T* gbuf, int kp, hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  dim3 grid(b.n_r * b.n_theta, (kp + 16 * PS_NT - 1) / (16 * PS_NT));
  const size_t lds = (2 * size_t(2 * D.S + 64) + size_t(D.S4) * (16 * PS_NT + 1)) * sizeof(T);
  k_phi_stage<T><<<grid, 256, lds, s>>>(gbuf, ab, D);
}

template <typename T>
void launch_legendre_analysis(const Basis& b, const DevTables<T>& tb, const T* gbuf, T* A,
                              int kp, hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  const int n_ic = (kp + 64 * LA_NT - 1) / (64 * LA_NT);
  dim3 grid(b.n_r * n_ic, D.S);
  k_legendre_analysis<T><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, D, n_ic);
}

int gram_chunks(int64_t rows, int k) {
  const int tiles = ((k + GR_T - 1) / GR_T) * ((k + GR_T - 1) / GR_T);
  int64_t want = (1024 + tiles - 1) / tiles;   // ~1024 workgroups in flight
  const int64_t maxc = (rows + 255) / 256;     // at least 256 rows per chunk
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  if (want > 256) want = 256;
  return static_cast<int>(want);
}

void launch_gram(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                 double* part, int64_t rows, int k, hipStream_t s) {
  const int nch = gram_chunks(rows, k);
  const int64_t chunk = (rows + nch - 1) / nch;
  dim3 grid((k + GR_T - 1) / GR_T, (k + GR_T - 1) / GR_T, nch);
  k_gram_partial<<<grid, 256, 0, s>>>(A, lda, B, ldb, part, rows, k, chunk);
  const int64_t kk = static_cast<int64_t>(k) * k;
  k_gram_reduce<<<static_cast<unsigned>((kk + 3) / 4), 256, 0, s>>>(part, C, k, nch);
}

#define CES_INST(T)                                                                          \
  template void launch_legendre_synth<T>(const Basis&, const DevTables<T>&, const T*, T*, int, \
                                         hipStream_t);                                       \
  template void launch_phi_stage<T>(const Basis&, const T*, T*, int, hipStream_t);             \
  template void launch_legendre_analysis<T>(const Basis&, const DevTables<T>&, const T*, T*,   \
                                            int, hipStream_t);
CES_INST(float)
CES_INST(double)
#undef CES_INST


}  // namespace ces
