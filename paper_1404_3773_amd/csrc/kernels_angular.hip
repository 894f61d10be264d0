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

namespace ces {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;
template <>
struct MF<float> {
  typedef f4 acc;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct MF<double> {
  typedef d4 acc;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename A>
__device__ __forceinline__ A zero_acc() {
  A z;
  z[0] = 0;
  z[1] = 0;
  z[2] = 0;
  z[3] = 0;
  return z;
}

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

// ------------------------------------------------------- legendre_synth

constexpr int LS_NT = 4;  // N-tiles (16 columns each) per wave

template <typename T>
__global__ __launch_bounds__(256) void k_legendre_synth(const T* __restrict__ Pm,
                                                        const T* __restrict__ G,
                                                        T* __restrict__ g, int L, int n_theta,
                                                        int kp, int64_t NC) {
  typedef typename MF<T>::acc acc_t;
  const int s = blockIdx.z;
  int m, sgn;
  slot_to_m(s, L, m, sgn);
  const int S = 2 * L - 1, LL = L * L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = blockIdx.y * 64 + wave * 16;
  const int64_t cbase = static_cast<int64_t>(blockIdx.x) * (16 * LS_NT);
  const int K = L - m;
  const int jrow = j0 + (lane & 15);
  const int kk = lane >> 4;
  acc_t acc[LS_NT];
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) acc[nt] = zero_acc<acc_t>();
  int64_t boff[LS_NT];
  bool bok[LS_NT];
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) {
    const int64_t c = cbase + nt * 16 + (lane & 15);
    bok[nt] = c < NC;
    const int64_t r = c / kp, i = c - r * kp;
    boff[nt] = r * LL * static_cast<int64_t>(kp) + i;
  }
  const T* Pmm = Pm + static_cast<int64_t>(m) * L * n_theta;
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int l = m + k0 + kk;
    const bool lok = l < L;
    const T a = (lok && jrow < n_theta) ? Pmm[static_cast<int64_t>(l) * n_theta + jrow] : T(0);
    const int64_t lmoff = static_cast<int64_t>(l * l + l + sgn * m) * kp;
#pragma unroll
    for (int nt = 0; nt < LS_NT; ++nt) {
      const T b = (lok && bok[nt]) ? G[boff[nt] + lmoff] : T(0);
      acc[nt] = MF<T>::mma(a, b, acc[nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) {
    const int64_t c = cbase + nt * 16 + (lane & 15);
    if (c >= NC) continue;
    const int64_t r = c / kp, i = c - r * kp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + MF<T>::row(lane, v);
      if (j < n_theta) g[((r * n_theta + j) * S + s) * kp + i] = acc[nt][v];
    }
  }
}

// ------------------------------------------------------------ phi_stage

// Coupling of input slot s into output slot so (see kernels.hip header):
// cos-cos a_|m-m'| + a_{m+m'}, cos(out)-sin(in) b_{m+m'} + b_{m-m'},
// sin(out)-cos(in) b_{m+m'} - b_{m-m'}, sin-sin a_|m-m'| - a_{m+m'}, with
// ha = a/2, hb = b/2 (already halved in the table) and b_{-q} = -b_q.
template <typename T>
__device__ __forceinline__ T coupling(const T* ha, const T* hb, int L, int so, int s) {
  const bool so_sin = so >= L, s_sin = s >= L;
  const int mo = so_sin ? so - L + 1 : so;
  const int m = s_sin ? s - L + 1 : s;
  const int dm = m - mo;
  const int adm = dm < 0 ? -dm : dm;
  const T bd = dm >= 0 ? hb[adm] : -hb[adm];
  const T hsum = so_sin == s_sin ? ha[m + mo] : hb[m + mo];
  const T hdif = so_sin == s_sin ? ha[adm] : bd;
  // cos-cos: hdif + hsum; sin-sin: hdif - hsum; cos-sin: hsum + bd;
  // sin-cos: hsum - bd
  if (so_sin == s_sin) return so_sin ? hdif - hsum : hdif + hsum;
  return so_sin ? hsum - bd : hsum + bd;
}

constexpr int PS_NT = 2;   // N-tiles per wave
constexpr int PS_MT = 3;   // M-tiles held per wave (S <= 16 * 4 * PS_MT = 192)

template <typename T>
__global__ __launch_bounds__(256) void k_phi_stage(T* __restrict__ g, const T* __restrict__ ab,
                                                   int L, int n_theta, int kp) {
  typedef typename MF<T>::acc acc_t;
  __shared__ T sab[2 * 192];
  const int S = 2 * L - 1;
  const int64_t rj = blockIdx.x;   // r * n_theta + j
  const int i0 = blockIdx.y * (16 * PS_NT);
  for (int q = threadIdx.x; q < 2 * S; q += blockDim.x) sab[q] = ab[rj * 2 * S + q];
  __syncthreads();
  const T* ha = sab;
  const T* hb = sab + S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nmt = (S + 15) / 16;
  T* gr = g + rj * S * static_cast<int64_t>(kp);
  acc_t acc[PS_MT][PS_NT];
#pragma unroll
  for (int u = 0; u < PS_MT; ++u)
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  const int kk = lane >> 4;
  for (int k0 = 0; k0 < S; k0 += 4) {
    const int s = k0 + kk;
    T b[PS_NT];
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) {
      const int i = i0 + nt * 16 + (lane & 15);
      b[nt] = (s < S && i < kp) ? gr[static_cast<int64_t>(s) * kp + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < PS_MT; ++u) {
      const int mt = wave + 4 * u;
      if (mt >= nmt) break;
      const int so = mt * 16 + (lane & 15);
      const T a = (so < S && s < S) ? coupling(ha, hb, L, so, s) : T(0);
#pragma unroll
      for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
    }
  }
  __syncthreads();  // every wave has read its g inputs; write gh in place
#pragma unroll
  for (int u = 0; u < PS_MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
#pragma unroll
    for (int nt = 0; nt < PS_NT; ++nt) {
      const int i = i0 + nt * 16 + (lane & 15);
      if (i >= kp) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int so = mt * 16 + MF<T>::row(lane, v);
        if (so < S) gr[static_cast<int64_t>(so) * kp + i] = acc[u][nt][v];
      }
    }
  }
}

// ---------------------------------------------------- legendre_analysis

constexpr int LA_NT = 2;   // N-tiles per wave
constexpr int LA_MT = 6;   // M-tiles per wave: L - m <= 96

template <typename T>
__global__ __launch_bounds__(256) void k_legendre_analysis(const T* __restrict__ PwT,
                                                           const T* __restrict__ g,
                                                           T* __restrict__ A, int L,
                                                           int n_theta, int kp, int64_t NC) {
  typedef typename MF<T>::acc acc_t;
  const int s = blockIdx.y;
  int m, sgn;
  slot_to_m(s, L, m, sgn);
  const int S = 2 * L - 1, LL = L * L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t cbase = static_cast<int64_t>(blockIdx.x) * (64 * LA_NT) + wave * (16 * LA_NT);
  const int M = L - m;
  const int nmt = (M + 15) / 16;
  const int kk = lane >> 4;
  acc_t acc[LA_MT][LA_NT];
#pragma unroll
  for (int u = 0; u < LA_MT; ++u)
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  int64_t boff[LA_NT];
  bool bok[LA_NT];
#pragma unroll
  for (int nt = 0; nt < LA_NT; ++nt) {
    const int64_t c = cbase + nt * 16 + (lane & 15);
    bok[nt] = c < NC;
    const int64_t r = c / kp, i = c - r * kp;
    boff[nt] = (r * n_theta * S + s) * static_cast<int64_t>(kp) + i;
  }
  const T* Pw = PwT + static_cast<int64_t>(m) * n_theta * L;
  const int64_t jstride = static_cast<int64_t>(S) * kp;
  for (int k0 = 0; k0 < n_theta; k0 += 4) {
    const int j = k0 + kk;
    const bool jok = j < n_theta;
    T b[LA_NT];
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) b[nt] = (jok && bok[nt]) ? g[boff[nt] + j * jstride] : T(0);
#pragma unroll
    for (int u = 0; u < LA_MT; ++u) {
      if (u >= nmt) break;
      const int l = m + u * 16 + (lane & 15);
      const T a = (jok && l < L) ? Pw[static_cast<int64_t>(j) * L + l] : T(0);
#pragma unroll
      for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < LA_NT; ++nt) {
    const int64_t c = cbase + nt * 16 + (lane & 15);
    if (c >= NC) continue;
    const int64_t r = c / kp, i = c - r * kp;
#pragma unroll
    for (int u = 0; u < LA_MT; ++u) {
      if (u >= nmt) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int l = m + u * 16 + MF<T>::row(lane, v);
        if (l < L) A[(r * LL + l * l + l + sgn * m) * kp + i] = acc[u][nt][v];
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

__global__ void k_gram_reduce(const double* __restrict__ part, double* __restrict__ C, int k,
                              int nchunk) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < kk;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[c * kk + e];
    C[e] = s;
  }
}

}  // namespace

template <typename T>
void launch_angular_mfma(const Basis& b, const DevTables<T>& tb, const T* ab, const T* G, T* gbuf,
                         T* A, int kp, hipStream_t s) {
  const int L = b.L, S = 2 * L - 1;
  const int64_t NC = static_cast<int64_t>(b.n_r) * kp;
  {
    dim3 grid(static_cast<unsigned>((NC + 16 * LS_NT - 1) / (16 * LS_NT)),
              (b.n_theta + 63) / 64, S);
    k_legendre_synth<T><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, L, b.n_theta, kp, NC);
  }
  {
    dim3 grid(b.n_r * b.n_theta, (kp + 16 * PS_NT - 1) / (16 * PS_NT));
    k_phi_stage<T><<<grid, 256, 0, s>>>(gbuf, ab, L, b.n_theta, kp);
  }
  {
    dim3 grid(static_cast<unsigned>((NC + 64 * LA_NT - 1) / (64 * LA_NT)), S);
    k_legendre_analysis<T><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, L, b.n_theta, kp, NC);
  }
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
  int gb = static_cast<int>((kk + 255) / 256);
  if (gb > 4096) gb = 4096;
  k_gram_reduce<<<gb, 256, 0, s>>>(part, C, k, nch);
}

template void launch_angular_mfma<float>(const Basis&, const DevTables<float>&, const float*,
                                         const float*, float*, float*, int, hipStream_t);
template void launch_angular_mfma<double>(const Basis&, const DevTables<double>&, const double*,
                                          const double*, double*, double*, int, hipStream_t);

}  // namespace ces
