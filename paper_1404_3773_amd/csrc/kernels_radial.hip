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
// in flight while the current one runs.
template <typename T, int MT>
__global__ __launch_bounds__(256) void k_radial_inverse_mfma(const T* __restrict__ RiT,
                                                             const T* __restrict__ X,
                                                             int64_t ldx, T* __restrict__ G,
                                                             int L, int N, int n_r, int k,
                                                             int kp) {
  typedef typename MF<T>::acc acc_t;
  constexpr int CW = 16 * RI_NT, XW = CW + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Xs = reinterpret_cast<T*>(smem_raw);  // [N16][XW]  X[n][i]
  const int N4 = rup(N, 4), N16 = rup(N, 16), R16 = rup(n_r, 16);
  const int lm = blockIdx.y;
  const int l = isqrt_lm(lm);
  const int i0 = blockIdx.x * CW;
  {
    const T* Xl = X + static_cast<int64_t>(lm) * N;
    const int ii = threadIdx.x >> 3, n0 = threadIdx.x & 7;
    const bool iok = i0 + ii < k;
    const T* xc = Xl + static_cast<int64_t>(i0 + ii) * ldx;
    for (int n = n0; n < N16; n += 8) Xs[n * XW + ii] = (iok && n < N) ? xc[n] : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int nmt = R16 / 16;
  const T* Rl = RiT + static_cast<int64_t>(l) * N4 * R16 + l16;
  int mrow[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) mrow[u] = min(wave + 4 * u, nmt - 1) * 16;
  acc_t acc[MT][RI_NT];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  const int nch = N16 / 16;
  T ca[4][MT], na[4][MT];
  auto load = [&](int chunk, T (*a)[MT]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = chunk * 16 + t * 4 + kk;
      const bool ok = n < N4;                       // table rows N..N4-1 are zero
      const int nc = ok ? n : N4 - 1;
#pragma unroll
      for (int u = 0; u < MT; ++u) {
        const T v = Rl[static_cast<int64_t>(nc) * R16 + mrow[u]];
        a[t][u] = ok ? v : T(0);
      }
    }
  };
  load(0, ca);
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) load(c + 1, na);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = c * 16 + t * 4 + kk;
      T b[RI_NT];
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) b[nt] = Xs[n * XW + nt * 16 + l16];
#pragma unroll
      for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = MF<T>::mma(ca[t][u], b[nt], acc[u][nt]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < MT; ++u) ca[t][u] = na[t][u];
  }
  const int64_t rstride = static_cast<int64_t>(L) * L * kp;
  T* Gb = G + static_cast<int64_t>(lm) * kp + i0 + l16;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) {
      if (i0 + nt * 16 >= kp) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mt * 16 + MF<T>::row(lane, v);
        if (r < n_r) Gb[r * rstride + nt * 16] = acc[u][nt][v];
      }
    }
  }
}

// Workgroup: one (l, m), 32 columns; M = N split over the 4 waves (MT tiles
// each, repeated past the last and not stored); K = n_r in chunks of four
// k-steps with the next chunk's operands in flight.  The projector term
// (column-major d x k, ld d) is added in the epilogue when Zkb is given.
template <typename T, int MT>
__global__ __launch_bounds__(256) void k_radial_forward_mfma(
    const T* __restrict__ RfT, const T* __restrict__ A, const T* __restrict__ lamh,
    const T* __restrict__ Yin, int64_t ldin, const T* __restrict__ Yold, int64_t ldold,
    T* __restrict__ out, int64_t ldout, T alpha, T cshift, T beta, int kinetic,
    const T* __restrict__ Zkb, int64_t d, int L, int N, int n_r, int k, int kp) {
  typedef typename MF<T>::acc acc_t;
  const int R4 = rup(n_r, 4), N16 = rup(N, 16);
  const int lm = blockIdx.y;
  const int l = isqrt_lm(lm);
  const int i0 = blockIdx.x * (16 * RI_NT);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int nmt = N16 / 16;
  int mrow[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) mrow[u] = min(wave + 4 * u, nmt - 1) * 16;
  // column of each N-tile clamped into the block (tiles past kp are not stored)
  int col[RI_NT];
#pragma unroll
  for (int nt = 0; nt < RI_NT; ++nt) col[nt] = min(nt * 16, kp - i0 - 16);
  acc_t acc[MT][RI_NT];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  const T* Rl = RfT + static_cast<int64_t>(l) * R4 * N16 + l16;
  const T* Ab = A + static_cast<int64_t>(lm) * kp + i0 + l16;
  const int64_t rstride = static_cast<int64_t>(L) * L * kp;
  const int nch = (R4 + 15) / 16;
  T ca[4][MT], cb[4][RI_NT], na[4][MT], nb[4][RI_NT];
  auto load = [&](int chunk, T (*a)[MT], T (*b)[RI_NT]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = chunk * 16 + t * 4 + kk;
      const bool ok = r < R4;                       // table rows n_r..R4-1 are zero
      const int rt = ok ? r : R4 - 1;
      const int64_t roff = static_cast<int64_t>(min(r, n_r - 1)) * rstride;
#pragma unroll
      for (int u = 0; u < MT; ++u) {
        const T v = Rl[static_cast<int64_t>(rt) * N16 + mrow[u]];
        a[t][u] = ok ? v : T(0);
      }
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) b[t][nt] = Ab[roff + col[nt]];
    }
  };
  load(0, ca, cb);
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) load(c + 1, na, nb);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int nt = 0; nt < RI_NT; ++nt)
          acc[u][nt] = MF<T>::mma(ca[t][u], cb[t][nt], acc[u][nt]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int u = 0; u < MT; ++u) ca[t][u] = na[t][u];
#pragma unroll
      for (int nt = 0; nt < RI_NT; ++nt) cb[t][nt] = nb[t][nt];
    }
  }
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int mt = wave + 4 * u;
    if (mt >= nmt) break;
#pragma unroll
    for (int nt = 0; nt < RI_NT; ++nt) {
      const int i = i0 + nt * 16 + l16;
      if (i >= k) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = mt * 16 + MF<T>::row(lane, v);
        if (n >= N) continue;
        const int64_t row = static_cast<int64_t>(lm) * N + n;
        T z = acc[u][nt][v];
        if (Zkb) z += Zkb[static_cast<int64_t>(i) * d + row];
        if (kinetic) {
          const T y = Yin[static_cast<int64_t>(i) * ldin + row];
          z += (lamh[static_cast<int64_t>(l) * N + n] - cshift) * y;
        }
        T val = alpha * z;
        if (beta != T(0)) val += beta * Yold[static_cast<int64_t>(i) * ldold + row];
        out[static_cast<int64_t>(i) * ldout + row] = val;
      }
    }
  }
}

}  // namespace

template <typename T>
void launch_radial_inverse(const Basis& b, const DevTables<T>& tb, const T* X, int64_t ldx,
                           T* G, int k, int kp, hipStream_t s) {
  dim3 grid((kp + 16 * RI_NT - 1) / (16 * RI_NT), b.L * b.L);
  const size_t lds = size_t(rup(b.N, 16)) * (16 * RI_NT + 1) * sizeof(T);
  const int mt = (rup(b.n_r, 16) / 16 + 3) / 4;   // n_r <= 256: at most 4 tiles per wave
  switch (mt) {
    case 1: k_radial_inverse_mfma<T, 1><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.L, b.N, b.n_r, k, kp); break;
    case 2: k_radial_inverse_mfma<T, 2><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.L, b.N, b.n_r, k, kp); break;
    case 3: k_radial_inverse_mfma<T, 3><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.L, b.N, b.n_r, k, kp); break;
    default: k_radial_inverse_mfma<T, 4><<<grid, 256, lds, s>>>(tb.RiT, X, ldx, G, b.L, b.N, b.n_r, k, kp); break;
  }
}

template <typename T>
void launch_radial_forward(const Basis& b, const DevTables<T>& tb, const T* A, const T* Yin,
                           int64_t ldin, const T* Yold, int64_t ldold, T* out, int64_t ldout,
                           T alpha, T cshift, T beta, bool kinetic, const T* Zkb, int k, int kp,
                           hipStream_t s) {
  dim3 grid((k + 16 * RI_NT - 1) / (16 * RI_NT), b.L * b.L);
  const int mt = (rup(b.N, 16) / 16 + 3) / 4;   // N <= 192: at most 3 tiles per wave
  switch (mt) {
    case 1: k_radial_forward_mfma<T, 1><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                ldout, alpha, cshift, beta, kinetic ? 1 : 0, Zkb,
                                                b.d, b.L, b.N, b.n_r, k, kp); break;
    case 2: k_radial_forward_mfma<T, 2><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                ldout, alpha, cshift, beta, kinetic ? 1 : 0, Zkb,
                                                b.d, b.L, b.N, b.n_r, k, kp); break;
    default: k_radial_forward_mfma<T, 3><<<grid, 256, 0, s>>>(tb.RfT, A, tb.lamh, Yin, ldin, Yold, ldold, out,
                                                ldout, alpha, cshift, beta, kinetic ? 1 : 0, Zkb,
                                                b.d, b.L, b.N, b.n_r, k, kp); break;
  }
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
