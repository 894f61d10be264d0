// Angular stage of H*X on MFMA (gfx950).
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

#include <algorithm>
#include <type_traits>

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

// Streaming stores for an output of `elems` values of T (see store_vec).
template <typename T>
bool stream_stores(size_t elems) {
  return elems * sizeof(T) > kStreamStoreBytes;
}
// f(std::true_type()) or f(std::false_type()) as `on` is set
template <typename F>
void with_nts(bool on, F&& f) {
  if (on)
    f(std::true_type());
  else
    f(std::false_type());
}

// ------------------------------------------------------- legendre_synth

// Workgroup: one m-slot, JT groups of 64 theta nodes (one 16-row tile of each
// group per wave), 16 NT columns i of one radial node r.
// g[r][j][s][i] = sum_l Pm[m][l][j] G[r][lm][i].  A wave loads the G fragments
// of a k-step once for all its JT theta tiles.
// KS > 0 (L <= 4 KS): every operand of the K loop is loaded before the first
// MFMA; KS = 0: the K loop streams its operands.
template <typename T, int LS_NT, int KS, int JT>
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
  // theta tiles of this wave; tiles past J64 (in the last workgroup) read the
  // last tile and store nothing
  int jt[JT];
  const T* Pa[JT];
#pragma unroll
  for (int u = 0; u < JT; ++u) {
    jt[u] = (blockIdx.y * JT + u) * 64 + wave * 16;
    Pa[u] = Pm + (static_cast<int64_t>(m) * (D.L + 4)) * D.J64 + min(jt[u], D.J64 - 16) + l16;
  }
  const T* Gr = G + static_cast<int64_t>(r) * D.LL * D.kp + i0 + l16;
  acc_t acc[JT][LS_NT];
#pragma unroll
  for (int u = 0; u < JT; ++u)
#pragma unroll
    for (int nt = 0; nt < LS_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  const int K = D.L - m;
  // column of each N-tile clamped into the block (tiles past nt_valid are not stored)
  int col[LS_NT];
#pragma unroll
  for (int nt = 0; nt < LS_NT; ++nt) col[nt] = min(nt * 16, D.kp - i0 - 16);
  if constexpr (KS > 0) {
    const int ks = (K + 3) >> 2;
    T a[KS][JT], b[KS][LS_NT];
    // up to 8 k-steps the loops exit early; longer ones take uniform guards
    // instead, which keeps them unrolled (an early exit there leaves a rolled
    // loop indexing the operand arrays through scratch)
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      if (KS <= 8 && t >= ks) break;
      if (t < ks) {
        // rows l >= L read row L - 1 and are masked where used
        const int lc = min(m + 4 * t + kk, D.L - 1);
#pragma unroll
        for (int u = 0; u < JT; ++u) a[t][u] = Pa[u][lc * D.J64];
        const int off = (lc * lc + lc + sgn * m) * D.kp;
#pragma unroll
        for (int nt = 0; nt < LS_NT; ++nt) b[t][nt] = Gr[off + col[nt]];
      }
    }
    __builtin_amdgcn_sched_barrier(0);   // every load issued before the first MFMA
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      if (KS <= 8 && t >= ks) break;
      if (t < ks) {
        const bool ok = m + 4 * t + kk < D.L;
#pragma unroll
        for (int u = 0; u < JT; ++u) {
          const T av = ok ? a[t][u] : T(0);
#pragma unroll
          for (int nt = 0; nt < LS_NT; ++nt) acc[u][nt] = MF<T>::mma(av, b[t][nt], acc[u][nt]);
        }
      }
    }
  } else {
  // steps whose four l rows are all below L: row offset (l^2 + l + sgn m) kp
  // advanced by second differences (l grows by 4 per step)
  const int nfull = K >> 2;
  {
    const int l = m + kk;
    int64_t off = static_cast<int64_t>(l * l + l + sgn * m) * D.kp;
    int64_t dof = static_cast<int64_t>(8 * l + 20) * D.kp;
    const int64_t ddof = 32 * static_cast<int64_t>(D.kp);
    int64_t pofs = static_cast<int64_t>(l) * D.J64;
#pragma unroll 4
    for (int t = 0; t < nfull; ++t) {
      T a[JT], b[LS_NT];
#pragma unroll
      for (int u = 0; u < JT; ++u) a[u] = Pa[u][pofs];
#pragma unroll
      for (int nt = 0; nt < LS_NT; ++nt) b[nt] = Gr[off + col[nt]];
#pragma unroll
      for (int u = 0; u < JT; ++u)
#pragma unroll
        for (int nt = 0; nt < LS_NT; ++nt) acc[u][nt] = MF<T>::mma(a[u], b[nt], acc[u][nt]);
      pofs += 4 * D.J64;
      off += dof;
      dof += ddof;
    }
  }
  if (K & 3) {
    const int l = m + 4 * nfull + kk;
    const int lc = min(l, D.L - 1);
    const int off = (lc * lc + lc + sgn * m) * D.kp;
    T b[LS_NT];
#pragma unroll
    for (int nt = 0; nt < LS_NT; ++nt) b[nt] = Gr[off + col[nt]];
#pragma unroll
    for (int u = 0; u < JT; ++u) {
      const T a = Pa[u][l * D.J64];                 // zero rows for l >= L
#pragma unroll
      for (int nt = 0; nt < LS_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
    }
  }
  }
  T* gr = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp + i0 + l16;
#pragma unroll
  for (int u = 0; u < JT; ++u)
#pragma unroll
    for (int nt = 0; nt < LS_NT; ++nt) {
      if (nt >= nt_valid) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jt[u] + MF<T>::row(lane, v);
        if (j < D.n_theta) gr[static_cast<int64_t>(j) * D.S * D.kp + nt * 16] = acc[u][nt][v];
      }
    }
}

// Folded form (L > 32).  The theta nodes come in mirror pairs t_{n-1-j} = -t_j
// and P_l^m(-t) = (-1)^{l+m} P_l^m(t), so with E(j) the sum over l + m even
// and O(j) over l + m odd, g(j) = E(j) + O(j) and g(n-1-j) = E(j) - O(j) for
// the nodes j < nh = ceil(n_theta / 2): half the MFMA work and half the table
// reads of the direct sum.  Workgroup: one m-slot, 4 waves x JT 16-row tiles
// of the first half, 16 NT columns of one radial node; a k-step takes four l
// of one parity, l = m + par + 2 (4t + kk); steps go in chunks of CH with the
// next chunk's operands in flight while the current one runs on MFMA.
// Column tile nt of lane l16 is column NT l16 + nt of the workgroup's block,
// so a lane reads its NT B values with one vector load and writes its NT
// results of a node with one vector store: each store instruction covers
// whole 16 NT-column row pieces of g rather than 16-column halves.
template <typename T, int NT, int JT, int CH, bool NTS>
__global__ __launch_bounds__(256) void k_legendre_synth_fold(const T* __restrict__ Pm,
                                                             const T* __restrict__ G,
                                                             T* __restrict__ g, AngDims D,
                                                             int n_ic, int nh) {
  typedef typename MF<T>::acc acc_t;
  const int s = blockIdx.z;
  int m, sgn;
  slot_to_m(s, D.L, m, sgn);
  const int r = blockIdx.x / n_ic;
  const int i0 = (blockIdx.x - r * n_ic) * (16 * NT);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int tile0 = (blockIdx.y * 4 + wave) * JT;
  if (tile0 * 16 >= nh) return;   // no barriers in this kernel
  int jt[JT];
  const T* Pa[JT];
#pragma unroll
  for (int u = 0; u < JT; ++u) {
    jt[u] = (tile0 + u) * 16;
    Pa[u] = Pm + (static_cast<int64_t>(m) * (D.L + 4)) * D.J64 + min(jt[u], D.J64 - 16) + l16;
  }
  // this lane's columns i0 + NT l16 + nt; in a ragged last block (kp - i0 a
  // multiple of 16 below 16 NT) the lanes past it read the last NT columns
  // and store nothing
  const int cl = min(NT * l16, D.kp - i0 - NT);
  const bool colok = i0 + NT * l16 < D.kp;
  const T* Gr = G + static_cast<int64_t>(r) * D.LL * D.kp + i0 + cl;
  acc_t E[JT][NT], O[JT][NT];
#pragma unroll
  for (int u = 0; u < JT; ++u)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      E[u][nt] = zero_acc<acc_t>();
      O[u][nt] = zero_acc<acc_t>();
    }
  const int K = D.L - m;
  const int nE = ((K + 1) / 2 + 3) / 4, nO = (K / 2 + 3) / 4;
  const int nst = nE + nO;
  // step st: parity par = (st >= nE), t = st - par nE; rows l >= L read row
  // L - 1 and are masked at the MFMA
  auto lrow = [&](int st) {
    const int par = st >= nE ? 1 : 0;
    const int t = st - par * nE;
    return m + par + 8 * t + 2 * kk;
  };
  auto load = [&](int st, T (&a)[JT], T (&b)[NT]) __attribute__((always_inline)) {
    const int lc = min(lrow(st), D.L - 1);
#pragma unroll
    for (int u = 0; u < JT; ++u) a[u] = Pa[u][lc * D.J64];
    const int64_t off = static_cast<int64_t>(lc * lc + lc + sgn * m) * D.kp;
    load_vec<T, NT>(Gr + off, b);
  };
  // CH steps per chunk, all loaded before the chunk's MFMAs; the next chunk
  // is in flight while the current one runs
  auto mma_step = [&](int st, const T (&a)[JT], const T (&b)[NT]) __attribute__((always_inline)) {
    const bool ok = st < nst && lrow(st) < D.L;
    if (st < nE) {
#pragma unroll
      for (int u = 0; u < JT; ++u) {
        const T av = ok ? a[u] : T(0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) E[u][nt] = MF<T>::mma(av, b[nt], E[u][nt]);
      }
    } else {
#pragma unroll
      for (int u = 0; u < JT; ++u) {
        const T av = ok ? a[u] : T(0);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) O[u][nt] = MF<T>::mma(av, b[nt], O[u][nt]);
      }
    }
  };
  const int nch = (nst + CH - 1) / CH;
  T ca[CH][JT], cb[CH][NT], na[CH][JT], nb[CH][NT];
#pragma unroll
  for (int t = 0; t < CH; ++t) load(min(t, nst - 1), ca[t], cb[t]);
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) {
#pragma unroll
      for (int t = 0; t < CH; ++t) load(min((c + 1) * CH + t, nst - 1), na[t], nb[t]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) mma_step(c * CH + t, ca[t], cb[t]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
#pragma unroll
      for (int u = 0; u < JT; ++u) ca[t][u] = na[t][u];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) cb[t][nt] = nb[t][nt];
    }
  }
  if (!colok) return;
  T* gr = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp + i0 + NT * l16;
  const int64_t jstride = static_cast<int64_t>(D.S) * D.kp;
#pragma unroll
  for (int u = 0; u < JT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = jt[u] + MF<T>::row(lane, v);
      if (j < nh) {
        T pe[NT], pm[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          pe[nt] = E[u][nt][v] + O[u][nt][v];
          pm[nt] = E[u][nt][v] - O[u][nt][v];
        }
        store_vec<T, NT, NTS>(gr + j * jstride, pe);
        const int jm = D.n_theta - 1 - j;
        if (jm != j) store_vec<T, NT, NTS>(gr + jm * jstride, pm);
      }
    }
}

// ------------------------------------------------------------ phi_stage

// Coupling of input slot s into output slot so of the phi stage: with
// ha = a/2, hb = b/2 and b_{-q} = -b_q,
//   cos <- cos  ha_|m-m'| + ha_{m+m'}      sin <- sin  ha_|m-m'| - ha_{m+m'}
//   cos <- sin  hb_{m+m'} + hb_{m-m'}      sin <- cos  hb_{m+m'} - hb_{m-m'}
constexpr int PS_NT = 2;             // 16-column tiles per workgroup
constexpr int kPhiRowsPerWg = 16;    // most rows each workgroup walks, the next one in flight
constexpr int64_t kPhiMinWgs = 2048; // fewer rows per workgroup below this many workgroups

// phi stage: gh = C g per (r, theta_j) row, C the (2L-1)^2 coupling of the
// product-to-sum identity above.  K (input slots) and M (output slots) are
// laid out as a cos part (m = 0..L-1) and a sin part (m = 1..L-1), each
// padded to LP = 16 ceil(L/16) rows, so that every 16 x 4 MFMA operand tile
// lies in one of four blocks with uniform signs:
//   (out cos, in cos)  a_|q| + a_p      (out cos, in sin)  b_q + b_p
//   (out sin, in cos) -b_q  + b_p       (out sin, in sin)  a_|q| - a_p
// with q = m - m', p = m + m'.  Each block entry is T[k - r + LP] + H[k + r]
// for block-local input / output indices k, r, from six LDS tables of 2 LP
// values per row, so an A operand costs two LDS reads and one add.  Every
// table entry is one of the row's Fourier sums times +1, -1 or 0, fixed by
// its position alone: each thread works out the source and sign of its
// entries once, and fetches their values with the row's g block, one row
// ahead, so a row takes one LDS fill and two barriers.  The K loop of each
// input block stops at its last slot, rounded up to a k-step, at compile
// time (LP - 4 TC rows of the cos block, 4 SS fewer of the sin block), so the
// padding rows cost no MFMA work and the loop stays fully unrolled.
// Column tile nt of lane l16 is column 2 l16 + nt of the workgroup's 32:
// a lane reads both B values of a k-step with one 8-byte LDS read (the four
// rows of a read then cover the banks once) and writes both results of an
// output row with one 8-byte store, so each store instruction covers whole
// 128-byte row pieces of g.
// FP32 is held to four waves per SIMD (at L = 81: 21.7 against 22.2 ms with
// the three the compiler chose by itself).
template <typename T, int LP, int TC, int SS, bool NTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1, 8)))
void k_phi_stage(T* __restrict__ g, const T* __restrict__ ab,
                                                   AngDims D, int64_t n_rows) {
  typedef typename MF<T>::acc acc_t;
  static_assert(PS_NT == 2, "a lane holds the two columns 2 l16 and 2 l16 + 1");
  constexpr int GW = 16 * PS_NT;
  constexpr int K2 = 2 * LP, NMT = K2 / 16, MT = (NMT + 3) / 4;   // M-tiles per wave
  constexpr int GPT = K2 / 8;                   // g values per thread per row
  constexpr int NE = (6 * K2 + 255) / 256;      // table entries per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int S = D.S, L = D.L;
  T* tab = reinterpret_cast<T*>(smem_raw);     // 6 tables of K2 values
  T* gs = tab + 6 * K2;                         // [K2][GW]
  const int i0 = blockIdx.x * (16 * PS_NT);
  const int tid = threadIdx.x;
  const int ii = tid & 31, kr = tid >> 5;
  // this thread's g rows k = kr + 8u (slot s < L -> K row s; slot L + j ->
  // row LP + j; k >= LP exactly when 8u >= LP).  Bit u of okm marks row k as
  // a slot; the others load a clamped address and are written as zero.
  // Offsets within a row are unsigned 32-bit (the row base stays in scalar
  // registers) and are formed at each use from cbase, which an empty asm
  // makes opaque per row so that the compiler keeps one register, not one
  // per load or store, live across the MFMA loop.
  unsigned okm = 0;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const int k = kr + 8 * u;
    const bool sn = k >= LP;
    const int kl = sn ? k - LP : k;
    const bool ok = (sn ? kl < L - 1 : kl < L) && i0 + ii < D.kp;
    okm |= (ok ? 1u : 0u) << u;
  }
  const unsigned cbase = unsigned(kr * D.kp + i0 + ii);
  const unsigned clast = unsigned(S * D.kp - 1);
  // this thread's table entries E = tid + 256 v (table E / K2, index E % K2):
  // value = sign * ab[src] with the row's sums a_x at x, b_x at S + x (x < S);
  // with q = index - LP:
  //   T0 a_|q|   T1 b_{q+1}   T2 -b_{q-1}   (b odd: b_{-x} = -b_x)
  //   H3 a_h     H4 b_{h+1}   H5 -a_{h+2}   (h = index; zero past S)
  int esrc[NE];
  T esgn[NE];
#pragma unroll
  for (int v = 0; v < NE; ++v) {
    const int E = tid + 256 * v;
    const int t = E / K2, e = E - t * K2, q = e - LP;
    int x = 0, base = 0;
    T sg = T(1);
    switch (t) {
      case 0: x = q < 0 ? -q : q; break;
      case 1: x = q + 1 < 0 ? -(q + 1) : q + 1; base = S; sg = q + 1 >= 0 ? T(1) : T(-1); break;
      case 2: x = q - 1 < 0 ? -(q - 1) : q - 1; base = S; sg = q - 1 >= 0 ? T(-1) : T(1); break;
      case 3: x = e; break;
      case 4: x = e + 1; base = S; break;
      default: x = e + 2; sg = T(-1); break;
    }
    const bool ok = E < 6 * K2 && x < S;
    esrc[v] = ok ? base + x : 0;
    esgn[v] = ok ? sg : T(0);
  }
  const int64_t rstride = static_cast<int64_t>(S) * D.kp;
  // registers holding the next row (software pipeline across rows)
  T gp[GPT], ap[NE];
  auto fetch = [&](int64_t row) {
    const T* gr = g + row * rstride;
    unsigned cb = cbase;
    asm volatile("" : "+v"(cb));
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const unsigned su = unsigned((8 * u + (8 * u >= LP ? L - LP : 0)) * D.kp);   // uniform
      gp[u] = gr[min(cb + su, clast)];
    }
    const T* abr = ab + row * 2 * S;
#pragma unroll
    for (int v = 0; v < NE; ++v) ap[v] = abr[esrc[v]];
  };
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const bool colok = i0 + 2 * l16 < D.kp;   // this lane's output columns exist
  int toff[MT], hoff[MT];
  bool ocs[MT];
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    // tiles past NMT (when NMT is not a multiple of 4) repeat the last tile;
    // their results are not written, so the MFMA loop needs no branch
    const int mt = min(wave + 4 * u, NMT - 1);
    ocs[u] = mt * 16 >= LP;
    const int rl = mt * 16 - (ocs[u] ? LP : 0) + l16;
    toff[u] = LP - rl + kk;
    hoff[u] = rl + kk;
  }
  // this wave's last tile holds no slot when it lies past NMT (a repeat, when
  // NMT is not a multiple of 4) or past the block's slots (the last sin tile
  // when L = 1 mod 16, which is TC = 3, SS = 1): its MFMAs are skipped (its
  // results are never stored).  Other shapes compile the full loop alone.
  constexpr bool CAN_SKIP = MT > 1 && ((TC == 3 && SS == 1) || NMT % 4 != 0);
  const int lastmt = wave + 4 * (MT - 1);
  const bool last_ok =
      lastmt < NMT && (lastmt * 16 < LP ? lastmt * 16 < L : lastmt * 16 - LP < L - 1);
  int64_t row = blockIdx.y;
  if (row < n_rows) fetch(row);
  for (; row < n_rows; row += gridDim.y) {
#pragma unroll
    for (int u = 0; u < GPT; ++u)
      gs[(kr + 8 * u) * GW + ii] = (okm >> u) & 1u ? gp[u] : T(0);
#pragma unroll
    for (int v = 0; v < NE; ++v) {
      const int E = tid + 256 * v;
      if (E < 6 * K2) tab[E] = esgn[v] * ap[v];
    }
    __syncthreads();
    if (row + gridDim.y < n_rows) fetch(row + gridDim.y);     // next row, in flight
    acc_t acc[MT][PS_NT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
      for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
    // the first MTE of this wave's tiles
    auto mfma_rows = [&](auto mte_tag) __attribute__((always_inline)) {
      constexpr int MTE = decltype(mte_tag)::value;
#pragma unroll
      for (int ic = 0; ic < 2; ++ic) {
        const T* Tb[MTE];
        const T* Hb[MTE];
#pragma unroll
        for (int u = 0; u < MTE; ++u) {
          const int tsel = ocs[u] == (ic == 1) ? 0 : (ic == 1 ? 1 : 2);
          const int hsel = ic == 0 ? (ocs[u] ? 4 : 3) : (ocs[u] ? 5 : 4);
          Tb[u] = tab + tsel * K2 + toff[u];
          Hb[u] = tab + hsel * K2 + hoff[u];
        }
        const T* grow = gs + (ic * LP + kk) * GW + 2 * l16;
        const int kend = ic == 0 ? LP - 4 * TC : LP - 4 * (TC + SS);   // known per unrolled ic
#pragma unroll
        for (int k0 = 0; k0 < kend; k0 += 4) {
          T b[PS_NT];
          load_vec<T, PS_NT>(grow + k0 * GW, b);
#pragma unroll
          for (int u = 0; u < MTE; ++u) {
            const T a = Tb[u][k0] + Hb[u][k0];
#pragma unroll
            for (int nt = 0; nt < PS_NT; ++nt) acc[u][nt] = MF<T>::mma(a, b[nt], acc[u][nt]);
          }
        }
      }
    };
    if constexpr (CAN_SKIP) {
      if (last_ok)
        mfma_rows(std::integral_constant<int, MT>());
      else
        mfma_rows(std::integral_constant<int, (MT > 1 ? MT - 1 : 1)>());
    } else {
      mfma_rows(std::integral_constant<int, MT>());
    }
    // inputs came from the LDS copy: write gh in place.  Lane rows of tile mt
    // are rl0 + dr(v), dr(v) = row(lane, v) - row(lane, 0) fixed per v; a
    // tile whose 16 rows all hold slots (every one but the last of each block)
    // stores without row tests.
    T* gr = g + row * rstride + i0;
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      const int mt = wave + 4 * u;
      if (mt >= NMT) break;
      const bool snu = mt * 16 >= LP;                     // sin block (uniform)
      const int lim = snu ? L - 1 : L;                    // slots in the block
      const int rt = mt * 16 - (snu ? LP : 0);            // tile's first block row
      const int rl0 = rt + MF<T>::row(lane, 0);
      unsigned ob = unsigned((rl0 + (snu ? L : 0)) * D.kp + 2 * l16);
      asm volatile("" : "+v"(ob));
      const unsigned kpu = unsigned(D.kp);
      if (colok && rt < lim) {
        const bool full = rt + 16 <= lim;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int dr = MF<T>::row(lane, v) - MF<T>::row(lane, 0);
          T pr[PS_NT];
#pragma unroll
          for (int nt = 0; nt < PS_NT; ++nt) pr[nt] = acc[u][nt][v];
          if (full || rl0 + dr < lim) store_vec<T, PS_NT, NTS>(gr + ob + dr * kpu, pr);
        }
      }
    }
    __syncthreads();   // LDS is refilled for the next row
  }
}

// ---------------------------------------------------- legendre_analysis

constexpr int LA_NT = 2;   // 16-column tiles per wave (32 columns per workgroup)
constexpr int LA_SW = 4;   // m-slots per workgroup, one per wave

// Workgroup: 32 columns of one radial node and four m-slots (one per wave).
// A[r][lm][i] = sum_j w_j Pm[m][l][j] gh[r][j][s][i].  Each wave computes all
// l-tiles of its slot (MT covers L) from one pass over gh, so gh is read once.
// Theta is taken CH k-steps (4 CH rows) at a time: with ONE (n_theta <= 4 CH)
// every operand is loaded before the first MFMA, otherwise chunks stream with
// the next one in flight while the current one runs.  Rows past n_theta read
// row n_theta - 1 and get a zero weight where used (a select on the load would
// make it wait).
template <typename T, int MT, int CH, bool ONE>
__global__ __launch_bounds__(256) void k_legendre_analysis(const T* __restrict__ PwT,
                                                           const T* __restrict__ g,
                                                           T* __restrict__ A, AngDims D,
                                                           int n_ic) {
  typedef typename MF<T>::acc acc_t;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = blockIdx.y * LA_SW + wave;
  if (s >= D.S) return;
  int m, sgn;
  slot_to_m(s, D.L, m, sgn);
  const int r = blockIdx.x / n_ic;
  const int l16 = lane & 15, kk = lane >> 4;
  const int i0 = (blockIdx.x - r * n_ic) * (16 * LA_NT);
  const int nt_valid = min(LA_NT, (D.kp - i0) / 16);
  const int nmt = (D.L - m + 15) / 16;     // l-tiles of this slot (<= MT)
  const int64_t jstride = static_cast<int64_t>(D.S) * D.kp;
  const T* gb = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp;
  // column of each N-tile, clamped into the block (tiles past nt_valid are
  // computed on valid data and not stored)
  int col[LA_NT];
#pragma unroll
  for (int nt = 0; nt < LA_NT; ++nt) col[nt] = min(i0 + nt * 16, D.kp - 16) + l16;
  const T* Pa = PwT + static_cast<int64_t>(m) * D.J4 * D.L16 + l16;
  acc_t acc[MT][LA_NT];
#pragma unroll
  for (int u = 0; u < MT; ++u)
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = zero_acc<acc_t>();
  auto load = [&](int c, T (*a)[MT], T (*b)[LA_NT]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int jc = min(c * 4 * CH + 4 * t + kk, D.n_theta - 1);
#pragma unroll
      for (int u = 0; u < MT; ++u)
        if (u < nmt) a[t][u] = Pa[jc * D.L16 + 16 * u];
#pragma unroll
      for (int nt = 0; nt < LA_NT; ++nt) b[t][nt] = gb[jc * jstride + col[nt]];
    }
  };
  auto step = [&](int j, const T* a, const T* b) __attribute__((always_inline)) {
    const bool ok = j < D.n_theta;
#pragma unroll
    for (int u = 0; u < MT; ++u) {
      if (u < nmt) {
        const T av = ok ? a[u] : T(0);
#pragma unroll
        for (int nt = 0; nt < LA_NT; ++nt) acc[u][nt] = MF<T>::mma(av, b[nt], acc[u][nt]);
      }
    }
  };
  T ca[CH][MT], cb[CH][LA_NT];
  load(0, ca, cb);
  __builtin_amdgcn_sched_barrier(0);     // the chunk's loads go out before its MFMAs
  if constexpr (ONE) {
#pragma unroll
    for (int t = 0; t < CH; ++t) step(4 * t + kk, ca[t], cb[t]);
  } else {
    const int nch = (D.n_theta + 4 * CH - 1) / (4 * CH);
    T na[CH][MT], nb[CH][LA_NT];
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) load(c + 1, na, nb);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < CH; ++t) step(c * 4 * CH + 4 * t + kk, ca[t], cb[t]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < CH; ++t) {
#pragma unroll
        for (int u = 0; u < MT; ++u) ca[t][u] = na[t][u];
#pragma unroll
        for (int nt = 0; nt < LA_NT; ++nt) cb[t][nt] = nb[t][nt];
      }
    }
  }
  T* Ar = A + static_cast<int64_t>(r) * D.LL * D.kp + l16;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    if (u >= nmt) break;
#pragma unroll
    for (int nt = 0; nt < LA_NT; ++nt) {
      if (nt >= nt_valid) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int l = m + u * 16 + MF<T>::row(lane, v);
        if (l < D.L) Ar[(l * l + l + sgn * m) * D.kp + i0 + nt * 16] = acc[u][nt][v];
      }
    }
  }
}

// Folded form (L > 32).  With mirror nodes t_{n-1-j} = -t_j, equal weights
// and P_l^m(-t) = (-1)^{l+m} P_l^m(t),
//   A(l,m) = sum_{j < nh} w_j P_l^m(t_j) [gh(j) + (-1)^{l+m} gh(n-1-j)],
// (the middle node of an odd n_theta taken once), so the l + m even rows
// contract the sums u(j) = gh(j) + gh(n-1-j) and the odd rows the differences
// v(j) over the first half of the nodes: half the MFMA work of the direct
// sum.  One m-slot per wave, NTA 16-column tiles; ME / MO 16-row l-tiles of
// each parity (rows l = m + par + 2 (16 tile + lane row)); theta in k-steps
// of four, CH steps per chunk with the next chunk's operands in flight.
// Column tile nt of lane l16 is column NTA l16 + nt of the block (as in the
// folded synthesis): one vector load per node and one vector store per row.
// FP32 with three l-tiles per parity is held to three waves per SIMD, which
// its two-step chunks fit without spills (309 atoms: 7.3 -> 7.1 ms).
template <typename T, int MH, int CH, int NTA, bool NTS>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && MH == 3 ? 3 : 1, 8)))
void k_legendre_analysis_fold(const T* __restrict__ PwT,
                                                                const T* __restrict__ g,
                                                                T* __restrict__ A, AngDims D,
                                                                int n_ic, int nh) {
  typedef typename MF<T>::acc acc_t;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = blockIdx.y * LA_SW + wave;
  if (s >= D.S) return;
  int m, sgn;
  slot_to_m(s, D.L, m, sgn);
  const int r = blockIdx.x / n_ic;
  const int l16 = lane & 15, kk = lane >> 4;
  const int i0 = (blockIdx.x - r * n_ic) * (16 * NTA);
  const int K = D.L - m;
  const int nme = ((K + 1) / 2 + 15) / 16, nmo = (K / 2 + 15) / 16;   // <= MH each
  const int64_t jstride = static_cast<int64_t>(D.S) * D.kp;
  const T* gb = g + (static_cast<int64_t>(r) * D.n_theta * D.S + s) * D.kp;
  // this lane's columns i0 + NTA l16 + nt; in a ragged last block the lanes
  // past it read the last NTA columns and store nothing
  const int cl = min(NTA * l16, D.kp - i0 - NTA);
  const bool colok = i0 + NTA * l16 < D.kp;
  const T* gbl = gb + i0 + cl;
  // table entry [m][j][q] = w_j P_{m+q}^m(t_j); row q = par + 2 (16 u + l16),
  // clamped into the padded row and masked where q >= K
  const T* Pa = PwT + static_cast<int64_t>(m) * D.J4 * D.L16;
  int qe[MH], qo[MH];
#pragma unroll
  for (int u = 0; u < MH; ++u) {
    qe[u] = 2 * (16 * u + l16);
    qo[u] = qe[u] + 1;
  }
  acc_t ae[MH][NTA], ao[MH][NTA];
#pragma unroll
  for (int u = 0; u < MH; ++u)
#pragma unroll
    for (int nt = 0; nt < NTA; ++nt) {
      ae[u][nt] = zero_acc<acc_t>();
      ao[u][nt] = zero_acc<acc_t>();
    }
  const int nst = (nh + 3) / 4;
  // step t: node j = 4t + kk (rows past nh read node nh - 1, zero weight)
  auto load = [&](int t, T (&a)[2][MH], T (&bu)[NTA], T (&bv)[NTA])
      __attribute__((always_inline)) {
    const int j = min(4 * t + kk, nh - 1);
    const int jm = D.n_theta - 1 - j;
#pragma unroll
    for (int u = 0; u < MH; ++u) {
      if (u < nme) a[0][u] = Pa[j * D.L16 + min(qe[u], D.L16 - 1)];
      if (u < nmo) a[1][u] = Pa[j * D.L16 + min(qo[u], D.L16 - 1)];
    }
    T x[NTA], y[NTA];
    load_vec<T, NTA>(gbl + j * jstride, x);
    load_vec<T, NTA>(gbl + jm * jstride, y);
    const bool mid = jm == j;
#pragma unroll
    for (int nt = 0; nt < NTA; ++nt) {
      bu[nt] = mid ? x[nt] : x[nt] + y[nt];
      bv[nt] = mid ? T(0) : x[nt] - y[nt];
    }
  };
  auto mma_step = [&](int t, const T (&a)[2][MH], const T (&bu)[NTA], const T (&bv)[NTA])
      __attribute__((always_inline)) {
    const bool okj = 4 * t + kk < nh;
#pragma unroll
    for (int u = 0; u < MH; ++u) {
      if (u < nme) {
        const T av = okj && qe[u] < K ? a[0][u] : T(0);
#pragma unroll
        for (int nt = 0; nt < NTA; ++nt) ae[u][nt] = MF<T>::mma(av, bu[nt], ae[u][nt]);
      }
      if (u < nmo) {
        const T av = okj && qo[u] < K ? a[1][u] : T(0);
#pragma unroll
        for (int nt = 0; nt < NTA; ++nt) ao[u][nt] = MF<T>::mma(av, bv[nt], ao[u][nt]);
      }
    }
  };
  // CH steps per chunk, loaded together, the next chunk in flight
  const int nch = (nst + CH - 1) / CH;
  T ca[CH][2][MH], cu[CH][NTA], cv[CH][NTA], na[CH][2][MH], nu[CH][NTA], nv[CH][NTA];
#pragma unroll
  for (int t = 0; t < CH; ++t) load(t, ca[t], cu[t], cv[t]);
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) {
#pragma unroll
      for (int t = 0; t < CH; ++t) load((c + 1) * CH + t, na[t], nu[t], nv[t]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) mma_step(c * CH + t, ca[t], cu[t], cv[t]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
#pragma unroll
      for (int u = 0; u < MH; ++u) {
        ca[t][0][u] = na[t][0][u];
        ca[t][1][u] = na[t][1][u];
      }
#pragma unroll
      for (int nt = 0; nt < NTA; ++nt) {
        cu[t][nt] = nu[t][nt];
        cv[t][nt] = nv[t][nt];
      }
    }
  }
  if (!colok) return;
  T* Ar = A + static_cast<int64_t>(r) * D.LL * D.kp + i0 + NTA * l16;
#pragma unroll
  for (int u = 0; u < MH; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 2 * (16 * u + MF<T>::row(lane, v));
      const int le = m + q, lo = le + 1;
      T pe[NTA], po[NTA];
#pragma unroll
      for (int nt = 0; nt < NTA; ++nt) {
        pe[nt] = ae[u][nt][v];
        po[nt] = ao[u][nt][v];
      }
      if (u < nme && le < D.L) store_vec<T, NTA, NTS>(Ar + (le * le + le + sgn * m) * D.kp, pe);
      if (u < nmo && lo < D.L) store_vec<T, NTA, NTS>(Ar + (lo * lo + lo + sgn * m) * D.kp, po);
    }
  }
}


// ------------------------------------------------------------- density

// Density from the Legendre-synthesis output g[r][j][s][i] (Section 2.2.5):
//   psi_i(r, j, p) = sum_s trig[s][p] g[r][j][s][i],
//   rho[r][j][p]   = 2 sum_i occ_i psi_i(r, j, p)^2,
// the phi synthesis of each (r, theta_j) row as a GEMM on MFMA (M = phi
// points, K = the cos and sin halves of the slots laid out as in the phi
// stage, N = orbitals in 32-column blocks) with each psi tile squared,
// weighted and summed over its columns in FP64.  Only the points p <= n_phi/2
// are formed, their cos part C and sin part S kept apart: since
// cos(m (n - p)) = cos(m p) and sin(m (n - p)) = -sin(m p), the mirror point
// has psi(n - p) = C - S next to psi(p) = C + S (p = 0 and p = n/2 are their
// own mirrors).  Persistent workgroups walk
// the rows; the (row, column block) g tile goes through LDS with the next one
// in registers.  The A operand cos / sin(2 pi m p / n_phi) is read from a
// table of the n_phi angles, its index (m p) mod n_phi advanced by 4p per
// k-step.  Each wave owns the M tiles wave + 4u and adds their column sums to
// an LDS row of rho, written out when the row is done.
constexpr int kDensityWorkgroups = 1024;

template <typename T, int LP>
__global__ __launch_bounds__(256) void k_density_phi(const T* __restrict__ g,
                                                     const double* __restrict__ occ,
                                                     double* __restrict__ rho,
                                                     const double* __restrict__ cs, AngDims D,
                                                     int n_phi, int k, int64_t n_rows) {
  typedef typename MF<T>::acc acc_t;
  constexpr int GW = 16 * PS_NT + 1;
  constexpr int K2 = 2 * LP, KPH = LP / 4;
  constexpr int GPT = K2 / 8;                   // g values per thread per tile
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int S = D.S, L = D.L;
  double* racc = reinterpret_cast<double*>(smem_raw);            // [n_phi]
  T* ct = reinterpret_cast<T*>(racc + n_phi);                    // [2][n_phi] cos | sin
  T* gs = ct + 2 * n_phi;                                        // [K2][GW]
  const int tid = threadIdx.x;
  const int ii = tid & 31, kr = tid >> 5;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, kk = lane >> 4;
  const int ncb = (D.kp + 16 * PS_NT - 1) / (16 * PS_NT);
  const int phalf = n_phi / 2;                  // points 0..phalf are formed
  const int nMT = (phalf + 1 + 15) / 16;
  for (int e = tid; e < 2 * n_phi; e += 256) ct[e] = static_cast<T>(cs[e]);
  // this thread's g rows (slot s < L -> K row s; slot L + j -> row LP + j)
  int sof[GPT];
  bool sok[GPT];
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const int kx = kr + 8 * u;
    const bool sn = kx >= LP;
    const int kl = sn ? kx - LP : kx;
    sok[u] = sn ? kl < L - 1 : kl < L;
    sof[u] = sok[u] ? (sn ? L + kl : kl) * D.kp : 0;
  }
  const int64_t rstride = static_cast<int64_t>(S) * D.kp;
  const int64_t ntask = n_rows * ncb;
  T gp[GPT];
  auto fetch = [&](int64_t task) {
    const int64_t row = task / ncb;
    const int cb = static_cast<int>(task - row * ncb);
    const int col = min(cb * 16 * PS_NT + ii, D.kp - 1);
    const T* gr = g + row * rstride + col;
#pragma unroll
    for (int u = 0; u < GPT; ++u) gp[u] = gr[sof[u]];
  };
  int64_t task = static_cast<int64_t>(blockIdx.x) * ncb;   // first column block of a row
  if (task < ntask) fetch(task);
  for (int64_t row = blockIdx.x; row < n_rows; row += gridDim.x) {
    for (int e = tid; e < n_phi; e += 256) racc[e] = 0.0;
    for (int cb = 0; cb < ncb; ++cb) {
      const int i0 = cb * 16 * PS_NT;
      const bool ok_col = i0 + ii < D.kp;
#pragma unroll
      for (int u = 0; u < GPT; ++u) gs[(kr + 8 * u) * GW + ii] = sok[u] && ok_col ? gp[u] : T(0);
      __syncthreads();   // gs (and, at cb = 0, the zeroed racc and the tables) visible
      const int64_t next = cb + 1 < ncb ? row * ncb + cb + 1 : (row + gridDim.x) * ncb;
      if (next < ntask) fetch(next);                  // next tile, in flight
      // column weights 2 occ_i of this lane's columns (0 past k)
      double wcol[PS_NT];
#pragma unroll
      for (int nt = 0; nt < PS_NT; ++nt) {
        const int i = i0 + nt * 16 + l16;
        wcol[nt] = i < k ? 2.0 * occ[i] : 0.0;
      }
      for (int mt = wave; mt < nMT; mt += 4) {
        const int p = mt * 16 + l16;
        const int pc = p <= phalf ? p : 0;            // padded rows: any finite value
        const int d4 = (4 * pc) % n_phi;
        acc_t acc[2][PS_NT];                          // [cos part, sin part]
#pragma unroll
        for (int half = 0; half < 2; ++half)
#pragma unroll
          for (int nt = 0; nt < PS_NT; ++nt) acc[half][nt] = zero_acc<acc_t>();
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          // m = 4t + kk (cos half) or 4t + kk + 1 (sin half): u = (m p) mod n_phi
          int u = ((kk + half) * pc) % n_phi;
          const T* tb = ct + half * n_phi;
          const T* grow = gs + (half * LP + kk) * GW + l16;
#pragma unroll
          for (int t = 0; t < KPH; ++t) {
            const T a = tb[u];
#pragma unroll
            for (int nt = 0; nt < PS_NT; ++nt)
              acc[half][nt] = MF<T>::mma(a, grow[4 * t * GW + nt * 16], acc[half][nt]);
            u += d4;
            u -= u >= n_phi ? n_phi : 0;
          }
        }
        // psi(p) = C + S and psi(n - p) = C - S: weighted squares summed over
        // this lane's columns, then over the 16 lanes of a row
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double sp = 0.0, sm = 0.0;
#pragma unroll
          for (int nt = 0; nt < PS_NT; ++nt) {
            const double c = static_cast<double>(acc[0][nt][v]);
            const double sn = static_cast<double>(acc[1][nt][v]);
            const double xp = c + sn, xm = c - sn;
            sp = fma(wcol[nt] * xp, xp, sp);
            sm = fma(wcol[nt] * xm, xm, sm);
          }
#pragma unroll
          for (int off = 1; off < 16; off <<= 1) {
            sp += __shfl_xor(sp, off, 64);
            sm += __shfl_xor(sm, off, 64);
          }
          const int pr = mt * 16 + MF<T>::row(lane, v);
          if (l16 == 0 && pr <= phalf) {
            racc[pr] += sp;
            if (pr > 0 && 2 * pr != n_phi) racc[n_phi - pr] += sm;
          }
        }
      }
      __syncthreads();   // gs is refilled next; racc complete after the last block
    }
    double* out = rho + row * n_phi;
    for (int e = tid; e < n_phi; e += 256) out[e] = racc[e];
    __syncthreads();   // racc is zeroed for the next row
  }
}

// Column-block phi transforms between grid functions (column i at f + i ldf,
// [r][theta_j][p]) and the Legendre stages' slot layout g[r][j][s][kp]: the
// SCF potential and density coefficients (one column, kp = 16) and
// ces_to_grid / ces_from_grid (k columns).  A workgroup takes four (r, theta_j)
// rows of one column, one per wave; the angle table cos | sin(2 pi u / n_phi)
// sits in LDS, and with n_phi <= kOneRowLds also the wave's input row, so the
// inner loops read LDS only.
constexpr int kOneRowLds = 1024;

// f_i[r][j][p] = sum_s g[r][j][s][i] trig[s][p]; lane p walks the slots with
// index (m p) mod n_phi.
__global__ __launch_bounds__(256) void k_phi_synthesis_cols(const double* __restrict__ g,
                                                            int kp, double* __restrict__ f,
                                                            int64_t ldf,
                                                            const double* __restrict__ cs,
                                                            int L, int n_phi, int64_t n_rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ct = reinterpret_cast<double*>(smem_raw);           // [2][n_phi]
  double* gw = ct + 2 * n_phi;                                 // [4][S] slot values per wave
  const int S = 2 * L - 1;
  const int i = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < 2 * n_phi; e += 256) ct[e] = cs[e];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  double* gv = gw + wave * S;
  if (row < n_rows)
    for (int e = lane; e < S; e += 64) gv[e] = g[(row * S + e) * kp + i];
  __syncthreads();
  if (row >= n_rows) return;
  double* fo = f + static_cast<int64_t>(i) * ldf + row * n_phi;
  for (int p = lane; p < n_phi; p += 64) {
    double acc = 0.0;
    int u = 0;                                   // cos part, m = 0..L-1
#pragma unroll 4
    for (int m = 0; m < L; ++m) {
      acc = fma(gv[m], ct[u], acc);
      u += p;
      u -= u >= n_phi ? n_phi : 0;
    }
    u = p;                                       // sin part, m = 1..L-1 at slot L - 1 + m
#pragma unroll 4
    for (int m = 1; m < L; ++m) {
      acc = fma(gv[L - 1 + m], ct[n_phi + u], acc);
      u += p;
      u -= u >= n_phi ? n_phi : 0;
    }
    fo[p] = acc;
  }
}

// g[r][j][s][i] = (2 pi / n_phi) sum_p f_i[r][j][p] trig[s][p] for the k
// columns; the workgroups of the last column also zero columns k .. kp-1.
// Lane s walks p with index (m p) mod n_phi.
__global__ __launch_bounds__(256) void k_phi_analysis_cols(const double* __restrict__ f,
                                                           int64_t ldf, int k, int kp,
                                                           double* __restrict__ gh,
                                                           const double* __restrict__ cs,
                                                           int L, int n_phi, int64_t n_rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ct = reinterpret_cast<double*>(smem_raw);           // [2][n_phi]
  double* fw = ct + 2 * n_phi;                                 // [4][n_phi] when staged
  const int S = 2 * L - 1;
  const int i = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool staged = n_phi <= kOneRowLds;
  for (int e = threadIdx.x; e < 2 * n_phi; e += 256) ct[e] = cs[e];
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  const double* fr = f + static_cast<int64_t>(i) * ldf + row * n_phi;
  if (staged && row < n_rows)
    for (int e = lane; e < n_phi; e += 64) fw[wave * n_phi + e] = fr[e];
  __syncthreads();
  if (row >= n_rows) return;
  const double* fv = staged ? fw + wave * n_phi : fr;
  const double dphi = 2.0 * M_PI / n_phi;
  for (int s = lane; s < S; s += 64) {
    const int m = s < L ? s : s - L + 1;
    const double* tb = ct + (s < L ? 0 : n_phi);
    double acc = 0.0;
    int u = 0;
#pragma unroll 4
    for (int p = 0; p < n_phi; ++p) {
      acc = fma(fv[p], tb[u], acc);
      u += m;
      u -= u >= n_phi ? n_phi : 0;
    }
    double* o = gh + (row * S + s) * kp;
    o[i] = dphi * acc;
    if (i == k - 1)
      for (int c = k; c < kp; ++c) o[c] = 0.0;
  }
}

}  // namespace

template <typename T>
void launch_legendre_synth(const Basis& b, const DevTables<T>& tb, const T* G, T* gbuf, int kp,
                           hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  if (b.L > 32) {
    // folded in theta: JT 16-row tiles of the first half of the nodes per wave
    const int nh = (b.n_theta + 1) / 2;
    const int ntile = (nh + 15) / 16;
    // one theta tile per wave: with a lane's columns read as one vector,
    // two tiles per wave sharing each G fragment no longer pay for the
    // occupancy they cost (309 atoms, six tiles: 10.3 ms with one against
    // 10.8 with two, at two and five waves per SIMD)
    constexpr int CH = 4;
    const bool nts = stream_stores<T>(size_t(b.n_r) * b.n_theta * D.S * kp);
    auto go = [&](auto nt_tag, int n_ic) {
      constexpr int NT = decltype(nt_tag)::value;
      dim3 grid(b.n_r * n_ic, (ntile + 3) / 4, D.S);
      with_nts(nts, [&](auto nts_tag) {
        constexpr bool NTS = decltype(nts_tag)::value;
        k_legendre_synth_fold<T, NT, 1, CH, NTS><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic, nh);
      });
    };
    // 16-column tiles per workgroup: four in FP32 on wide blocks (147 atoms:
    // 1.95 against 2.13 ms with two; 309 atoms, with each lane's four
    // columns read and written as one vector: 10.7 against 11.5 ms), else
    // two (FP64 at 309 atoms: 19.9 against 24.1 ms, more waves resident)
    if (sizeof(T) == 4 && kp > 32)
      return go(std::integral_constant<int, 4>(), (kp + 63) / 64);
    return go(std::integral_constant<int, 2>(), (kp + 31) / 32);
  }
  // two column tiles when the block is narrow (no idle MFMA columns), else four
  // (K loops of up to 8 k-steps, L <= 32, load all their operands at once;
  // up to 16 (L <= 64) in FP32, where the registers allow it)
  // In FP32 with 32 < L <= 64, wide blocks (four column tiles) take up to four
  // 64-row theta groups per workgroup, so each G fragment is read once per
  // wave for all of them (measured faster there; slower in FP64 and for the
  // streamed K loop, where the g stores rather than the G reads bound it).
  const int ngrp = (b.n_theta + 63) / 64;
  auto go = [&](auto nt_tag, auto jt_tag, int n_ic) {
    constexpr int NT = decltype(nt_tag)::value, JT = decltype(jt_tag)::value;
    dim3 grid(b.n_r * n_ic, (ngrp + JT - 1) / JT, D.S);
    if constexpr (JT > 1) {
      k_legendre_synth<T, NT, 16, JT><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic);
    } else {
      if (b.L <= 32) {
        k_legendre_synth<T, NT, 8, 1><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic);
        return;
      }
      if constexpr (sizeof(T) == 4) {
        if (b.L <= 64) {
          k_legendre_synth<T, NT, 16, 1><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic);
          return;
        }
      }
      k_legendre_synth<T, NT, 0, 1><<<grid, 256, 0, s>>>(tb.Pm, G, gbuf, D, n_ic);
    }
  };
  using I = std::integral_constant<int, 1>;
  if (kp <= 32) return go(std::integral_constant<int, 2>(), I(), (kp + 31) / 32);
  const int n_ic = (kp + 63) / 64;
  std::integral_constant<int, 4> nt4;
  if constexpr (sizeof(T) == 4) {
    if (b.L > 32 && b.L <= 64) {
      switch (std::min(ngrp, 4)) {
        case 1: return go(nt4, I(), n_ic);
        case 2: return go(nt4, std::integral_constant<int, 2>(), n_ic);
        case 3: return go(nt4, std::integral_constant<int, 3>(), n_ic);
        default: return go(nt4, std::integral_constant<int, 4>(), n_ic);
      }
    }
  }
  go(nt4, I(), n_ic);
}

template <typename T>
void launch_phi_stage(const Basis& b, const T* ab, T* gbuf, int kp, hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  const bool nts = stream_stores<T>(size_t(b.n_r) * b.n_theta * D.S * kp);
  // each workgroup walks about kPhiRowsPerWg (r, theta_j) rows with a stride
  // of the grid, prefetching the next row while the current one runs on
  // MFMA; many short workgroups leave no partly filled last round (309
  // atoms: 22.0 against 22.2 ms with 1792 long-lived ones).  The column
  // block is the fast grid index, so the workgroups dispatched together
  // cover whole rows of g (147 atoms: 3.04 -> 2.82 ms; 309: 20.4 -> 20.1)
  const int64_t n_rows = int64_t(b.n_r) * b.n_theta;
  const int ncg = (kp + 16 * PS_NT - 1) / (16 * PS_NT);
  // rows per workgroup: up to kPhiRowsPerWg while the grid keeps at least
  // kPhiMinWgs workgroups (13 atoms, one column block: 2 rows, 2790
  // workgroups; with 16 rows its 349 workgroups left most CUs idle)
  const int64_t rpw = std::max<int64_t>(
      1, std::min<int64_t>(kPhiRowsPerWg, n_rows * ncg / kPhiMinWgs));
  const int64_t want = (n_rows + rpw - 1) / rpw;
  dim3 grid(ncg, static_cast<unsigned>(std::min<int64_t>(want, 65535)));
  const size_t lds = (6 * size_t(2 * D.L16) + size_t(2 * D.L16) * (16 * PS_NT)) * sizeof(T);
  // K rows that hold slots: rup(L, 4) of the cos block, rup(L - 1, 4) of the
  // sin block; with L in (LP - 16, LP] that is LP - 4 TC and 4 SS fewer
  const int kend0 = rup(D.L, 4), kend1 = rup(D.L - 1, 4);
  const int tc = (D.L16 - kend0) / 4, ss = (kend0 - kend1) / 4;
  auto go = [&](auto lp_tag) {
    constexpr int LP = decltype(lp_tag)::value;
    with_nts(nts, [&](auto nts_tag) {
      constexpr bool NTS = decltype(nts_tag)::value;
      switch (tc * 2 + ss) {
        case 0: k_phi_stage<T, LP, 0, 0, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 1: k_phi_stage<T, LP, 0, 1, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 2: k_phi_stage<T, LP, 1, 0, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 3: k_phi_stage<T, LP, 1, 1, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 4: k_phi_stage<T, LP, 2, 0, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 5: k_phi_stage<T, LP, 2, 1, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        case 6: k_phi_stage<T, LP, 3, 0, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
        default: k_phi_stage<T, LP, 3, 1, NTS><<<grid, 256, lds, s>>>(gbuf, ab, D, n_rows); break;
      }
    });
  };
  switch (D.L16) {   // L <= 96 (checked at basis creation)
    case 16: go(std::integral_constant<int, 16>()); break;
    case 32: go(std::integral_constant<int, 32>()); break;
    case 48: go(std::integral_constant<int, 48>()); break;
    case 64: go(std::integral_constant<int, 64>()); break;
    case 80: go(std::integral_constant<int, 80>()); break;
    default: go(std::integral_constant<int, 96>()); break;
  }
}

template <typename T>
void launch_legendre_analysis(const Basis& b, const DevTables<T>& tb, const T* gbuf, T* A,
                              int kp, hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  const bool nts = stream_stores<T>(size_t(b.n_r) * D.LL * kp);
  const int n_ic = (kp + 16 * LA_NT - 1) / (16 * LA_NT);
  dim3 grid(b.n_r * n_ic, (D.S + LA_SW - 1) / LA_SW);
  constexpr bool f32 = sizeof(T) == 4;
  if (b.L > 32) {   // folded in theta; l-tiles of each parity cover ceil(L/2)
    // FP32 on wide blocks: 64 columns per wave share each table fragment
    // (309 atoms, kp = 1008: 8.85 -> 8.0 ms; 147 atoms, kp = 400, measured
    // slower); FP64 keeps 32 (64 measured slower)
    const int nh = (b.n_theta + 1) / 2;
    auto go = [&](auto nta_tag) {
      constexpr int NTA = decltype(nta_tag)::value;
      const int n_icf = (kp + 16 * NTA - 1) / (16 * NTA);
      dim3 gridf(b.n_r * n_icf, (D.S + LA_SW - 1) / LA_SW);
      with_nts(nts, [&](auto nts_tag) {
        constexpr bool NTS = decltype(nts_tag)::value;
        if (b.L <= 64)
          k_legendre_analysis_fold<T, 2, f32 ? 4 : 2, NTA, NTS><<<gridf, 256, 0, s>>>(
              tb.PwT, gbuf, A, D, n_icf, nh);
        else
          k_legendre_analysis_fold<T, 3, 2, NTA, NTS><<<gridf, 256, 0, s>>>(tb.PwT, gbuf, A, D,
                                                                            n_icf, nh);
      });
    };
    if (f32 && kp >= 512)
      go(std::integral_constant<int, 4>());
    else
      go(std::integral_constant<int, 2>());
    return;
  }
  // l-tiles per slot cover L; theta chunks sized to the registers left
  if (b.L <= 32) {
    if (b.n_theta <= 64)
      k_legendre_analysis<T, 2, 16, true><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, D, n_ic);
    else
      k_legendre_analysis<T, 2, 8, false><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, D, n_ic);
  } else if (b.L <= 64) {
    k_legendre_analysis<T, 4, f32 ? 8 : 4, false><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, D, n_ic);
  } else {   // L <= 96
    k_legendre_analysis<T, 6, f32 ? 4 : 2, false><<<grid, 256, 0, s>>>(tb.PwT, gbuf, A, D, n_ic);
  }
}

template <typename T>
void launch_density_phi(const Basis& b, const T* gbuf, const double* occ, double* rho, int k,
                        int kp, hipStream_t s) {
  const AngDims D = ang_dims(b, kp);
  const int64_t n_rows = int64_t(b.n_r) * b.n_theta;
  dim3 grid(static_cast<unsigned>(std::min<int64_t>(n_rows, kDensityWorkgroups)));
  const size_t lds = size_t(b.n_phi) * sizeof(double) + 2 * size_t(b.n_phi) * sizeof(T) +
                     size_t(2 * D.L16) * (16 * PS_NT + 1) * sizeof(T);
  auto go = [&](auto kern) {
    // large n_phi needs more than the default 64 KB (set per kernel: the
    // instantiations share one function-pointer type, so no static flag)
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    kern<<<grid, 256, lds, s>>>(gbuf, occ, rho, b.dev_cs, D, b.n_phi, k, n_rows);
  };
  switch (D.L16) {   // L <= 96 (checked at basis creation)
    case 16: go(&k_density_phi<T, 16>); break;
    case 32: go(&k_density_phi<T, 32>); break;
    case 48: go(&k_density_phi<T, 48>); break;
    case 64: go(&k_density_phi<T, 64>); break;
    case 80: go(&k_density_phi<T, 80>); break;
    default: go(&k_density_phi<T, 96>); break;
  }
}

void launch_phi_synthesis_cols(const Basis& b, const double* g, int k, int kp, double* f,
                               int64_t ldf, hipStream_t s) {
  const int64_t n_rows = int64_t(b.n_r) * b.n_theta;
  const size_t lds = (2 * size_t(b.n_phi) + 4 * (2 * size_t(b.L) - 1)) * sizeof(double);
  k_phi_synthesis_cols<<<dim3(static_cast<unsigned>((n_rows + 3) / 4), k), 256, lds, s>>>(
      g, kp, f, ldf, b.dev_cs, b.L, b.n_phi, n_rows);
}

void launch_phi_analysis_cols(const Basis& b, const double* f, int64_t ldf, int k, int kp,
                              double* gh, hipStream_t s) {
  const int64_t n_rows = int64_t(b.n_r) * b.n_theta;
  const size_t lds = (2 * size_t(b.n_phi) + (b.n_phi <= kOneRowLds ? 4 * size_t(b.n_phi) : 0)) *
                     sizeof(double);
  k_phi_analysis_cols<<<dim3(static_cast<unsigned>((n_rows + 3) / 4), k), 256, lds, s>>>(
      f, ldf, k, kp, gh, b.dev_cs, b.L, b.n_phi, n_rows);
}

void launch_phi_synthesis_one(const Basis& b, const double* g, double* f, hipStream_t s) {
  launch_phi_synthesis_cols(b, g, 1, kColPad, f, b.n_grid, s);
}

void launch_phi_analysis_one(const Basis& b, const double* f, double* gh, hipStream_t s) {
  launch_phi_analysis_cols(b, f, b.n_grid, 1, kColPad, gh, s);
}

#define CES_INST(T)                                                                          \
  template void launch_legendre_synth<T>(const Basis&, const DevTables<T>&, const T*, T*, int, \
                                         hipStream_t);                                       \
  template void launch_phi_stage<T>(const Basis&, const T*, T*, int, hipStream_t);             \
  template void launch_legendre_analysis<T>(const Basis&, const DevTables<T>&, const T*, T*,   \
                                            int, hipStream_t);                                 \
  template void launch_density_phi<T>(const Basis&, const T*, const double*, double*, int, int,  \
                                      hipStream_t);
CES_INST(float)
CES_INST(double)
#undef CES_INST


}  // namespace ces
