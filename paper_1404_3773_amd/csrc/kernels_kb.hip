// Kleinman-Bylander projector products of H*X (Section 2.3.2):
//   kb_gemm   C[q][i] = h_q sum_alpha P[q][alpha] Y[alpha][i]   (M = n_proj, N = k, K = d)
//   kb_apply  Z[alpha][i] = sum_q P[q][alpha] C[q][i]          (M = k, N = d, K = n_proj)
// Z is added in the radial forward kernel's epilogue.
//
// kb_gemm:
// Both operands run contiguously along the contraction index alpha (P is
// stored n_proj x d row-major, Y column-major): a workgroup stages a BM x BK
// tile of P and a BN x BK tile of Y per step in LDS, loaded as whole row
// segments (consecutive lanes on consecutive alpha), the next step's tiles
// in registers while the current one runs on 16x16x4 MFMA (2 x 2 waves, TM x
// TN fragments each).  K is split into chunks whose partial products go to a
// buffer; a second kernel sums them in a fixed order and applies h.
// Workgroup ids are dealt round-robin over the 8 XCDs.  With xcd_chunk set
// (a chunk count that is a multiple of 8) every workgroup of a chunk (all
// its M and N tiles) is placed on XCD chunk mod 8, in M-tile order, so the
// workgroups in flight on an XCD walk the same chunk's alpha steps together:
// its L2 serves the Y steps they share (all M tiles) and the P steps (all N
// tiles of an M tile), and each is fetched from HBM about once.  Otherwise
// the groups (chunk, M tile) of nN workgroups are dealt round-robin over the
// XCDs, which keeps all of them busy for any chunk count.  FP32 operands with
// 16-byte aligned rows are staged 64 alpha per step from 16-byte loads into
// one LDS buffer (309 atoms: 22.9 -> 20.8 ms against 32 alpha per step from
// 4-byte loads, double-buffered; 32 per step from 16-byte loads,
// double-buffered, 22.1 ms; 32 per step single-buffered at three waves per
// SIMD, 21.4 ms; wave tiles of 128 x 64 with 16 or 32 alpha per step, 22.7
// ms or slower).  FP64 operands with even leading dimensions and
// 16-byte aligned bases are staged from 16-byte loads (2 doubles; 309 atoms:
// 48.9 -> 45.4 ms), the Gram products of Cholesky-QR and Rayleigh-Ritz too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "ces_internal.h"
#include "mfma.h"

namespace ces {
namespace {

template <typename T>
struct KbShape;
template <>
struct KbShape<float> {   // wave tile 64 x 64, workgroup 128 x 128, 32 alpha per step
  static constexpr int KB = 32, TM = 4, TN = 4;
};
template <>
struct KbShape<double> {  // wave tile 64 x 32, workgroup 128 x 64, 32 alpha per step
  static constexpr int KB = 32, TM = 4, TN = 2;
};
// C = P^T Y, FP32 with 16-byte aligned rows: the same 128 x 128 workgroup
// tiles, 64 alpha per step staged from 16-byte loads (each row's segment of
// a step is two whole 128-byte lines) into one LDS buffer (69.6 KB, two
// workgroups per CU).
struct KgVec {
  static constexpr int KB = 64, TM = 4, TN = 4;
};
constexpr int kKbPerXcd = 64;   // resident workgroups per XCD (32 CUs, 2 each)

// LDS row pitch of the staged tiles: the MFMA operand reads take 16 rows x 4
// consecutive alpha (rows c16, columns kk); with pitch KB + 2 (FP32) the 64
// lanes of a read fall on distinct banks, where KB + 1 left them two-way
// (309-atom C = P^T Y: 25.4 -> 24.5 ms).  FP64 reads 8-byte words and keeps
// KB + 1 (its C was slower with KB + 2).
// Rows staged from 16-byte loads take an aligned pitch: FP32 (vw = 4) KB + 4,
// which spreads the operand reads the same way (64 alpha per step: rows c16
// start 4 c16 banks apart); FP64 (vw = 2) KB + 2, where the faster staging
// outweighs the slower reads.
template <typename T>
constexpr int kb_pitch(int kb, int vw = 1) {
  return kb + (sizeof(T) == 4 ? (vw > 1 ? 4 : 2) : (vw > 1 ? 2 : 1));
}

// With DB the P and Y tiles are double-buffered in (dynamic) LDS: a step
// computes from one buffer while the next step's tiles are written into the
// other, so it takes one barrier instead of two.
// S: KB alpha per step, TM x TN fragments per wave; VW: alpha per staging
// load (1, or 4 with 16-byte aligned rows: fewer row addresses to hold).
template <typename T, bool DB, typename S, int VW>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(VW == 4 ? 2 : 1, 8)))
void k_kb_gemm(const T* __restrict__ P, int64_t d, int64_t ldp, const T* __restrict__ Y,
               int64_t ldy, T* __restrict__ part, int n_proj, int k, int kp, int64_t kchunk,
               int nM, int nN, int nchunk, int xcd_chunk) {
  typedef typename MF<T>::acc acc_t;
  constexpr int KB = S::KB, TM = S::TM, TN = S::TN;
  constexpr int BM = 32 * TM, BN = 32 * TN;      // 2 x 2 waves
  constexpr int KW = kb_pitch<T>(KB, VW);        // padded LDS row
  static_assert(KW % VW == 0, "vector LDS writes need an aligned row pitch");
  constexpr int KV = KB / VW;                    // threads per tile row
  constexpr int RA = 256 / KV;                   // tile rows loaded per pass
  constexpr int LA = BM / RA, LB = BN / RA;      // passes for the P and Y tiles
  constexpr int STAGE = (BM + BN) * KW;          // one buffer: A tile then B tile
  extern __shared__ __align__(16) unsigned char kb_smem[];
  T* const lds = reinterpret_cast<T*>(kb_smem);
  // workgroup id -> (XCD x, position j on it) -> (t-th group of XCD x, N tile)
  // -> (chunk x + 8 (t / nM), M tile t % nM), or group x + 8 t = (chunk, M tile)
  const int id = blockIdx.x;
  const int x = id & 7, j = id >> 3;
  const int t = j / nN, ntb = j - t * nN;
  int chunk, mtb;
  if (xcd_chunk) {
    const int cx = t / nM;
    mtb = t - cx * nM;
    chunk = x + 8 * cx;
  } else {
    const int g = x + 8 * t;
    chunk = g / nM;
    mtb = g - chunk * nM;
  }
  if (chunk >= nchunk) return;
  const int64_t k0 = static_cast<int64_t>(chunk) * kchunk;
  const int64_t k1 = k0 + kchunk < d ? k0 + kchunk : d;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int c16 = lane & 15, kk = lane >> 4;
  // staging: thread -> (tile row r0 + RA p, alpha offset kc .. kc + VW - 1);
  // row addresses are formed per load (fewer registers held)
  const int kc = VW * (tid % KV), r0 = tid / KV;
  const int arow0 = mtb * BM + r0, bcol0 = ntb * BN + r0;
  // loads read clamped addresses and are masked when stored to LDS (a
  // select on a load makes the wave wait for it, which would serialise the
  // next step's loads); a vector past k1 is clamped to the last aligned one
  // (inside the rows, whose lengths are multiples of VW)
  T ra[LA][VW], rb[LB][VW];
  auto fetch = [&](int64_t kb) {
    const int64_t kx = kb + kc;
    const int64_t kcl = kx < k1 ? kx : (k1 - 1) / VW * VW;
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      const int row = arow0 + RA * p;
      load_vec<T, VW>(P + static_cast<int64_t>(row < n_proj ? row : n_proj - 1) * ldp + kcl, ra[p]);
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      const int col = bcol0 + RA * p;
      load_vec<T, VW>(Y + static_cast<int64_t>(col < k ? col : k - 1) * ldy + kcl, rb[p]);
    }
  };
  acc_t acc[TM][TN];
#pragma unroll
  for (int u = 0; u < TM; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v) acc[u][v] = zero_acc<acc_t>();
  // the staged tiles of step kb into buffer `buf`
  auto stage = [&](int64_t kb, int buf) __attribute__((always_inline)) {
    T* As = lds + buf * STAGE;
    T* Bs = As + BM * KW;
#pragma unroll
    for (int p = 0; p < LA; ++p) {
      const bool okr = arow0 + RA * p < n_proj;
      T w[VW];
#pragma unroll
      for (int e = 0; e < VW; ++e) w[e] = okr && kb + kc + e < k1 ? ra[p][e] : T(0);
      if constexpr (VW == 1)
        As[(r0 + RA * p) * KW + kc] = w[0];
      else
        store_vec<T, VW, false>(As + (r0 + RA * p) * KW + kc, w);
    }
#pragma unroll
    for (int p = 0; p < LB; ++p) {
      const bool okr = bcol0 + RA * p < k;
      T w[VW];
#pragma unroll
      for (int e = 0; e < VW; ++e) w[e] = okr && kb + kc + e < k1 ? rb[p][e] : T(0);
      if constexpr (VW == 1)
        Bs[(r0 + RA * p) * KW + kc] = w[0];
      else
        store_vec<T, VW, false>(Bs + (r0 + RA * p) * KW + kc, w);
    }
  };
  // k-steps [s0, s1) of the staged tiles in buffer `buf`
  auto compute_steps = [&](int buf, int s0, int s1) __attribute__((always_inline)) {
    const T* Aw = lds + buf * STAGE + (wm * 16 * TM + c16) * KW + kk;
    const T* Bw = lds + buf * STAGE + BM * KW + (wn * 16 * TN + c16) * KW + kk;
#pragma unroll
    for (int st = s0; st < s1; ++st) {
      T a[TM], b[TN];
#pragma unroll
      for (int u = 0; u < TM; ++u) a[u] = Aw[16 * u * KW + 4 * st];
#pragma unroll
      for (int v = 0; v < TN; ++v) b[v] = Bw[16 * v * KW + 4 * st];
#pragma unroll
      for (int u = 0; u < TM; ++u)
#pragma unroll
        for (int v = 0; v < TN; ++v) acc[u][v] = MF<T>::mma(a[u], b[v], acc[u][v]);
    }
  };
  auto compute = [&](int buf) __attribute__((always_inline)) { compute_steps(buf, 0, KB / 4); };
  if (k0 < k1) fetch(k0);
  if constexpr (DB) {
    if (k0 < k1) {
      stage(k0, 0);
      if (k0 + KB < k1) fetch(k0 + KB);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t kb = k0; kb < k1; kb += KB) {
      // the other buffer was last read in the previous step, before its
      // barrier: its LDS writes and the next global loads go out between the
      // two halves of this step's MFMAs
      const bool more = kb + KB < k1;
      compute_steps(buf, 0, KB / 8);
      if (more) stage(kb + KB, buf ^ 1);
      compute_steps(buf, KB / 8, KB / 4);
      if (more && kb + 2 * KB < k1) fetch(kb + 2 * KB);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int64_t kb = k0; kb < k1; kb += KB) {
      stage(kb, 0);
      __syncthreads();
      if (kb + KB < k1) fetch(kb + KB);          // next step's tiles, in flight
      compute(0);
      __syncthreads();
    }
  }
  T* pc = part + static_cast<int64_t>(chunk) * n_proj * kp;
#pragma unroll
  for (int u = 0; u < TM; ++u)
#pragma unroll
    for (int v = 0; v < TN; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mtb * BM + wm * 16 * TM + 16 * u + MF<T>::row(lane, r);
        const int col = ntb * BN + wn * 16 * TN + 16 * v + c16;
        if (row < n_proj && col < k) pc[static_cast<int64_t>(row) * kp + col] = acc[u][v][r];
      }
}

// kb_apply: Z^T = C^T P on 16x16x4 MFMA, workgroup tile BM columns i x BN rows
// alpha, both operands staged per step of KB projectors in LDS (C rows run
// along i, P rows along alpha), the next step's tiles in registers.  The
// result lane holds 16 consecutive alpha of one column, so stores are
// coalesced.  Workgroups that read the same P tile (same alpha tile) share
// an XCD.  It serves the operands that the wide-tile kernel below cannot
// load as 16-byte vectors (FP64 projector rows of odd length d).  FP32 is held
// to four waves per SIMD (309 atoms, before the wide tiles: 23.1 -> 22.7 ms;
// three VGPRs spill, outside the K loop), FP64 to three (51.7 -> 46.7 ms, no
// spills).
template <typename T, bool DB, int KB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3, 8)))
void k_kb_apply(const T* __restrict__ P, int64_t d,
                                                  int64_t ldp, const T* __restrict__ C,
                                                  int n_proj, int k, int kp, T* __restrict__ Z,
                                                  int nI, int nA) {
  typedef typename MF<T>::acc acc_t;
  constexpr int TM = KbShape<T>::TM, TN = KbShape<T>::TN;
  constexpr int BM = 32 * TN, BN = 32 * TM;      // i tile, alpha tile (2 x 2 waves)
  constexpr int KW = kb_pitch<T>(KB);
  constexpr int RC = 256 / BM, RP = 256 / BN;    // q rows per staging pass
  constexpr int LC = KB / RC, LP = KB / RP;
  constexpr int STAGE = (BM + BN) * KW;          // one buffer: Cs [i][q] then Ps [alpha][q]
  extern __shared__ __align__(16) unsigned char kb_smem[];
  T* const lds = reinterpret_cast<T*>(kb_smem);
  const int id = blockIdx.x;
  const int x = id & 7, j = id >> 3;
  const int ga = x + 8 * (j / nI), itb = j - (j / nI) * nI;
  if (ga >= nA) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int c16 = lane & 15, kk = lane >> 4;
  const int ci = tid % BM, cq = tid / BM;
  const int pa_ = tid % BN, pq = tid / BN;
  const int i_s = itb * BM + ci;
  const bool iok = i_s < kp;
  const int64_t a_s = static_cast<int64_t>(ga) * BN + pa_;
  const bool aok = a_s < d;
  const T* cbase = C + (iok ? i_s : 0);
  const T* pbase = P + (aok ? a_s : 0);
  T rc[LC], rp[LP];
  // clamped loads, masked when stored to LDS (see k_kb_gemm)
  auto fetch = [&](int q0) {
#pragma unroll
    for (int p = 0; p < LC; ++p) {
      const int q = q0 + cq + RC * p;
      rc[p] = cbase[static_cast<int64_t>(q < n_proj ? q : n_proj - 1) * kp];
    }
#pragma unroll
    for (int p = 0; p < LP; ++p) {
      const int q = q0 + pq + RP * p;
      rp[p] = pbase[static_cast<int64_t>(q < n_proj ? q : n_proj - 1) * ldp];
    }
  };
  acc_t acc[TN][TM];
#pragma unroll
  for (int u = 0; u < TN; ++u)
#pragma unroll
    for (int v = 0; v < TM; ++v) acc[u][v] = zero_acc<acc_t>();
  auto stage = [&](int q0, int buf) __attribute__((always_inline)) {
    T* Cs = lds + buf * STAGE;
    T* Ps = Cs + BM * KW;
#pragma unroll
    for (int p = 0; p < LC; ++p)
      Cs[ci * KW + cq + RC * p] = iok && q0 + cq + RC * p < n_proj ? rc[p] : T(0);
#pragma unroll
    for (int p = 0; p < LP; ++p)
      Ps[pa_ * KW + pq + RP * p] = aok && q0 + pq + RP * p < n_proj ? rp[p] : T(0);
  };
  // k-steps [s0, s1) of the staged tiles in buffer `buf`
  auto compute_steps = [&](int buf, int s0, int s1) __attribute__((always_inline)) {
    const T* Aw = lds + buf * STAGE + (wm * 16 * TN + c16) * KW + kk;
    const T* Bw = lds + buf * STAGE + BM * KW + (wn * 16 * TM + c16) * KW + kk;
#pragma unroll
    for (int st = s0; st < s1; ++st) {
      T a[TN], b[TM];
#pragma unroll
      for (int u = 0; u < TN; ++u) a[u] = Aw[16 * u * KW + 4 * st];
#pragma unroll
      for (int v = 0; v < TM; ++v) b[v] = Bw[16 * v * KW + 4 * st];
#pragma unroll
      for (int u = 0; u < TN; ++u)
#pragma unroll
        for (int v = 0; v < TM; ++v) acc[u][v] = MF<T>::mma(a[u], b[v], acc[u][v]);
    }
  };
  auto compute = [&](int buf) __attribute__((always_inline)) { compute_steps(buf, 0, KB / 4); };
  fetch(0);
  if constexpr (DB) {
    stage(0, 0);
    if (KB < n_proj) fetch(KB);
    __syncthreads();
    int buf = 0;
    for (int q0 = 0; q0 < n_proj; q0 += KB) {
      // the other buffer's LDS writes and the next global loads go out
      // between the two halves of this step's MFMAs (see k_kb_gemm)
      const bool more = q0 + KB < n_proj;
      compute_steps(buf, 0, KB / 8);
      if (more) stage(q0 + KB, buf ^ 1);
      compute_steps(buf, KB / 8, KB / 4);
      if (more && q0 + 2 * KB < n_proj) fetch(q0 + 2 * KB);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int q0 = 0; q0 < n_proj; q0 += KB) {
      stage(q0, 0);
      __syncthreads();
      if (q0 + KB < n_proj) fetch(q0 + KB);
      compute(0);
      __syncthreads();
    }
  }
#pragma unroll
  for (int u = 0; u < TN; ++u)
#pragma unroll
    for (int v = 0; v < TM; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = itb * BM + wm * 16 * TN + 16 * u + MF<T>::row(lane, r);
        const int64_t a = static_cast<int64_t>(ga) * BN + wn * 16 * TM + 16 * v + c16;
        if (i < k && a < d) Z[static_cast<int64_t>(i) * d + a] = acc[u][v][r];
      }
}

// kb_apply, wide tiles.  FP32: workgroup tile 128 columns i x 256 rows alpha,
// 2 x 2 waves of 64 x 128 (4 x 8 MFMA fragments, 128 accumulators per lane),
// so each staged operand value feeds twice the MFMAs of the 64 x 64 wave
// tile.  The projector steps (KA per step) are staged in LDS row-major by
// projector (C rows along i, P rows along alpha) from 16-byte loads and
// 16-byte LDS writes; the MFMA operand reads take 16 consecutive columns of 4
// projector rows whose starts lie 16 banks apart (row pitch = width + 16
// words).  Column loads are clamped into the arrays (rows are padded to a
// multiple of 4): a clamped column only feeds outputs of columns i >= kp or
// alpha >= ldp, which are not stored.  Projector rows past n_proj are
// clamped on load and zeroed in the C tile.  309 atoms (k = 1000, 1236
// projectors): 22.8 ms with the 64 x 64 wave tiles, 19.5 ms here (the same
// result bits: each accumulator takes the projectors in the same order);
// 8, 16 and 32 projectors per step (32 single-buffered) time alike, 32
// double-buffered (one workgroup per CU) 26.3 ms.  Measured and not kept:
// lanes owning 4 adjacent columns so that the operands come as 16-byte LDS
// reads (3 instead of 12 per 4 projectors: 19.5 ms as well), and a raised
// wave priority around the MFMA sections (19.4 -> 19.2 ms here, but C =
// P^T Y 20.6 -> 20.9 and both FP64 products slower).
// FP64 (operands with even rows): 2 x 2 waves of 64 x 64 (4 x 4 fragments),
// 128 x 128 workgroup tiles, 2 doubles per 16-byte access, row pitch width +
// 16 doubles (the 4 projector rows of an operand read start 128 bytes apart
// modulo 256); 309 atoms: 46.5 -> 39.2 ms, the same result bits.
template <typename T>
struct ApShape;
template <>
struct ApShape<float> {
  static constexpr int TI = 4, TA = 8, KA = 16;
};
template <>
struct ApShape<double> {
  static constexpr int TI = 4, TA = 4, KA = 16;
};
constexpr bool kApDB = true;   // double-buffered LDS

template <typename T>
constexpr size_t kb_apply_wide_lds() {
  typedef ApShape<T> S;
  return (kApDB ? 2 : 1) * size_t(S::KA) * (32 * S::TI + 16 + 32 * S::TA + 16) * sizeof(T);
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_kb_apply_wide(const T* __restrict__ P, int64_t d, int64_t ldp, const T* __restrict__ C,
                     int n_proj, int k, int kp, T* __restrict__ Z, int nI, int nA) {
  typedef typename MF<T>::acc acc_t;
  typedef ApShape<T> S;
  constexpr int TI = S::TI, TA = S::TA, KA = S::KA;
  constexpr bool DB = kApDB;
  constexpr int BI = 32 * TI, BA = 32 * TA;     // workgroup tile: i, alpha
  constexpr int PI = BI + 16, PA = BA + 16;     // LDS row pitch (elements)
  constexpr int VW = 16 / static_cast<int>(sizeof(T));   // elements per 16-byte access
  constexpr int STAGE = KA * (PI + PA);
  constexpr int CV = KA * BI / (VW * 256);      // 16-byte C loads per thread per step
  constexpr int PV = KA * BA / (VW * 256);      // 16-byte P loads per thread per step
  constexpr int CR = 256 / (BI / VW), PR = 256 / (BA / VW);   // rows per pass
  static_assert(CV >= 1 && PV >= 1, "step too short for the staging passes");
  extern __shared__ __align__(16) unsigned char kb_smem[];
  T* const lds = reinterpret_cast<T*>(kb_smem);
  const int id = blockIdx.x;
  const int x = id & 7, j = id >> 3;
  const int ga = x + 8 * (j / nI), itb = j - (j / nI) * nI;
  if (ga >= nA) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wa = wave & 1;
  const int c16 = lane & 15, kk = lane >> 4;
  const int cr = tid / (BI / VW), cc = VW * (tid % (BI / VW));
  const int pr = tid / (BA / VW), pc = VW * (tid % (BA / VW));
  const int ic = min(itb * BI + cc, kp - VW);
  const int64_t ac = min(static_cast<int64_t>(ga) * BA + pc, ldp - VW);
  const T* cbase = C + ic;
  const T* pbase = P + ac;
  T rc[CV][VW], rp[PV][VW];
  auto fetch = [&](int q0) {
#pragma unroll
    for (int p = 0; p < CV; ++p) {
      const int q = q0 + cr + CR * p;
      load_vec<T, VW>(cbase + static_cast<int64_t>(q < n_proj ? q : n_proj - 1) * kp, rc[p]);
    }
#pragma unroll
    for (int p = 0; p < PV; ++p) {
      const int q = q0 + pr + PR * p;
      load_vec<T, VW>(pbase + static_cast<int64_t>(q < n_proj ? q : n_proj - 1) * ldp, rp[p]);
    }
  };
  acc_t acc[TI][TA];
#pragma unroll
  for (int u = 0; u < TI; ++u)
#pragma unroll
    for (int v = 0; v < TA; ++v) acc[u][v] = zero_acc<acc_t>();
  auto stage = [&](int q0, int buf) __attribute__((always_inline)) {
    T* Cs = lds + buf * STAGE;
    T* Ps = Cs + KA * PI;
#pragma unroll
    for (int p = 0; p < CV; ++p) {
      const bool ok = q0 + cr + CR * p < n_proj;
      T w[VW];
#pragma unroll
      for (int e = 0; e < VW; ++e) w[e] = ok ? rc[p][e] : T(0);
      store_vec<T, VW, false>(Cs + (cr + CR * p) * PI + cc, w);
    }
#pragma unroll
    for (int p = 0; p < PV; ++p) store_vec<T, VW, false>(Ps + (pr + PR * p) * PA + pc, rp[p]);
  };
  auto compute_steps = [&](int buf, int s0, int s1) __attribute__((always_inline)) {
    const T* Aw = lds + buf * STAGE + kk * PI + wi * 16 * TI + c16;
    const T* Bw = lds + buf * STAGE + KA * PI + kk * PA + wa * 16 * TA + c16;
#pragma unroll
    for (int st = s0; st < s1; ++st) {
      T a[TI], b[TA];
#pragma unroll
      for (int u = 0; u < TI; ++u) a[u] = Aw[4 * st * PI + 16 * u];
#pragma unroll
      for (int v = 0; v < TA; ++v) b[v] = Bw[4 * st * PA + 16 * v];
#pragma unroll
      for (int u = 0; u < TI; ++u)
#pragma unroll
        for (int v = 0; v < TA; ++v) acc[u][v] = MF<T>::mma(a[u], b[v], acc[u][v]);
    }
  };
  fetch(0);
  if constexpr (DB) {
    stage(0, 0);
    if (KA < n_proj) fetch(KA);
    __syncthreads();
    int buf = 0;
    for (int q0 = 0; q0 < n_proj; q0 += KA) {
      const bool more = q0 + KA < n_proj;
      compute_steps(buf, 0, KA / 8);
      if (more) stage(q0 + KA, buf ^ 1);
      compute_steps(buf, KA / 8, KA / 4);
      if (more && q0 + 2 * KA < n_proj) fetch(q0 + 2 * KA);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    for (int q0 = 0; q0 < n_proj; q0 += KA) {
      stage(q0, 0);
      __syncthreads();
      if (q0 + KA < n_proj) fetch(q0 + KA);
      compute_steps(0, 0, KA / 4);
      __syncthreads();
    }
  }
#pragma unroll
  for (int u = 0; u < TI; ++u)
#pragma unroll
    for (int v = 0; v < TA; ++v)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = itb * BI + wi * 16 * TI + 16 * u + MF<T>::row(lane, r);
        const int64_t a = static_cast<int64_t>(ga) * BA + wa * 16 * TA + 16 * v + c16;
        if (i < k && a < d) Z[static_cast<int64_t>(i) * d + a] = acc[u][v][r];
      }
}

// C[q][i] = h_q sum_c part[c][q][i] for i < k (chunks in order), 0 for k <= i < kp.
template <typename T>
__global__ void k_kb_reduce(const T* __restrict__ part, int nchunk, const T* __restrict__ h,
                            T* __restrict__ C, int n_proj, int k, int kp) {
  const int64_t n = static_cast<int64_t>(n_proj) * kp;
  const int64_t stride = n;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int q = static_cast<int>(e / kp), i = static_cast<int>(e - static_cast<int64_t>(q) * kp);
    T s = T(0);
    if (i < k)
      for (int c = 0; c < nchunk; ++c) s += part[c * stride + e];
    C[e] = h[q] * s;
  }
}

struct KbGrid {
  int nM, nN, nchunk;
  int64_t kchunk;
};

// Workgroups of a split-K grid with nchunk chunks: 8 XCDs x their largest
// group count x nN, with whole chunks per XCD (xcd_chunk) or groups dealt
// round-robin.
inline unsigned kb_workgroups(int nchunk, int nM, int nN, bool xcd_chunk) {
  const int per_xcd = xcd_chunk ? (nchunk + 7) / 8 * nM : (nchunk * nM + 7) / 8;
  return static_cast<unsigned>(8 * per_xcd * nN);
}

template <typename S>
KbGrid kb_grid(int n_proj, int k, int64_t d) {
  constexpr int KB = S::KB;
  KbGrid gr;
  gr.nM = (n_proj + 32 * S::TM - 1) / (32 * S::TM);
  gr.nN = (k + 32 * S::TN - 1) / (32 * S::TN);
  // 8 c chunks (c per XCD, each XCD's workgroups c nM nN), c <= 4 chosen so
  // that those workgroups fill whole rounds of kKbPerXcd resident ones as
  // nearly as possible (309 atoms, FP32: nM = 10, nN = 8, c = 4: 5 full
  // rounds); chunks of at least 16 steps
  const int64_t steps = (d + KB - 1) / KB;
  int c_best = 1;
  double waste_best = 2.0;
  for (int c = 1; c <= 4; ++c) {
    if (c > 1 && steps < int64_t(8 * c) * 16) break;
    const int64_t wg = int64_t(c) * gr.nM * gr.nN;
    const int64_t rounds = (wg + kKbPerXcd - 1) / kKbPerXcd;
    const double waste = double(rounds * kKbPerXcd - wg) / double(rounds * kKbPerXcd);
    if (waste < waste_best - 1e-9) {
      waste_best = waste;
      c_best = c;
    }
  }
  const int want = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(8 * c_best, steps)));
  gr.kchunk = round_up((d + want - 1) / want, KB);
  gr.nchunk = static_cast<int>((d + gr.kchunk - 1) / gr.kchunk);
  return gr;
}

}  // namespace

// Split-K partial sums of a product with up to k columns: the chunk count
// grows as the column count falls, so the largest need over every width <= k
// (a narrower call, e.g. a Lanczos vector or the last column chunk).
size_t kb_partial_bytes(int n_proj, int k, int64_t d) {
  if (n_proj <= 0) return 0;
  size_t most = 0;
  for (int kc = 1; kc <= k; ++kc) {
    const size_t kp = size_t(round_up(kc, kColPad));
    const size_t c32 = size_t(std::max(kb_grid<KgVec>(n_proj, kc, d).nchunk,
                                       kb_grid<KbShape<float>>(n_proj, kc, d).nchunk)) *
                       sizeof(float);
    const size_t c64 = size_t(kb_grid<KbShape<double>>(n_proj, kc, d).nchunk) * sizeof(double);
    most = std::max(most, std::max(c32, c64) * size_t(n_proj) * kp);
  }
  return most;
}

// LDS bytes of the projector kernels: one (A tile + B tile) stage, or two when
// double-buffered.  Measured on MI355X (309-atom shape, 32 alpha per step
// from 4-byte loads): double buffering took the FP32 C = P^T Y product from
// 28.3 to 25.4 ms and made P C slower
// (22.3 -> 24.3 ms), so only the former uses it (2 x 33.8 KB, two workgroups
// per CU still fit).
template <typename T>
constexpr size_t kb_lds_bytes(bool db, int kb = KbShape<T>::KB) {
  return (db ? 2 : 1) * size_t(32 * KbShape<T>::TM + 32 * KbShape<T>::TN) * kb_pitch<T>(kb) * sizeof(T);
}
template <typename T, typename S>
constexpr size_t kg_lds_bytes(bool db, int vw) {
  return (db ? 2 : 1) * size_t(32 * S::TM + 32 * S::TN) * kb_pitch<T>(S::KB, vw) * sizeof(T);
}

// Allow more than the default 64 KB of dynamic LDS for a kernel that needs it
// (set per kernel on each launch: no process-wide state).
template <typename K>
void allow_lds(K kern, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename T>
void launch_kb_gemm(const T* P, int64_t d, int64_t ldp, const T* Y, int64_t ldy, const T* h,
                    T* C, T* part, int n_proj, int k, int kp, hipStream_t s) {
  int nchunk = 0;
  auto go = [&](auto shape, auto db, auto vw) {
    typedef decltype(shape) S;
    constexpr bool DB = decltype(db)::value;
    constexpr int VW = decltype(vw)::value;
    const KbGrid gr = kb_grid<S>(n_proj, k, d);
    const bool xc = gr.nchunk % 8 == 0;
    const unsigned nwg = kb_workgroups(gr.nchunk, gr.nM, gr.nN, xc);
    constexpr size_t lds = kg_lds_bytes<T, S>(DB, VW);
    allow_lds(&k_kb_gemm<T, DB, S, VW>, lds);
    k_kb_gemm<T, DB, S, VW><<<nwg, 256, lds, s>>>(P, d, ldp, Y, ldy, part, n_proj, k, kp,
                                                   gr.kchunk, gr.nM, gr.nN, gr.nchunk, xc ? 1 : 0);
    nchunk = gr.nchunk;
  };
  if constexpr (sizeof(T) == 4) {
    if (ldp % 4 == 0 && ldy % 4 == 0 && reinterpret_cast<uintptr_t>(P) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(Y) % 16 == 0)
      go(KgVec{}, std::false_type{}, std::integral_constant<int, 4>{});
    else
      go(KbShape<float>{}, std::true_type{}, std::integral_constant<int, 1>{});
  } else {
    if (ldp % 2 == 0 && ldy % 2 == 0 && reinterpret_cast<uintptr_t>(P) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(Y) % 16 == 0)
      go(KbShape<double>{}, std::false_type{}, std::integral_constant<int, 2>{});
    else
      go(KbShape<double>{}, std::false_type{}, std::integral_constant<int, 1>{});
  }
  const int64_t n = int64_t(n_proj) * kp;
  const unsigned rb = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 4096));
  k_kb_reduce<T><<<rb, 256, 0, s>>>(part, nchunk, h, C, n_proj, k, kp);
}

int launch_atb_partial(const double* A, int64_t lda, const double* B, int64_t ldb, double* part,
                       int64_t part_cap, int64_t rows, int k, int kp, hipStream_t s) {
  // the projector product's split-K grid, with no more chunks than `part` holds
  KbGrid gr = kb_grid<KbShape<double>>(k, k, rows);
  const int64_t per_chunk = static_cast<int64_t>(k) * kp;
  const int64_t maxc = std::max<int64_t>(1, part_cap / per_chunk);
  if (gr.nchunk > maxc) {
    constexpr int KB = KbShape<double>::KB;
    gr.kchunk = round_up((rows + maxc - 1) / maxc, KB);
    gr.nchunk = static_cast<int>((rows + gr.kchunk - 1) / gr.kchunk);
  }
  const bool xc = gr.nchunk % 8 == 0;
  const unsigned nwg = kb_workgroups(gr.nchunk, gr.nM, gr.nN, xc);
  auto run = [&](auto vw) {
    constexpr int VW = decltype(vw)::value;
    k_kb_gemm<double, false, KbShape<double>, VW>
        <<<nwg, 256, kg_lds_bytes<double, KbShape<double>>(false, VW), s>>>(
            A, rows, lda, B, ldb, part, k, k, kp, gr.kchunk, gr.nM, gr.nN, gr.nchunk, xc ? 1 : 0);
  };
  if (lda % 2 == 0 && ldb % 2 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(B) % 16 == 0)
    run(std::integral_constant<int, 2>{});
  else
    run(std::integral_constant<int, 1>{});
  return gr.nchunk;
}

template <typename T>
void launch_kb_apply(const T* P, int64_t d, int64_t ldp, const T* C, T* Z, int n_proj, int k,
                     int kp, hipStream_t s) {
  // wide tiles when the 16-byte column loads stay aligned
  constexpr int VW = 16 / static_cast<int>(sizeof(T));
  if (ldp % VW == 0 && kp % VW == 0 && reinterpret_cast<uintptr_t>(P) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(C) % 16 == 0) {
    constexpr int BI = 32 * ApShape<T>::TI, BA = 32 * ApShape<T>::TA;
    const int nI = (k + BI - 1) / BI;
    const int nA = static_cast<int>((d + BA - 1) / BA);
    const unsigned nwg = static_cast<unsigned>(8 * ((nA + 7) / 8) * nI);
    constexpr size_t lds = kb_apply_wide_lds<T>();
    allow_lds(&k_kb_apply_wide<T>, lds);
    k_kb_apply_wide<T><<<nwg, 256, lds, s>>>(P, d, ldp, C, n_proj, k, kp, Z, nI, nA);
    return;
  }
  constexpr int BM = 32 * KbShape<T>::TN, BN = 32 * KbShape<T>::TM;
  const int nI = (k + BM - 1) / BM;
  const int nA = static_cast<int>((d + BN - 1) / BN);
  const unsigned nwg = static_cast<unsigned>(8 * ((nA + 7) / 8) * nI);
  constexpr int KBA = KbShape<T>::KB;   // projectors per staged step
  constexpr size_t lds = kb_lds_bytes<T>(false, KBA);
  allow_lds(&k_kb_apply<T, false, KBA>, lds);
  k_kb_apply<T, false, KBA><<<nwg, 256, lds, s>>>(P, d, ldp, C, n_proj, k, kp, Z, nI, nA);
}

template void launch_kb_apply<float>(const float*, int64_t, int64_t, const float*, float*, int,
                                     int, int, hipStream_t);
template void launch_kb_apply<double>(const double*, int64_t, int64_t, const double*, double*,
                                      int, int, int, hipStream_t);
template void launch_kb_gemm<float>(const float*, int64_t, int64_t, const float*, int64_t,
                                    const float*, float*, float*, int, int, int, hipStream_t);
template void launch_kb_gemm<double>(const double*, int64_t, int64_t, const double*, int64_t,
                                     const double*, double*, double*, int, int, int, hipStream_t);

}  // namespace ces
