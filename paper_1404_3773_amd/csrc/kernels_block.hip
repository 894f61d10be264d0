// FP64 kernels on tall-skinny blocks and their small k x k matrices, for
// Cholesky-QR and Rayleigh-Ritz (Section 3.1.1, steps of the subspace
// iteration): the Gram product C = A^T B over d rows, the Cholesky factor of
// the scaled Gram matrix, the projected symmetric eigenproblem, and the block
// rotations X <- X D R^{-1} and X <- X S with the Ritz residuals.
//
// Blocks are column-major d x k (leading dimension ld >= d).  For k <=
// kJacobiMax the k x k results that rotate the block are written zero-padded
// with leading dimension small_ld(k) = k rounded up to 16, so that the
// rotation kernels run loops of fixed length.
#include <hip/hip_runtime.h>

#include "ces_internal.h"
#include "mfma.h"

namespace ces {
namespace {

// Sum over the workgroup, returned in every thread.
__device__ __forceinline__ double block_sum_all(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int u = 0; u < (int)(blockDim.x + 63) / 64; ++u) t += red[u];
  return t;
}

// 1/x and 1/sqrt(x) in FP64 from the hardware estimates refined by two
// Newton steps each (r <- r (2 - x r); y <- y (3 - x y^2) / 2), accurate to a
// few ulps for the normal positive arguments used here.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-0.5 * x * y, y, 0.5), y);
  y = fma(y, fma(-0.5 * x * y, y, 0.5), y);
  return y;
}

// ----------------------------------------------------------------- Gram

// part[c] = sum over the rows of chunk c of A[row][i] B[row][j] (k x k,
// column-major), k <= 16 KT, on FP64 MFMA.  The rows are the contraction
// index: k-step rows go to lanes as A[i][kk] = A[row0 + kk][i] and B[kk][j] =
// B[row0 + kk][j], so both operands use the same lane mapping (and one load
// serves both when A = B).  Each wave takes 16-row groups of the chunk, GB
// groups per batch with all of a batch's loads issued before its MFMAs; the
// four waves' tiles are summed in LDS in a fixed order.
template <int KT, bool SAME>
__global__ __launch_bounds__(256) void k_gram_ts(const double* __restrict__ A, int64_t lda,
                                                 const double* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ part, int64_t rows, int k,
                                                 int64_t chunk) {
  constexpr int GB = KT <= 2 ? 4 : 2;     // 16-row groups per batch
  constexpr int KS = 4 * GB;              // k-steps per batch
  __shared__ double red[KT * KT * 4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, kk = lane >> 4;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * chunk;
  const int64_t r1 = r0 + chunk < rows ? r0 + chunk : rows;
  const double* pa[KT];
  const double* pb[KT];
  bool cok[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) {
    const int col = 16 * t + c16;
    cok[t] = col < k;
    const int cc = col < k ? col : k - 1;
    pa[t] = A + static_cast<int64_t>(cc) * lda;
    pb[t] = B + static_cast<int64_t>(cc) * ldb;
  }
  d4 acc[KT][KT];
#pragma unroll
  for (int a = 0; a < KT; ++a)
#pragma unroll
    for (int b = 0; b < KT; ++b) acc[a][b] = zero_acc<d4>();
  // batch: groups g = 0..GB-1 of this wave at rows base + 64 g .. + 16
  for (int64_t base = r0 + 16 * wave; base < r1; base += 64 * GB) {
    // every load of the batch is issued first (clamped rows and columns),
    // the masks are applied at the MFMA (a select on a load would wait for it)
    double av[KS][KT], bv[KS][KT];
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int64_t row = base + 64 * (u >> 2) + 4 * (u & 3) + kk;
      const int64_t rc = row < r1 ? row : r1 - 1;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        av[u][t] = pa[t][rc];
        if (!SAME) bv[u][t] = pb[t][rc];
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const bool ok = base + 64 * (u >> 2) + 4 * (u & 3) + kk < r1;
      double am[KT], bm[KT];
#pragma unroll
      for (int a = 0; a < KT; ++a) {
        am[a] = ok && cok[a] ? av[u][a] : 0.0;
        bm[a] = SAME ? am[a] : (ok && cok[a] ? bv[u][a] : 0.0);
      }
#pragma unroll
      for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b) acc[a][b] = MF<double>::mma(am[a], bm[b], acc[a][b]);
    }
  }
  // waves 3, 2, 1 pass their running sums down; wave 0 writes the chunk sum
  for (int w = 3; w >= 0; --w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < KT; ++a)
#pragma unroll
        for (int b = 0; b < KT; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            double* slot = red + ((a * KT + b) * 4 + v) * 64 + lane;
            const double x = w == 3 ? acc[a][b][v] : acc[a][b][v] + *slot;
            if (w > 0) {
              *slot = x;
            } else {
              const int i = 16 * a + MF<double>::row(lane, v), j = 16 * b + c16;
              if (i < k && j < k)
                part[static_cast<int64_t>(blockIdx.x) * k * k + static_cast<int64_t>(j) * k + i] = x;
            }
          }
    }
    __syncthreads();
  }
}

// Output tile edge used to size the Gram's partial-sum region for large k.
constexpr int GR_T = 64;

// C (column-major k x k) = sum_c part[c] with part[c] row-major k x kp (the
// large-k Gram's chunks), or with sym (S + S^T) / 2, bitwise symmetric; one
// thread per element, chunks summed in order.
__global__ __launch_bounds__(256) void k_gram_reduce_rm(const double* __restrict__ part,
                                                        double* __restrict__ C, int k, int kp,
                                                        int nchunk, int sym) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= kk) return;
  const int64_t q = e % k, i = e / k;
  const int64_t cs = static_cast<int64_t>(k) * kp;
  double sv = 0.0, tv = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    sv += part[c * cs + q * kp + i];
    if (sym) tv += part[c * cs + i * kp + q];
  }
  C[e] = sym ? 0.5 * (sv + tv) : sv;
}

// C[i][j] = sum_c part[c][i][j], or with sym the symmetric part
// (sum_c part[c][i][j] + sum_c part[c][j][i]) / 2, bitwise symmetric.
// One wave per element; lanes stride the chunks.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part,
                                                     double* __restrict__ C, int k, int nchunk,
                                                     int sym) {
  const int64_t kk = static_cast<int64_t>(k) * k;
  const int lane = threadIdx.x & 63;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (e >= kk) return;
  const int64_t i = e % k, j = e / k;
  const int64_t et = i * k + j;
  double s = 0.0, t = 0.0;
  for (int c = lane; c < nchunk; c += 64) {
    s += part[c * kk + e];
    if (sym) t += part[c * kk + et];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_down(s, o, 64);
    t += __shfl_down(t, o, 64);
  }
  if (lane == 0) C[e] = sym ? 0.5 * (s + t) : s;
}

// ------------------------------------------------------------- Cholesky

// Cholesky-QR factor step for k <= kJacobiMax in one workgroup (Section
// 3.1.1): from the Gram matrix S (k x k, column-major, ld k), D =
// diag(S)^{-1/2} into dinv, D S D + shift I = R^T R (R upper), and W = D
// R^{-1} written over S with leading dimension ldw, zero below the diagonal
// and outside k x k, so that X D R^{-1} = X W.  Right-looking, one barrier per
// column: step j reads row j of the trailing matrix (upper triangle of A),
// writes the scaled row R(j, i) = A(j, i) / R(j, j) transposed into the
// unused lower triangle of A, and updates the trailing upper triangle in
// place; each thread owns fixed upper-triangle entries.  Then the upper
// triangle, free again, receives R^{-1} row by row from the bottom.  *info = 0, or j + 1 if the j-th pivot is not above 2 k eps
// (a numerically dependent column).
template <int KP, int NT>
__global__ __launch_bounds__(NT) void k_chol(double* __restrict__ S, int k, int ldw,
                                             double shift, double* __restrict__ dinv, int* info) {
  constexpr int NE = KP * (KP + 1) / 2;          // upper-triangle entries of KP x KP
  constexpr int U = (NE + NT - 1) / NT;
  __shared__ double A[KP][KP + 1];   // upper: trailing matrix, then R^{-1}; lower: A[i][j] = R(j, i)
  __shared__ double rd[KP];          // 1/R(j, j)
  __shared__ double dv[KP];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int i = tid; i < k; i += NT) {
    const double di = rsq64(S[static_cast<int64_t>(i) * k + i]);
    dv[i] = di;
    dinv[i] = di;
  }
  if (tid == 0) bad = 0;
  // owned entries (a, c), a <= c, enumerated row by row
  int oa[U], oc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    int e = tid + u * NT, a = 0;
    while (a < KP && e >= KP - a) {
      e -= KP - a;
      ++a;
    }
    oa[u] = a;
    oc[u] = a + e;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int a = oa[u], c = oc[u];
    if (a < k && c < k)
      A[a][c] = S[static_cast<int64_t>(c) * k + a] * dv[a] * dv[c] + (a == c ? shift : 0.0);
  }
  __syncthreads();
  // D S D has a unit diagonal: a pivot at rounding level (<= 2 k eps) means a
  // numerically dependent column and fails the pass like a non-positive one
  const double ptol = 2.0 * k * 2.220446049250313e-16;
  for (int j = 0; j < k; ++j) {
    const double djj = A[j][j];
    const bool pos = djj > ptol;
    const double piv = pos ? djj : 1.0;
    const double rinv = rsq64(piv);
    const double inv = rinv * rinv;
    if (tid == 0) {
      if (!pos && bad == 0) bad = j + 1;
      rd[j] = rinv;
    }
    for (int i = j + 1 + tid; i < k; i += NT) A[i][j] = A[j][i] * rinv;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a = oa[u], c = oc[u];
      if (a > j && c < k) A[a][c] -= A[j][a] * A[j][c] * inv;
    }
    __syncthreads();
  }
  // R^{-1} by rows from the bottom, right-looking: the owner of (a, c) keeps
  // s = sum_{l > a} R(a, l) R^{-1}(l, c) and sets R^{-1}(a, c) = -s / R(a, a)
  // (1 / R(a, a) on the diagonal) when row a comes; one barrier per row.
  double sacc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) sacc[u] = 0.0;
  for (int l = k - 1; l >= 0; --l) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a = oa[u], c = oc[u];
      if (a == l && c < k) A[l][c] = a == c ? rd[l] : -rd[l] * sacc[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int a = oa[u], c = oc[u];
      if (a < l && l <= c && c < k) sacc[u] = fma(A[l][a], A[l][c], sacc[u]);
    }
  }
  __syncthreads();
  for (int e = tid; e < ldw * ldw; e += NT) {
    const int c = e / ldw, i = e - c * ldw;
    S[e] = (c < k && i <= c) ? dv[i] * A[i][c] : 0.0;
  }
  if (tid == 0) {
    info[0] = bad;
    info[1] = 0;   // the triangular-inverse flag of the library path: nothing to report
  }
}

// ------------------------------------------------- Jacobi eigensolver

// Symmetric eigenproblem of a small k x k matrix (k <= kJacobiMax) in one
// workgroup: parallel cyclic Jacobi.  Each round rotates n/2 disjoint pairs
// (p, q) of the round-robin (circle) schedule over n = k rounded up to even
// players, so that n - 1 rounds make a sweep over all pairs.  Each rotation
// is the 2 x 2 symmetric Schur rotation that zeroes A_pq (Golub and Van
// Loan, Algorithm 8.4.1: th = (A_qq - A_pp) / (2 A_pq), t = sign(th) / (|th| +
// sqrt(th^2 + 1)), c = 1 / sqrt(1 + t^2), s = t c); pairs with |A_pq| below
// 1e-20 ||A||_F are left alone.  With J the product of a round's rotations,
// A <- J^T A J is formed in one pass over 2 x 2 blocks, block (P, P') of the
// pairs P, P' becoming R_P^T A_PP' R_P' (the diagonal blocks take the exact
// Schur form A_pp - t A_pq, A_qq + t A_pq), written mirrored into a second
// buffer so that A stays exactly symmetric; V <- V J in the same pass.  A
// round costs two barriers: rotation parameters, then the update.  Sweeps
// stop when the off-diagonal Frobenius norm is below 1e-14 of the whole;
// eigenvalues are sorted ascending (ties by index) with their columns of V,
// written over S with leading dimension ldo, zero-padded.  info = 0 on
// convergence within 40 sweeps, else 1.
__device__ __forceinline__ int rr_player(int pos, int r, int n) {
  return pos == 0 ? 0 : (pos - 1 + r) % (n - 1) + 1;
}

constexpr int kJacobiThreads = 1024;

inline size_t jacobi_lds_bytes(int k, int np) {
  const int n = k + (k & 1), half = np / 2;
  return (3 * size_t(n) * (n + 1) + 3 * size_t(half)) * sizeof(double) + size_t(half) * 4 +
         size_t(n - 1) * (n / 2) * 2;
}

template <int NP>
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi_eig(double* __restrict__ S, int k,
                                                              int ldo, double* __restrict__ evals,
                                                              int* info) {
  constexpr int HALF = NP / 2;
  constexpr int NT = kJacobiThreads;
  constexpr int NB = HALF * HALF, NTASK = NB + HALF * NP;
  constexpr int U = (NTASK + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = k + (k & 1), nh = n / 2, ld = n + 1;
  double* Acur = reinterpret_cast<double*>(smem_raw);   // [n][ld]
  double* Anext = Acur + n * ld;                         // [n][ld]
  double* V = Anext + n * ld;                            // [n][ld]
  double* rot = V + n * ld;                              // [HALF][3]: c, s, t
  int* pq = reinterpret_cast<int*>(rot + 3 * HALF);      // [HALF]: p | q << 8
  unsigned short* sched = reinterpret_cast<unsigned short*>(pq + HALF);   // [n-1][nh]
  __shared__ double red[16];
  __shared__ int done;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, j = e - i * n;
    const double a = (i < k && j < k) ? S[static_cast<int64_t>(j) * k + i] : 0.0;
    Acur[i * ld + j] = a;
    Anext[i * ld + j] = a;
    V[i * ld + j] = i == j ? 1.0 : 0.0;
  }
  for (int e = tid; e < (n - 1) * nh; e += NT) {
    const int r = e / nh, pi = e - r * nh;
    int p = rr_player(pi, r, n), q = rr_player(n - 1 - pi, r, n);
    if (p > q) {
      const int t = p;
      p = q;
      q = t;
    }
    sched[r * nh + pi] = static_cast<unsigned short>(p | (q << 8));
  }
  __syncthreads();
  double f = 0.0;
  for (int e = tid; e < n * n; e += NT) {
    const double a = Acur[(e / n) * ld + e % n];
    f += a * a;
  }
  const double fro2 = block_sum_all(f, red);
  const double tiny = 1e-20 * sqrt(fro2);
  int converged = 0;
  for (int sweep = 0; sweep < 40 && !converged; ++sweep) {
    for (int r = 0; r < n - 1; ++r) {
      if (tid < nh) {
        const int pk = sched[r * nh + tid];
        const int p = pk & 255, q = pk >> 8;
        double c = 1.0, sn = 0.0, t = 0.0;
        const double apq = Acur[p * ld + q];
        if (q < k && fabs(apq) > tiny) {
          const double th = (Acur[q * ld + q] - Acur[p * ld + p]) * rcp64(2.0 * apq);
          const double u = fma(th, th, 1.0);
          const double tm = rcp64(fabs(th) + u * rsq64(u));
          t = th >= 0.0 ? tm : -tm;
          c = rsq64(fma(t, t, 1.0));
          sn = t * c;
        }
        rot[3 * tid] = c;
        rot[3 * tid + 1] = sn;
        rot[3 * tid + 2] = t;
        pq[tid] = pk;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int task = tid + u * NT;
        if (task < NB) {
          const int P = task / HALF, Q = task % HALF;
          if (P > Q || Q >= nh) continue;
          const int pk1 = pq[P], pk2 = pq[Q];
          const int p = pk1 & 255, q = pk1 >> 8, p2 = pk2 & 255, q2 = pk2 >> 8;
          double o0, o1, o2, o3;
          if (P == Q) {
            const double t = rot[3 * P + 2], apq = Acur[p * ld + q];
            o0 = Acur[p * ld + p] - t * apq;
            o3 = Acur[q * ld + q] + t * apq;
            o1 = o2 = t == 0.0 ? apq : 0.0;
          } else {
            const double c1 = rot[3 * P], s1 = rot[3 * P + 1];
            const double c2 = rot[3 * Q], s2 = rot[3 * Q + 1];
            const double b00 = Acur[p * ld + p2], b01 = Acur[p * ld + q2];
            const double b10 = Acur[q * ld + p2], b11 = Acur[q * ld + q2];
            const double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
            const double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
            o0 = c2 * t00 - s2 * t01;
            o1 = s2 * t00 + c2 * t01;
            o2 = c2 * t10 - s2 * t11;
            o3 = s2 * t10 + c2 * t11;
            Anext[p2 * ld + p] = o0;
            Anext[q2 * ld + p] = o1;
            Anext[p2 * ld + q] = o2;
            Anext[q2 * ld + q] = o3;
          }
          Anext[p * ld + p2] = o0;
          Anext[p * ld + q2] = o1;
          Anext[q * ld + p2] = o2;
          Anext[q * ld + q2] = o3;
        } else if (task < NTASK) {
          const int e = task - NB;
          const int P = e / NP, i = e % NP;
          if (P >= nh || i >= n) continue;
          const int pk = pq[P];
          const int p = pk & 255, q = pk >> 8;
          const double c = rot[3 * P], sn = rot[3 * P + 1];
          const double va = V[i * ld + p], vb = V[i * ld + q];
          V[i * ld + p] = c * va - sn * vb;
          V[i * ld + q] = sn * va + c * vb;
        }
      }
      __syncthreads();
      double* tmp = Acur;
      Acur = Anext;
      Anext = tmp;
    }
    double o = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const int i = e / n, j = e - i * n;
      if (i != j) o += Acur[i * ld + j] * Acur[i * ld + j];
    }
    const double off = block_sum_all(o, red);
    if (tid == 0) done = off <= 1e-28 * fro2 ? 1 : 0;
    __syncthreads();
    converged = done;
    __syncthreads();
  }
  for (int e = tid; e < ldo * ldo; e += NT) {
    const int c = e / ldo, i = e - c * ldo;
    if (i >= k || c >= k) S[e] = 0.0;
  }
  for (int i = tid; i < k; i += NT) {
    const double lam = Acur[i * ld + i];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double mu = Acur[j * ld + j];
      rank += (mu < lam || (mu == lam && j < i)) ? 1 : 0;
    }
    evals[rank] = lam;
    for (int rr = 0; rr < k; ++rr) S[static_cast<int64_t>(rank) * ldo + rr] = V[rr * ld + i];
  }
  if (tid == 0) *info = converged ? 0 : 1;
}

// ----------------------------------------------------- block rotation

// Rows are written only where flags[0] and flags[1] are zero (the
// Cholesky-QR pass that produced the block succeeded).

// X <- X W in place (and with TWO also Y <- Y W) on FP64 MFMA, W (KC x KC,
// KC = 16 KT, zero outside k x k) held in registers.  A wave takes 16-row
// tiles and forms the transposed product (X W)^T = W^T X^T: the A operand
// lane q holds W[4s + q/16][16b + q%16] (k-step s, column tile b), the B
// operand X[row0 + q%16][4s + q/16], so the result of lane q, register v is
// (X W)[row0 + q%16][16b + q/16 + 4v] and every load and store covers 16
// consecutive rows.  Columns past k read column k - 1 (their rows of W are
// zero); a tile is read whole before it is written.  With TWO, part[j *
// gridDim.x + block] receives the block's sum of ((Y W)_j - theta_j
// (X W)_j)^2, written whatever the flags say.
template <int KT, bool TWO>
__global__ __launch_bounds__(256) void k_block_mfma(double* __restrict__ X, int64_t ldx,
                                                    double* __restrict__ Y, int64_t ldy,
                                                    const double* __restrict__ W, int k,
                                                    int64_t rows, const int* __restrict__ flags,
                                                    const double* __restrict__ theta,
                                                    double* __restrict__ part) {
  constexpr int KC = 16 * KT, KS = 4 * KT;
  __shared__ double red[TWO ? 4 * KC : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c16 = lane & 15, kk = lane >> 4;
  const bool write = flags[0] == 0 && flags[1] == 0;
  double wf[KS][KT];
#pragma unroll
  for (int st = 0; st < KS; ++st)
#pragma unroll
    for (int b = 0; b < KT; ++b) wf[st][b] = W[(16 * b + c16) * KC + 4 * st + kk];
  double th[KT][4], res[KT][4];
#pragma unroll
  for (int b = 0; b < KT; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = 16 * b + kk + 4 * v;
      th[b][v] = TWO && col < k ? theta[col] : 0.0;
      res[b][v] = 0.0;
    }
  int64_t coff[KS];                       // columns of the B operand
#pragma unroll
  for (int st = 0; st < KS; ++st) coff[st] = (4 * st + kk < k ? 4 * st + kk : k - 1);
  const int64_t ntiles = (rows + 15) / 16;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + wave; t < ntiles;
       t += static_cast<int64_t>(gridDim.x) * 4) {
    const int64_t row = t * 16 + c16;
    const bool ok = row < rows;
    const int64_t rc = ok ? row : rows - 1;
    double xb[KS], yb[TWO ? KS : 1];
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      xb[st] = X[coff[st] * ldx + rc];
      if (TWO) yb[st] = Y[coff[st] * ldy + rc];
    }
    d4 ax[KT], ay[KT];
#pragma unroll
    for (int b = 0; b < KT; ++b) {
      ax[b] = zero_acc<d4>();
      ay[b] = zero_acc<d4>();
    }
#pragma unroll
    for (int st = 0; st < KS; ++st)
#pragma unroll
      for (int b = 0; b < KT; ++b) {
        ax[b] = MF<double>::mma(wf[st][b], xb[st], ax[b]);
        if (TWO) ay[b] = MF<double>::mma(wf[st][b], yb[st], ay[b]);
      }
#pragma unroll
    for (int b = 0; b < KT; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = 16 * b + kk + 4 * v;
        if (ok && col < k) {
          if (write) {
            X[col * ldx + row] = ax[b][v];
            if (TWO) Y[col * ldy + row] = ay[b][v];
          }
          if (TWO) {
            const double r = ay[b][v] - th[b][v] * ax[b][v];
            res[b][v] = fma(r, r, res[b][v]);
          }
        }
      }
  }
  if (TWO) {
    // sum over the 16 rows of a lane group, then over the waves
#pragma unroll
    for (int b = 0; b < KT; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = res[b][v];
        for (int o = 8; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (c16 == 0) red[wave * KC + 16 * b + kk + 4 * v] = x;
      }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += blockDim.x)
      part[static_cast<int64_t>(j) * gridDim.x + blockIdx.x] =
          red[j] + red[KC + j] + red[2 * KC + j] + red[3 * KC + j];
  }
}

// out[c] = sqrt(sum_b part[c * nb + b]): one wave per column.
__global__ __launch_bounds__(256) void k_finish_sqrt(const double* __restrict__ part, int nb,
                                                     int ncol, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= ncol) return;
  double t = 0.0;
  for (int b = lane; b < nb; b += 64) t += part[static_cast<int64_t>(c) * nb + b];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
  if (lane == 0) out[c] = sqrt(t);
}

inline unsigned tile_blocks(int64_t rows, int64_t cap) {
  int64_t nb = ((rows + 15) / 16 + 3) / 4;   // one 16-row tile per wave
  if (nb > 1024) nb = 1024;
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  return static_cast<unsigned>(nb);
}

template <int KT>
void rotate_kt(double* X, int64_t ldx, double* Y, int64_t ldy, const double* W, int k,
               int64_t rows, const int* flags, const double* theta, double* res, double* part,
               int64_t part_cap, hipStream_t s) {
  if (!Y) {
    k_block_mfma<KT, false><<<tile_blocks(rows, 1024), 256, 0, s>>>(X, ldx, nullptr, 0, W, k,
                                                                    rows, flags, nullptr, nullptr);
    return;
  }
  if (KT <= 2 && part_cap / k >= 1) {
    const unsigned nb = tile_blocks(rows, part_cap / k);
    k_block_mfma<KT <= 2 ? KT : 2, true><<<nb, 256, 0, s>>>(X, ldx, Y, ldy, W, k, rows, flags,
                                                            theta, part);
    k_finish_sqrt<<<(k + 3) / 4, 256, 0, s>>>(part, static_cast<int>(nb), k, res);
    return;
  }
  const unsigned nb = tile_blocks(rows, 1024);
  k_block_mfma<KT, false><<<nb, 256, 0, s>>>(X, ldx, nullptr, 0, W, k, rows, flags, nullptr,
                                             nullptr);
  k_block_mfma<KT, false><<<nb, 256, 0, s>>>(Y, ldy, nullptr, 0, W, k, rows, flags, nullptr,
                                             nullptr);
  launch_residuals(Y, ldy, X, ldx, theta, res, rows, k, part, part_cap, s);
}

template <int NP>
void jacobi_np(double* S, int k, double* evals, int* info, hipStream_t s) {
  const size_t lds = jacobi_lds_bytes(k, NP);
  // more than the default 64 KB of LDS (k > 50): raised on every such launch
  // rather than behind a process-wide flag, so concurrent callers and other
  // devices need no synchronisation; a refusal makes the launch fail, which
  // the caller's launch check reports
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_eig<NP>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  k_jacobi_eig<NP><<<1, kJacobiThreads, lds, s>>>(S, k, small_ld(k), evals, info);
}

}  // namespace

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
                 double* part, int64_t rows, int k, hipStream_t s, bool sym) {
  const int nch = gram_chunks(rows, k);
  int64_t chunk = (rows + nch - 1) / nch;
  const int64_t kk = static_cast<int64_t>(k) * k;
  if (k <= 64) {
    chunk = (chunk + 63) / 64 * 64;
    const int nb = static_cast<int>((rows + chunk - 1) / chunk);
    const bool same = A == B && lda == ldb;
    switch ((k + 15) / 16) {
#define CES_GRAM(KT)                                                                          \
  case KT:                                                                                    \
    if (same)                                                                                 \
      k_gram_ts<KT, true><<<nb, 256, 0, s>>>(A, lda, B, ldb, part, rows, k, chunk);           \
    else                                                                                      \
      k_gram_ts<KT, false><<<nb, 256, 0, s>>>(A, lda, B, ldb, part, rows, k, chunk);          \
    break;
      CES_GRAM(1)
      CES_GRAM(2)
      CES_GRAM(3)
      default: CES_GRAM(4)
#undef CES_GRAM
    }
    k_gram_reduce<<<static_cast<unsigned>((kk + 3) / 4), 256, 0, s>>>(part, C, k, nb, sym ? 1 : 0);
    return;
  }
  // k > 64: the split-K FP64 MFMA GEMM of the projector products, in the
  // region sized for gram_chunks(rows, k) chunks of k x k
  const int kp = (k + 15) / 16 * 16;
  const int nc = launch_atb_partial(A, lda, B, ldb, part, int64_t(nch) * kk, rows, k, kp, s);
  k_gram_reduce_rm<<<static_cast<unsigned>((kk + 255) / 256), 256, 0, s>>>(part, C, k, kp, nc,
                                                                           sym ? 1 : 0);
}

int small_ld(int k) { return (k + 15) / 16 * 16; }

void launch_jacobi_eig(double* S, int k, double* evals, int* info, hipStream_t s) {
  switch (small_ld(k)) {
    case 16: jacobi_np<16>(S, k, evals, info, s); break;
    case 32: jacobi_np<32>(S, k, evals, info, s); break;
    case 48: jacobi_np<48>(S, k, evals, info, s); break;
    default: jacobi_np<64>(S, k, evals, info, s); break;
  }
}

void launch_chol_inv(double* S, int k, double shift, double* dinv, int* info, hipStream_t s) {
  switch (small_ld(k)) {
    case 16: k_chol<16, 256><<<1, 256, 0, s>>>(S, k, 16, shift, dinv, info); break;
    case 32: k_chol<32, 512><<<1, 512, 0, s>>>(S, k, 32, shift, dinv, info); break;
    case 48: k_chol<48, 1024><<<1, 1024, 0, s>>>(S, k, 48, shift, dinv, info); break;
    default: k_chol<64, 1024><<<1, 1024, 0, s>>>(S, k, 64, shift, dinv, info); break;
  }
}

void launch_block_apply(double* X, int64_t ldx, const double* W, int k, int64_t rows,
                        const int* flags, hipStream_t s) {
  launch_block_rotate(X, ldx, nullptr, 0, W, k, rows, flags, nullptr, nullptr, nullptr, 0, s);
}

void launch_block_rotate(double* X, int64_t ldx, double* Y, int64_t ldy, const double* W, int k,
                         int64_t rows, const int* flags, const double* theta, double* res,
                         double* part, int64_t part_cap, hipStream_t s) {
  switch (small_ld(k) / 16) {
    case 1: rotate_kt<1>(X, ldx, Y, ldy, W, k, rows, flags, theta, res, part, part_cap, s); break;
    case 2: rotate_kt<2>(X, ldx, Y, ldy, W, k, rows, flags, theta, res, part, part_cap, s); break;
    case 3: rotate_kt<3>(X, ldx, Y, ldy, W, k, rows, flags, theta, res, part, part_cap, s); break;
    default: rotate_kt<4>(X, ldx, Y, ldy, W, k, rows, flags, theta, res, part, part_cap, s); break;
  }
}

}  // namespace ces
