// HIP kernels (gfx950) of the learned start density: an FP32 MFMA GEMM for
// the dense layers of the per-atom network (forward and both backward
// products), bias / SiLU / gradient / Adam elementwise kernels, the
// atom-centred correction functions on the quadrature grid, and the
// per-cluster quadratic density loss.
#include <hip/hip_runtime.h>

#include "ces_internal.h"
#include "mfma.h"

namespace ces {

namespace {

inline int grid1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  return static_cast<int>(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

// ------------------------------------------------------------------ GEMM
// C[M][N] = alpha op(A)[M][K] op(B)[K][N] + beta C, all row-major;
// op(A)[m][k] = TA ? A[k][m] : A[m][k], op(B)[k][n] = TB ? B[n][k] : B[k][n].
// 64 x 64 tile per workgroup, K in steps of 16 through LDS, four waves of
// 2 x 2 MFMA 16x16x4 tiles each.
constexpr int GT = 64, GK = 16;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb,
                                                  float* __restrict__ C, int ldc, int M, int N,
                                                  int K, float alpha, float beta) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = zero_acc<f4>();
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int mm = TA ? (e & (GT - 1)) : (e >> 4);
      const int kk = TA ? (e >> 6) : (e & (GK - 1));
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < K)
        v = TA ? A[static_cast<int64_t>(gk) * lda + gm] : A[static_cast<int64_t>(gm) * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = tid; e < GT * GK; e += 256) {
      const int nn = TB ? (e >> 4) : (e & (GT - 1));
      const int kk = TB ? (e & (GK - 1)) : (e >> 6);
      const int gn = n0 + nn, gk = k0 + kk;
      float v = 0.f;
      if (gn < N && gk < K)
        v = TB ? B[static_cast<int64_t>(gn) * ldb + gk] : B[static_cast<int64_t>(gk) * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[ks + lk][wm + 16 * t + lr];
        b[t] = Bs[ks + lk][wn + 16 * t + lr];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = MF<float>::mma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + 16 * i + MF<float>::row(lane, v);
        const int col = n0 + wn + 16 * j + lr;
        if (row < M && col < N) {
          float* c = C + static_cast<int64_t>(row) * ldc + col;
          *c = alpha * acc[i][j][v] + (beta != 0.f ? beta * *c : 0.f);
        }
      }
}

// ------------------------------------------------------------- elementwise

// H[r][c] = (X[r][c] - mean[c]) / std[c]
__global__ void k_standardize(const float* __restrict__ X, const float* __restrict__ mean,
                              const float* __restrict__ sd, float* __restrict__ H, int64_t rows,
                              int cols) {
  const int64_t n = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(e % cols);
    H[e] = (X[e] - mean[c]) / sd[c];
  }
}

// Z += b (broadcast over rows); H = silu(Z) if act, else H = Z (H may be Z).
__global__ void k_bias_act(float* __restrict__ Z, const float* __restrict__ b, float* H,
                           int64_t rows, int cols, int act) {
  const int64_t n = rows * cols;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float z = Z[e] + b[e % cols];
    Z[e] = z;
    H[e] = act ? z / (1.f + __expf(-z)) : z;
  }
}

// G *= silu'(Z),  silu'(z) = s (1 + z (1 - s)), s = 1 / (1 + e^-z)
__global__ void k_act_grad(float* __restrict__ G, const float* __restrict__ Z, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float z = Z[e];
    const float s = 1.f / (1.f + __expf(-z));
    G[e] *= s * (1.f + z * (1.f - s));
  }
}

// db[c] = sum_r G[r][c]; one workgroup per column block of 64, rows split
// over the four waves and reduced in LDS.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, float* __restrict__ db,
                                                int64_t rows, int cols) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  float s = 0.f;
  if (c < cols)
    for (int64_t r = w; r < rows; r += 4) s += G[r * cols + c];
  red[w][threadIdx.x & 63] = s;
  __syncthreads();
  if (w == 0 && c < cols)
    db[c] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Adam (Kingma and Ba), bias-corrected.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// ----------------------------------------------------- correction functions

constexpr int kSph = 5, kDip = 3, kChan = kSph + kDip;
__constant__ double c_sph_sigma[kSph] = {0.6, 0.9, 1.3, 1.9, 2.8};
__constant__ double c_dip_sigma[kDip] = {0.9, 1.4, 2.2};

__device__ __forceinline__ void grid_point(int64_t g, const double* rnode, const double* cth,
                                           const double* sth, const double* cs, int n_theta,
                                           int n_phi, double& x, double& y, double& z, int& ir,
                                           int& j) {
  const int p = static_cast<int>(g % n_phi);
  const int64_t rj = g / n_phi;
  j = static_cast<int>(rj % n_theta);
  ir = static_cast<int>(rj / n_theta);
  const double r = rnode[ir];
  x = r * sth[j] * cs[p];
  y = r * sth[j] * cs[n_phi + p];
  z = r * cth[j];
}

// The eight functions of one atom at displacement (dx, dy, dz).
__device__ __forceinline__ void channels(double dx, double dy, double dz, const double* u,
                                         double* phi) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double proj = dx * u[0] + dy * u[1] + dz * u[2];
#pragma unroll
  for (int q = 0; q < kSph; ++q) {
    const double s = c_sph_sigma[q];
    const double a = r2 / (2.0 * s * s);
    phi[q] = a < 80.0 ? exp(-a) / (s * s * s * 15.749609945722419) : 0.0;  // (2 pi)^1.5
  }
#pragma unroll
  for (int q = 0; q < kDip; ++q) {
    const double s = c_dip_sigma[q];
    const double a = r2 / (2.0 * s * s);
    phi[kSph + q] = a < 80.0 ? exp(-a) * proj / (s * s * s * s * 15.749609945722419) : 0.0;
  }
}

// F[c][g] (column-major n_grid x (8 n_atoms + 1)): sqrt(W_g) Phi_c(x_g) for
// c = 8 j + q, and sqrt(W_g) target(x_g) in the last column.
__global__ __launch_bounds__(256) void k_fit_columns(
    const double* __restrict__ rnode, const double* __restrict__ wr, const double* __restrict__ cth,
    const double* __restrict__ sth, const double* __restrict__ wt, const double* __restrict__ cs,
    int n_theta, int n_phi, int64_t n_grid, const double* __restrict__ atoms,
    const double* __restrict__ dirs, int n_atoms, const double* __restrict__ target,
    double* __restrict__ F) {
  const double dphi = 2.0 * M_PI / n_phi;
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < n_grid;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double x, y, z;
    int ir, j;
    grid_point(g, rnode, cth, sth, cs, n_theta, n_phi, x, y, z, ir, j);
    const double sw = sqrt(wr[ir] * wt[j] * dphi);
    for (int a = 0; a < n_atoms; ++a) {
      double phi[kChan];
      channels(x - atoms[3 * a], y - atoms[3 * a + 1], z - atoms[3 * a + 2], dirs + 3 * a, phi);
#pragma unroll
      for (int q = 0; q < kChan; ++q) F[(static_cast<int64_t>(kChan) * a + q) * n_grid + g] = sw * phi[q];
    }
    F[static_cast<int64_t>(kChan) * n_atoms * n_grid + g] = target ? sw * target[g] : 0.0;
  }
}

// rho[g] += sum_{j,q} coef[j][q] Phi_q(x_g - a_j)
__global__ __launch_bounds__(256) void k_density_correction(
    const double* __restrict__ rnode, const double* __restrict__ cth, const double* __restrict__ sth,
    const double* __restrict__ cs, int n_theta, int n_phi, int64_t n_grid,
    const double* __restrict__ atoms, const double* __restrict__ dirs, int n_atoms,
    const float* __restrict__ coef, double* __restrict__ rho) {
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < n_grid;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double x, y, z;
    int ir, j;
    grid_point(g, rnode, cth, sth, cs, n_theta, n_phi, x, y, z, ir, j);
    double acc = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
      double phi[kChan];
      channels(x - atoms[3 * a], y - atoms[3 * a + 1], z - atoms[3 * a + 2], dirs + 3 * a, phi);
#pragma unroll
      for (int q = 0; q < kChan; ++q) acc += static_cast<double>(coef[kChan * a + q]) * phi[q];
    }
    rho[g] += acc;
  }
}

// Per cluster c (one workgroup): y = M c (M symmetric, read by columns so
// consecutive threads read consecutive addresses), loss = c.y - 2 p.c + t,
// gout = scale (2 y - 2 p).
__global__ __launch_bounds__(256) void k_cluster_quad_loss(
    const int64_t* __restrict__ row_off, const int64_t* __restrict__ m_off,
    const float* __restrict__ Mall, const float* __restrict__ pall, const float* __restrict__ tall,
    const float* __restrict__ out, float* __restrict__ gout, float* __restrict__ loss,
    float scale, int max_nq) {
  extern __shared__ float cvec[];
  __shared__ float red[4];
  const int c = blockIdx.x;
  const int64_t r0 = row_off[c];
  const int64_t nq64 = (row_off[c + 1] - r0) * kChan;
  if (nq64 < 0 || nq64 > max_nq) {   // cluster larger than the launch allows
    if (threadIdx.x == 0) loss[c] = __builtin_nanf("");
    return;
  }
  const int nq = static_cast<int>(nq64);
  const float* M = Mall + m_off[c];
  const float* p = pall + r0 * kChan;
  const float* x = out + r0 * kChan;
  for (int i = threadIdx.x; i < nq; i += blockDim.x) cvec[i] = x[i];
  __syncthreads();
  float part = 0.f;
  for (int i = threadIdx.x; i < nq; i += blockDim.x) {
    float y = 0.f;
    for (int jj = 0; jj < nq; ++jj) y += M[static_cast<int64_t>(jj) * nq + i] * cvec[jj];
    part += cvec[i] * (y - 2.f * p[i]);
    gout[r0 * kChan + i] = scale * (2.f * y - 2.f * p[i]);
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) loss[c] = red[0] + red[1] + red[2] + red[3] + tall[c];
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_gemm_f32(bool ta, bool tb, const float* A, int lda, const float* B, int ldb, float* C,
                     int ldc, int M, int N, int K, float alpha, float beta, hipStream_t s) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  if (!ta && !tb) k_gemm_f32<false, false><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
  else if (ta && !tb) k_gemm_f32<true, false><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
  else if (!ta && tb) k_gemm_f32<false, true><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
  else k_gemm_f32<true, true><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K, alpha, beta);
}

void launch_standardize(const float* X, const float* mean, const float* sd, float* H,
                        int64_t rows, int cols, hipStream_t s) {
  k_standardize<<<grid1d(rows * cols), 256, 0, s>>>(X, mean, sd, H, rows, cols);
}
void launch_bias_act(float* Z, const float* b, float* H, int64_t rows, int cols, bool act,
                     hipStream_t s) {
  k_bias_act<<<grid1d(rows * cols), 256, 0, s>>>(Z, b, H, rows, cols, act ? 1 : 0);
}
void launch_act_grad(float* G, const float* Z, int64_t n, hipStream_t s) {
  k_act_grad<<<grid1d(n), 256, 0, s>>>(G, Z, n);
}
void launch_colsum(const float* G, float* db, int64_t rows, int cols, hipStream_t s) {
  k_colsum<<<(cols + 63) / 64, 256, 0, s>>>(G, db, rows, cols);
}
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s) {
  k_adam<<<grid1d(n), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void launch_fit_columns(const Basis& b, const double* atoms, const double* dirs, int n_atoms,
                        const double* target, double* F, hipStream_t s) {
  k_fit_columns<<<grid1d(b.n_grid), 256, 0, s>>>(b.dev_rnode, b.dev_wr, b.dev_cth, b.dev_sth,
                                                 b.t64.wt, b.dev_cs, b.n_theta, b.n_phi, b.n_grid,
                                                 atoms, dirs, n_atoms, target, F);
}

void launch_density_correction(const Basis& b, const double* atoms, const double* dirs,
                               int n_atoms, const float* coef, double* rho, hipStream_t s) {
  k_density_correction<<<grid1d(b.n_grid), 256, 0, s>>>(b.dev_rnode, b.dev_cth, b.dev_sth,
                                                        b.dev_cs, b.n_theta, b.n_phi, b.n_grid,
                                                        atoms, dirs, n_atoms, coef, rho);
}

void launch_cluster_quad_loss(int n_clusters, const int64_t* row_off, const int64_t* m_off,
                              const float* M, const float* p, const float* t, const float* out,
                              float* gout, float* loss, float scale, int max_nq, hipStream_t s) {
  k_cluster_quad_loss<<<n_clusters, 256, size_t(max_nq) * sizeof(float), s>>>(
      row_off, m_off, M, p, t, out, gout, loss, scale, max_nq);
}

}  // namespace ces
