// Block kernels of LOBPCG (Section 3.1): the residuals of the active
// (unconverged) Ritz pairs gathered into the search block, the diagonal
// Teter-Payne-Allan preconditioner of Section 3.1.2 applied to them, and
// column gathers of the conjugate directions.  All FP64, HBM-bound
// streaming over column-major d x n blocks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ces_internal.h"

namespace ces {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// W[:, j] = AX[:, a_j] - theta[a_j] X[:, a_j] for the active list a; per block
// partial sums of |r|^2 and (Lambda / 2) |r|^2 into part[j][0 or 1][block].
__global__ __launch_bounds__(kThreads) void k_active_residual(
    const double* __restrict__ X, int64_t ldx, const double* __restrict__ AX, int64_t ldax,
    const double* __restrict__ theta, const int* __restrict__ act, double* __restrict__ W,
    int64_t ldw, const double* __restrict__ lam, int64_t rows,
    double* __restrict__ part) {
  __shared__ double red[2][kThreads / 64];
  const int j = blockIdx.y, nb = gridDim.x;
  const int c = act[j];
  const double th = theta[c];
  const double* x = X + c * ldx;
  const double* ax = AX + c * ldax;
  double* w = W + j * ldw;
  double s2 = 0.0, sk = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(nb) * kThreads) {
    const double r = ax[e] - th * x[e];
    w[e] = r;
    const double r2 = r * r;
    s2 += r2;
    sk += 0.5 * lam[e] * r2;
  }
  s2 = wave_sum(s2);
  sk = wave_sum(sk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = s2;
    red[1][wv] = sk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int u = 0; u < kThreads / 64; ++u) {
      t0 += red[0][u];
      t1 += red[1][u];
    }
    part[(static_cast<int64_t>(j) * 2 + 0) * nb + blockIdx.x] = t0;
    part[(static_cast<int64_t>(j) * 2 + 1) * nb + blockIdx.x] = t1;
  }
}

// ke[j] = sum (Lambda/2) r^2 / sum r^2: the kinetic energy of residual j per
// unit norm (0 for a zero residual).
__global__ void k_kinetic_per_norm(const double* __restrict__ part, int nb, int na,
                                   double* __restrict__ ke) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < na; j += gridDim.x * blockDim.x) {
    double s2 = 0.0, sk = 0.0;
    for (int b = 0; b < nb; ++b) {
      s2 += part[(static_cast<int64_t>(j) * 2 + 0) * nb + b];
      sk += part[(static_cast<int64_t>(j) * 2 + 1) * nb + b];
    }
    ke[j] = s2 > 0.0 ? sk / s2 : 0.0;
  }
}

// W[alpha, j] *= T(g), g = g_scale Lambda_alpha / ke[j],
// T(g) = (27 + 18 g + 12 g^2 + 8 g^3) / (27 + 18 g + 12 g^2 + 8 g^3 + 16 g^4).
__global__ __launch_bounds__(kThreads) void k_tpa_scale(double* __restrict__ W, int64_t ldw,
                                                        const double* __restrict__ ke,
                                                        const double* __restrict__ lam,
                                                        double g_scale, int64_t rows) {
  const int j = blockIdx.y;
  const double kej = ke[j];
  if (!(kej > 0.0)) return;   // zero residual: nothing to scale
  const double inv = g_scale / kej;
  double* w = W + j * ldw;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double g = lam[e] * inv;
    const double num = 27.0 + g * (18.0 + g * (12.0 + 8.0 * g));
    const double g2 = g * g;
    w[e] *= num / (num + 16.0 * g2 * g2);
  }
}

// dst[:, j] = src[:, list[j]]
__global__ __launch_bounds__(kThreads) void k_gather_cols(const double* __restrict__ src,
                                                          int64_t lds, const int* __restrict__ list,
                                                          double* __restrict__ dst, int64_t ldd,
                                                          int64_t rows) {
  const int j = blockIdx.y;
  const double* s = src + list[j] * lds;
  double* d = dst + j * ldd;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * kThreads)
    d[e] = s[e];
}

unsigned stream_blocks(int64_t rows, int cols) {
  // about 4 waves of 256-thread blocks per CU over all columns
  const int64_t want = std::max<int64_t>(1, 2048 / std::max(cols, 1));
  return static_cast<unsigned>(std::min<int64_t>((rows + kThreads - 1) / kThreads, want));
}

}  // namespace

int lobpcg_residual_blocks(int64_t rows, int na) {
  return static_cast<int>(std::min<unsigned>(stream_blocks(rows, na), 64u));
}

void launch_active_residual(const double* X, int64_t ldx, const double* AX, int64_t ldax,
                            const double* theta, const int* act, int na, double* W, int64_t ldw,
                            const double* lam, int64_t rows, double* part, double* ke,
                            hipStream_t s) {
  const int nb = lobpcg_residual_blocks(rows, na);
  k_active_residual<<<dim3(nb, na), kThreads, 0, s>>>(X, ldx, AX, ldax, theta, act, W, ldw,
                                                      lam, rows, part);
  k_kinetic_per_norm<<<(na + 255) / 256, 256, 0, s>>>(part, nb, na, ke);
}

void launch_tpa_scale(double* W, int64_t ldw, int na, const double* ke, const double* lam,
                      double g_scale, int64_t rows, hipStream_t s) {
  k_tpa_scale<<<dim3(stream_blocks(rows, na), na), kThreads, 0, s>>>(W, ldw, ke, lam, g_scale,
                                                                    rows);
}

void launch_gather_cols(const double* src, int64_t lds, const int* list, int n, double* dst,
                        int64_t ldd, int64_t rows, hipStream_t s) {
  k_gather_cols<<<dim3(stream_blocks(rows, n), n), kThreads, 0, s>>>(src, lds, list, dst, ldd,
                                                                    rows);
}

}  // namespace ces
