// HIP kernels (gfx950): V_eff phi-Fourier sums, the complex <-> real
// coefficient maps, and small FP64 helpers of Cholesky-QR, Rayleigh-Ritz and
// Lanczos.  The H*X stages are in kernels_radial.hip and
// kernels_angular.hip.
//
// phi stage of H*X.  With f(phi) = sum_m g^c_m cos(m phi) + g^s_m sin(m phi), the
// analysis of V f over the uniform phi grid is, exactly,
//   gh^c_m' = sum_m (a_{|m-m'|} + a_{m+m'}) g^c_m + (b_{m+m'} + b_{m-m'}) g^s_m
//   gh^s_m' = sum_m (b_{m'+m} + b_{m'-m}) g^c_m + (a_{|m-m'|} - a_{m+m'}) g^s_m
// with a_q, b_q = (pi / N_phi) sum_p V_p {cos, sin}(q phi_p), b_{-q} = -b_q
// (product-to-sum identities; |q| <= 2L-2 < N_phi).  a, b depend on V only,
// so they are computed once per V_eff and the per-orbital work needs no FFT.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ces_internal.h"

namespace ces {

namespace {

// ab[r][j][0][q] = (pi/N_phi) sum_p V cos(q phi_p), ab[..][1][q] the sine sums;
// cs holds cos / sin(2 pi u / N_phi), u < N_phi, indexed by (q p) mod N_phi.
__global__ void k_veff_fourier(const double* __restrict__ V, const double* __restrict__ cs,
                               double* __restrict__ ab64, float* __restrict__ ab32, int n_phi,
                               int S, double scale) {
  const int64_t rj = blockIdx.x;
  const double* v = V + rj * n_phi;
  for (int q = threadIdx.x; q < 2 * S; q += blockDim.x) {
    const bool sn = q >= S;
    const int qq = sn ? q - S : q;
    const double* tab = cs + (sn ? n_phi : 0);
    double acc = 0.0;
    int u = 0;
    for (int p = 0; p < n_phi; ++p) {
      acc += v[p] * tab[u];
      u += qq;
      if (u >= n_phi) u -= n_phi;
    }
    ab64[rj * 2 * S + q] = scale * acc;
    ab32[rj * 2 * S + q] = static_cast<float>(scale * acc);
  }
}

// --------------------------------------------------------------- utilities

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ src, int64_t lds, Tout* __restrict__ dst,
                          int64_t ldd, int64_t rows, int cols) {
  const int c = blockIdx.y;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[c * ldd + e] = static_cast<Tout>(src[c * lds + e]);
  (void)cols;
}

__global__ void k_scale_gram(double* S, int k, double* dinv) {
  // one block; dinv_i = 1/sqrt(S_ii), S_ij *= dinv_i dinv_j
  for (int i = threadIdx.x; i < k; i += blockDim.x) dinv[i] = 1.0 / sqrt(S[i * (int64_t)k + i]);
  __syncthreads();
  for (int64_t e = threadIdx.x; e < int64_t(k) * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    S[e] *= dinv[i] * dinv[j];
  }
}

__global__ void k_scale_cols(double* X, int64_t ldx, int64_t rows, const double* dinv) {
  const int c = blockIdx.y;
  const double s = dinv[c];
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    X[c * ldx + e] *= s;
}

__global__ void k_symmetrize(double* S, int k) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
       e < int64_t(k) * k; e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = e % k, j = e / k;
    if (i < j) {
      const double v = 0.5 * (S[e] + S[int64_t(i) * k + j]);
      S[e] = v;
      S[int64_t(i) * k + j] = v;
    }
  }
}

// Zero the strictly lower triangle of a column-major k x k matrix.
__global__ void k_zero_lower(double* S, int k) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
       e < int64_t(k) * k; e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int i = e % k, j = e / k;
    if (i > j) S[e] = 0.0;
  }
}

// One wave: the first j with R_jj^2 <= 2 k eps (R from potrf of a matrix with
// unit diagonal) fails the factorisation if potrf itself did not.
__global__ void k_check_pivots(const double* R, int k, int* info) {
  const double ptol = 2.0 * k * 2.220446049250313e-16;
  int first = 0x7fffffff;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double r = R[int64_t(j) * k + j];
    if (!(r * r > ptol) && j < first) first = j;
  }
  for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_down(first, o, 64));
  if (threadIdx.x == 0 && first != 0x7fffffff && info[0] == 0) info[0] = first + 1;
}

__global__ void k_add_diag(double* S, int k, double shift) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x)
    S[int64_t(i) * k + i] += shift;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int u = 0; u < (int)(blockDim.x + 63) / 64; ++u) t += red[u];
  return t;
}

// Two-pass reductions over long vectors: per-block partial sums, then one
// thread per result.  res_c = || HX_c - theta_c X_c ||_2 and dot = x . y.
__global__ __launch_bounds__(256) void k_residual_partial(const double* HX, int64_t ldh,
                                                          const double* X, int64_t ldx,
                                                          const double* theta, double* part,
                                                          int64_t rows) {
  __shared__ double red[4];
  const int c = blockIdx.y, nb = gridDim.x;
  const double th = theta[c];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(nb) * blockDim.x) {
    const double v = HX[c * ldh + e] - th * X[c * ldx + e];
    acc += v * v;
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[static_cast<int64_t>(c) * nb + blockIdx.x] = t;
}

__global__ void k_finish_sums(const double* part, int nb, int ncol, double* out, int take_sqrt) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncol; c += gridDim.x * blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[static_cast<int64_t>(c) * nb + b];
    out[c] = take_sqrt ? sqrt(t) : t;
  }
}

__global__ void k_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd,
                         int64_t rows) {
  const int c = blockIdx.y;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[c * ldd + e] = src[c * lds + e];
}

__global__ __launch_bounds__(256) void k_dot_partial(const double* x, const double* y, int64_t n,
                                                     double* part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    acc += x[e] * y[e];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}


// S(i, j) *= dinv[i] for a k x k column-major matrix
__global__ void k_scale_rows_k(double* S, int k, const double* dinv) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x)
    S[e] *= dinv[e % k];
}

// dst = src where flags[0] == 0 and flags[1] == 0 (device-side guard)
__global__ void k_copy2d_if(const double* src, int64_t lds, double* dst, int64_t ldd,
                            int64_t rows, const int* flags) {
  if (flags[0] != 0 || flags[1] != 0) return;
  const int c = blockIdx.y;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < rows;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[c * ldd + e] = src[c * lds + e];
}

inline int grid1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  return static_cast<int>(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

// Complex <-> real harmonic coefficients, one thread per output entry
// (alpha, column i) of d x k interleaved complex blocks.  With mu = |m| > 0,
// each (l, n) pairs f_{+mu} and f_{-mu}:
//   complex -> real   s_{+mu} = (f_{+mu} + f_{-mu}) / sqrt2
//                     s_{-mu} = i (f_{+mu} - f_{-mu}) / sqrt2
//   real -> complex   f_{+mu} = (s_{+mu} - i s_{-mu}) / sqrt2
//                     f_{-mu} = (s_{+mu} + i s_{-mu}) / sqrt2
// and m = 0 is copied.  in and out do not overlap (checked by the caller).
// The layout gives each l its first index off_l and N_l radial functions
// (lay[2l], lay[2l+1]): alpha = off_l + (l + m) N_l + n.
template <bool TO_REAL>
__global__ void k_coeffs_map(const double2* __restrict__ in, int64_t ldi,
                             double2* __restrict__ out, int64_t ldo,
                             const int* __restrict__ lay, int L, int64_t d, int k) {
  const int64_t total = d * k;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i = e / d, a = e - i * d;
    // l: the last l with off_l <= a (binary search over the offsets)
    int lo = 0, hi = L - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (lay[2 * mid] <= a) lo = mid; else hi = mid - 1;
    }
    const int l = lo, Nl = lay[2 * l + 1];
    const int64_t off = lay[2 * l];
    const int lmi = static_cast<int>((a - off) / Nl);       // l + m
    const int n = static_cast<int>(a - off - int64_t(lmi) * Nl);
    const int m = lmi - l, mu = m < 0 ? -m : m;
    const double2* col = in + i * ldi;
    double2 r;
    if (m == 0) {
      r = col[a];
    } else {
      const double2 p = col[off + int64_t(l + mu) * Nl + n];   // the +mu entry
      const double2 q = col[off + int64_t(l - mu) * Nl + n];   // the -mu entry
      const double h = 0.70710678118654752440;                 // 1 / sqrt2
      if (TO_REAL) {
        // s_{+mu} = (p + q) h;  s_{-mu} = i (p - q) h = (-(p - q).y, (p - q).x) h
        r = m > 0 ? make_double2((p.x + q.x) * h, (p.y + q.y) * h)
                  : make_double2(-(p.y - q.y) * h, (p.x - q.x) * h);
      } else {
        // here p = s_{+mu}, q = s_{-mu}; i q = (-q.y, q.x)
        r = m > 0 ? make_double2((p.x + q.y) * h, (p.y - q.x) * h)     // (p - i q) h
                  : make_double2((p.x - q.y) * h, (p.y + q.x) * h);    // (p + i q) h
      }
    }
    out[i * ldo + a] = r;
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_veff_fourier(const Basis& b, const double* V, double* ab64, float* ab32,
                         hipStream_t s) {
  const int S = 2 * b.L - 1;
  k_veff_fourier<<<b.n_r * b.n_theta, 128, 0, s>>>(V, b.dev_cs, ab64, ab32, b.n_phi, S,
                                                   M_PI / b.n_phi);
}

template <typename Tin, typename Tout>
void launch_convert(const Tin* src, int64_t lds, Tout* dst, int64_t ldd, int64_t rows,
                    int cols, hipStream_t s) {
  dim3 grid(grid1d(rows), cols);
  k_convert<Tin, Tout><<<grid, 256, 0, s>>>(src, lds, dst, ldd, rows, cols);
}

void launch_coeffs_c2r(const Basis& b, const double* f, int64_t ldf, double* sr, int64_t lds,
                       int k, hipStream_t s) {
  const int64_t total = b.d * k;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 8192));
  k_coeffs_map<true><<<g, 256, 0, s>>>(reinterpret_cast<const double2*>(f), ldf,
                                        reinterpret_cast<double2*>(sr), lds, b.dev_lay, b.L, b.d, k);
}

void launch_coeffs_r2c(const Basis& b, const double* sr, int64_t lds, double* f, int64_t ldf,
                       int k, hipStream_t s) {
  const int64_t total = b.d * k;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 8192));
  k_coeffs_map<false><<<g, 256, 0, s>>>(reinterpret_cast<const double2*>(sr), lds,
                                         reinterpret_cast<double2*>(f), ldf, b.dev_lay, b.L, b.d, k);
}

void launch_scale_gram(double* S, int k, double* dinv, hipStream_t s) {
  k_scale_gram<<<1, 256, 0, s>>>(S, k, dinv);
}
void launch_scale_cols(double* X, int64_t ldx, int64_t rows, int k, const double* dinv,
                       hipStream_t s) {
  dim3 grid(grid1d(rows), k);
  k_scale_cols<<<grid, 256, 0, s>>>(X, ldx, rows, dinv);
}
void launch_symmetrize(double* S, int k, hipStream_t s) {
  k_symmetrize<<<grid1d(int64_t(k) * k), 256, 0, s>>>(S, k);
}
void launch_zero_lower(double* S, int k, hipStream_t s) {
  k_zero_lower<<<grid1d(int64_t(k) * k), 256, 0, s>>>(S, k);
}
void launch_check_pivots(const double* R, int k, int* info, hipStream_t s) {
  k_check_pivots<<<1, 64, 0, s>>>(R, k, info);
}
void launch_add_diag(double* S, int k, double shift, hipStream_t s) {
  k_add_diag<<<grid1d(k), 256, 0, s>>>(S, k, shift);
}
void launch_residuals(const double* HX, int64_t ldh, const double* X, int64_t ldx,
                      const double* theta, double* res, int64_t rows, int k, double* part,
                      int64_t part_cap, hipStream_t s) {
  int64_t nb = (rows + 2047) / 2048;                 // >= 2048 rows per block
  nb = nb < 1 ? 1 : (nb > 64 ? 64 : nb);
  if (nb * k > part_cap) nb = part_cap / k > 0 ? part_cap / k : 1;
  k_residual_partial<<<dim3(static_cast<unsigned>(nb), k), 256, 0, s>>>(HX, ldh, X, ldx, theta,
                                                                         part, rows);
  k_finish_sums<<<(k + 255) / 256, 256, 0, s>>>(part, static_cast<int>(nb), k, res, 1);
}
void launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                   int cols, hipStream_t s) {
  dim3 grid(grid1d(rows), cols);
  k_copy2d<<<grid, 256, 0, s>>>(src, lds, dst, ldd, rows);
}
void launch_scale_rows_k(double* S, int k, const double* dinv, hipStream_t s) {
  k_scale_rows_k<<<grid1d(int64_t(k) * k), 256, 0, s>>>(S, k, dinv);
}
void launch_copy2d_if(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                      int cols, const int* flags, hipStream_t s) {
  dim3 grid(grid1d(rows), cols);
  k_copy2d_if<<<grid, 256, 0, s>>>(src, lds, dst, ldd, rows, flags);
}
void launch_dot(const double* x, const double* y, int64_t n, double* out, double* part,
                hipStream_t s) {
  int64_t nb = (n + 2047) / 2048;
  nb = nb < 1 ? 1 : (nb > kDotBlocks ? kDotBlocks : nb);
  k_dot_partial<<<static_cast<unsigned>(nb), 256, 0, s>>>(x, y, n, part);
  k_finish_sums<<<1, 64, 0, s>>>(part, static_cast<int>(nb), 1, out, 0);
}
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  k_axpby<<<grid1d(n), 256, 0, s>>>(a, x, b, y, n);
}


template void launch_convert<double, float>(const double*, int64_t, float*, int64_t, int64_t,
                                            int, hipStream_t);
template void launch_convert<float, double>(const float*, int64_t, double*, int64_t, int64_t,
                                            int, hipStream_t);

}  // namespace ces
