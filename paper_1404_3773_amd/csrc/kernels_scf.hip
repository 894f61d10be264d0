// HIP kernels (gfx950) of the self-consistent field extras: grid-pointwise
// pieces of the Kohn-Sham potential (Section 2.1: V_eff = V_ext + V_H + V_x,
// LDA exchange in the Slater form), the Anderson mixing combination
// (Section 3.4.1), and the superposition-of-atomic-densities start
// (Section 3.2).  All of them stream grid-sized FP64 arrays once and are
// bound by HBM bandwidth; they use grid-stride loops over flat indices.
#include <hip/hip_runtime.h>

#include "ces_internal.h"

namespace ces {

namespace {

inline int grid1d(int64_t n) {
  int64_t g = (n + 255) / 256;
  return static_cast<int>(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

// out = a - b
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ out, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[e] = a[e] - b[e];
}

// Slater (LDA) exchange potential V_x = -(3 rho_+ / pi)^(1/3), rho_+ =
// max(rho, 0): negative densities from quadrature noise count as zero.
__device__ __forceinline__ double slater_vx(double rho) {
  return -cbrt((3.0 / M_PI) * (rho > 0.0 ? rho : 0.0));
}

// vx[g] = V_x(rho[g]); vx may be rho (each element is read before it is written)
__global__ void k_slater_x(const double* rho, double* vx, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    vx[e] = slater_vx(rho[e]);
}

// Perdew-Zunger (1981) fit of the Ceperley-Alder correlation energy per
// electron of the unpolarised gas (the LDA of Section 2.1), r_s =
// (3 / (4 pi rho))^(1/3):
//   r_s >= 1:  eps = gamma / (1 + beta1 sqrt(r_s) + beta2 r_s)
//   r_s < 1:   eps = A ln r_s + B + C r_s ln r_s + D r_s
// v = d(rho eps)/d rho = eps - (r_s / 3) d eps / d r_s; rho <= 0 gives 0.
__device__ __forceinline__ void pz81(double rho, double& eps, double& v) {
  eps = 0.0;
  v = 0.0;
  if (!(rho > 0.0)) return;
  const double rs = cbrt(3.0 / (4.0 * M_PI * rho));
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs), den = 1.0 + b1 * sq + b2 * rs;
    eps = g / den;
    // v = eps (1 + 7/6 b1 sqrt(r_s) + 4/3 b2 r_s) / den
    v = eps * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double ln = log(rs);
    eps = A * ln + B + C * rs * ln + D * rs;
    v = A * ln + (B - A / 3.0) + (2.0 / 3.0) * C * rs * ln + ((2.0 * D - C) / 3.0) * rs;
  }
}

// v[g] = vext[g] + v[g] + V_x(rho[g]) [+ v_c(rho[g]) when corr]   (v holds
// V_H on entry)
__global__ void k_ks_finish(const double* __restrict__ vext, const double* __restrict__ rho,
                            double* __restrict__ v, int64_t n, int corr) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double r = rho[e];
    double out = vext[e] + v[e] + slater_vx(r);
    if (corr) {
      double eps, vc;
      pz81(r, eps, vc);
      out += vc;
    }
    v[e] = out;
  }
}

// vc[g] = v_c(rho[g]) and, when ec is not null, ec[g] = eps_c(rho[g]); vc may
// be rho (each element is read before it is written)
__global__ void k_pz_correlation(const double* rho, double* vc, double* ec, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double eps, v;
    pz81(rho[e], eps, v);
    vc[e] = v;
    if (ec) ec[e] = eps;
  }
}

// out[g] = sum_i c_i (V[g][i] + beta F[g][i]),  V, F column-major n x m.
__global__ void k_anderson_combine(const double* __restrict__ V, const double* __restrict__ F,
                                   int64_t ld, const double* __restrict__ c, int m, double beta,
                                   double* __restrict__ out, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc += c[i] * (V[i * ld + e] + beta * F[i * ld + e]);
    out[e] = acc;
  }
}

// rho[r][j][p] = sum_atoms sum_n cn[n] j0(k_n |x - a|), k_n = (n+1) pi / R
// (the zeros of j_0 are the multiples of pi), zero where |x - a| >= R.
// sin((n+1) u) by the three-term recurrence s_{n+1} = 2 cos(u) s_n - s_{n-1}.
__global__ __launch_bounds__(256) void k_sad_density(
    const double* __restrict__ rnode, const double* __restrict__ cth,
    const double* __restrict__ sth, const double* __restrict__ cs, const double* __restrict__ atoms,
    int n_atoms, const double* __restrict__ cn, int N, double R, int n_theta, int n_phi,
    int64_t n_grid, double* __restrict__ rho) {
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < n_grid;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int p = static_cast<int>(g % n_phi);
    const int64_t rj = g / n_phi;
    const int j = static_cast<int>(rj % n_theta);
    const int ir = static_cast<int>(rj / n_theta);
    const double r = rnode[ir];
    const double x = r * sth[j] * cs[p], y = r * sth[j] * cs[n_phi + p], z = r * cth[j];
    double acc = 0.0;
    for (int a = 0; a < n_atoms; ++a) {
      const double dx = x - atoms[3 * a], dy = y - atoms[3 * a + 1], dz = z - atoms[3 * a + 2];
      const double rr = sqrt(dx * dx + dy * dy + dz * dz);
      if (rr >= R) continue;
      if (rr == 0.0) {
        for (int n = 0; n < N; ++n) acc += cn[n];
        continue;
      }
      const double u = M_PI * rr / R;
      double su, cu;
      sincos(u, &su, &cu);
      const double c2 = 2.0 * cu;
      double s_prev = 0.0, s_cur = su;   // sin(0 u), sin(1 u)
      double part = 0.0;
      for (int n = 0; n < N; ++n) {
        part += cn[n] * s_cur / static_cast<double>(n + 1);
        const double s_next = c2 * s_cur - s_prev;
        s_prev = s_cur;
        s_cur = s_next;
      }
      acc += part / u;   // j0(k_n rr) = sin((n+1) u) / ((n+1) u)
    }
    rho[g] = acc;
  }
}

}  // namespace

void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s) {
  k_sub<<<grid1d(n), 256, 0, s>>>(a, b, out, n);
}

void launch_ks_finish(const double* vext, const double* rho, double* v, int64_t n, int corr,
                      hipStream_t s) {
  k_ks_finish<<<grid1d(n), 256, 0, s>>>(vext, rho, v, n, corr);
}

void launch_pz_correlation(const double* rho, double* vc, double* ec, int64_t n,
                           hipStream_t s) {
  k_pz_correlation<<<grid1d(n), 256, 0, s>>>(rho, vc, ec, n);
}

void launch_slater_x(const double* rho, double* vx, int64_t n, hipStream_t s) {
  k_slater_x<<<grid1d(n), 256, 0, s>>>(rho, vx, n);
}

void launch_anderson_combine(const double* V, const double* F, int64_t ld, const double* c,
                             int m, double beta, double* out, int64_t n, hipStream_t s) {
  k_anderson_combine<<<grid1d(n), 256, 0, s>>>(V, F, ld, c, m, beta, out, n);
}

void launch_sad_density(const Basis& b, const double* atoms, int n_atoms, const double* cn,
                        double* rho, hipStream_t s) {
  k_sad_density<<<grid1d(b.n_grid), 256, 0, s>>>(b.dev_rnode, b.dev_cth, b.dev_sth, b.dev_cs,
                                                 atoms, n_atoms, cn, b.Nl[0], b.R, b.n_theta,
                                                 b.n_phi, b.n_grid, rho);
}

}  // namespace ces
