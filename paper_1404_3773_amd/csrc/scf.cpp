// Self-consistent field extras of the C interface (declared in include/ces.h):
// Hartree potential (Section 2.3.1), the Kohn-Sham effective potential of the
// cluster model (Section 2.1, LDA exchange only), Anderson mixing of
// potentials (Section 3.4.1), the superposition-of-atomic-densities start
// (Section 3.2) and the SCF driver, which sequences the eigensolver calls of
// this library on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "ces_internal.h"
#include "setup_tables.h"

namespace ces {
namespace {

constexpr int kLanczosSteps = 20;
constexpr int kMaxHistory = 64;

// Inverse transform of one coefficient vector with the Hartree radial table
// in place of R_ln: V_H on the grid.
void hartree_to_grid(const Basis& b, const Layout& ly, void* work, const double* tau,
                     double* vh, hipStream_t s) {
  DevTables<double> th = b.t64;
  th.RiT = b.dev_hart;
  double* G = Ptr<double>::at(work, ly.G);
  double* g = Ptr<double>::at(work, ly.gbuf);
  launch_radial_inverse<double>(b, th, tau, b.d, G, 1, kColPad, s);
  launch_legendre_synth<double>(b, b.t64, G, g, kColPad, s);
  launch_phi_synthesis_one(b, g, vh, s);
}

// min || sum_t c_t F_t ||_2 subject to sum_t c_t = 1 over the columns in
// `cols`, from their Gram matrix G (m x m, column-major over all columns):
// the bordered system [G 1; 1^T 0] [c; mu] = [0; 1], solved by Gaussian
// elimination with partial pivoting after scaling G by its largest diagonal.
bool solve_bordered(const std::vector<double>& G, int m, const std::vector<int>& cols,
                    std::vector<double>& c) {
  const int q = static_cast<int>(cols.size());
  const int n = q + 1;
  double gmax = 0.0;
  for (int t = 0; t < q; ++t) gmax = std::max(gmax, G[size_t(cols[t]) * m + cols[t]]);
  if (!(gmax > 0.0) || !std::isfinite(gmax)) gmax = 1.0;
  std::vector<double> M(size_t(n) * n, 0.0), rhs(n, 0.0);
  for (int i = 0; i < q; ++i) {
    for (int j = 0; j < q; ++j) M[size_t(i) * n + j] = G[size_t(cols[j]) * m + cols[i]] / gmax;
    M[size_t(i) * n + q] = 1.0;
    M[size_t(q) * n + i] = 1.0;
  }
  rhs[q] = 1.0;
  double amax = 0.0;
  for (double v : M) amax = std::max(amax, std::fabs(v));
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int i = col + 1; i < n; ++i)
      if (std::fabs(M[size_t(i) * n + col]) > std::fabs(M[size_t(piv) * n + col])) piv = i;
    if (!(std::fabs(M[size_t(piv) * n + col]) > 1e-13 * amax)) return false;
    if (piv != col) {
      for (int j = 0; j < n; ++j) std::swap(M[size_t(piv) * n + j], M[size_t(col) * n + j]);
      std::swap(rhs[piv], rhs[col]);
    }
    for (int i = col + 1; i < n; ++i) {
      const double f = M[size_t(i) * n + col] / M[size_t(col) * n + col];
      if (f == 0.0) continue;
      for (int j = col; j < n; ++j) M[size_t(i) * n + j] -= f * M[size_t(col) * n + j];
      rhs[i] -= f * rhs[col];
    }
  }
  std::vector<double> x(n);
  for (int i = n - 1; i >= 0; --i) {
    double acc = rhs[i];
    for (int j = i + 1; j < n; ++j) acc -= M[size_t(i) * n + j] * x[j];
    x[i] = acc / M[size_t(i) * n + i];
  }
  c.assign(m, 0.0);
  for (int t = 0; t < q; ++t) {
    if (!std::isfinite(x[t])) return false;
    c[cols[t]] = x[t];
  }
  return true;
}

size_t anderson_bytes(int64_t n, int m) {
  return align256(size_t(gram_chunks(n, m)) * m * m * 8) + align256(size_t(m) * m * 8) +
         align256(size_t(m) * 8);
}

// Regions of the SCF workspace beyond the eigensolver workspace.
struct ScfLayout {
  size_t base = 0, vin = 0, vout = 0, rho = 0, Vh = 0, Fh = 0, occ = 0, res = 0, anderson = 0,
         anderson_bytes = 0, total = 0;
};

ces_status scf_layout(Ham& h, int k, int prec, int hist, ScfLayout& L) {
  size_t b1 = 0, b2 = 0, b3 = 0;
  b1 = layout_for(h, k, prec).total;
  b2 = layout_for(h, k, CES_PREC_FP64).total;
  b3 = layout_for(h, 1, CES_PREC_FP64).total;
  if (h.scf_solver != 0) b3 = std::max(b3, lobpcg_workspace_bytes(h, k, 0, prec));
  const size_t ng = size_t(h.basis->n_grid);
  size_t off = align256(std::max(b1, std::max(b2, b3)));
  L.base = off;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.vin = take(ng * 8);
  L.vout = take(ng * 8);
  L.rho = take(ng * 8);
  L.Vh = take(ng * hist * 8);
  L.Fh = take(ng * hist * 8);
  L.occ = take(size_t(k) * 8);
  L.res = take(size_t(k) * 8);
  L.anderson_bytes = anderson_bytes(h.basis->n_grid, hist);
  L.anderson = take(L.anderson_bytes);
  L.total = off;
  return CES_OK;
}


// Fermi factor 1 / (1 + exp((lam - mu) / kT)) without overflow.
double fermi_factor(double lam, double mu, double kT) {
  const double x = (lam - mu) / kT;
  if (x > 0.0) {
    const double e = std::exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + std::exp(x));
}

// Root of a continuous g on [a, b] with g(a) and g(b) of opposite signs by
// Brent's method (Brent 1973, Algorithms for Minimization Without
// Derivatives, ch. 4): each step tries inverse quadratic interpolation
// through the last three iterates (a secant step when two coincide), and
// falls back to bisection of the bracket [b, c] whenever the interpolated
// step is not well inside it or the previous steps did not shrink enough;
// stops when the bracket half-width is within 2 eps |b| + xtol / 2.
template <typename G>
double brent_root(G g, double a, double b, double ga, double gb, double xtol) {
  double c = a, gc = ga, step = b - a, prev = step;
  for (int it = 0; it < 400; ++it) {
    if ((gb > 0.0) == (gc > 0.0)) {   // keep the root between b and c
      c = a;
      gc = ga;
      step = prev = b - a;
    }
    if (std::fabs(gc) < std::fabs(gb)) {   // b is the best estimate
      a = b;
      b = c;
      c = a;
      ga = gb;
      gb = gc;
      gc = ga;
    }
    const double tol = 2.0 * 2.220446049250313e-16 * std::fabs(b) + 0.5 * xtol;
    const double half = 0.5 * (c - b);
    if (std::fabs(half) <= tol || gb == 0.0) return b;
    if (std::fabs(prev) >= tol && std::fabs(ga) > std::fabs(gb)) {
      double p, q;
      const double sb = gb / ga;
      if (a == c) {   // secant through a and b
        p = 2.0 * half * sb;
        q = 1.0 - sb;
      } else {        // inverse quadratic through a, b, c
        const double qa = ga / gc, rb = gb / gc;
        p = sb * (2.0 * half * qa * (qa - rb) - (b - a) * (rb - 1.0));
        q = (qa - 1.0) * (rb - 1.0) * (sb - 1.0);
      }
      if (p > 0.0) q = -q;
      else p = -p;
      if (2.0 * p < std::min(3.0 * half * q - std::fabs(tol * q), std::fabs(prev * q))) {
        prev = step;
        step = p / q;
      } else {
        step = prev = half;
      }
    } else {
      step = prev = half;
    }
    a = b;
    ga = gb;
    b += std::fabs(step) > tol ? step : (half > 0.0 ? tol : -tol);
    gb = g(b);
  }
  return b;
}

}  // namespace
}  // namespace ces

using namespace ces;

extern "C" {

ces_status ces_ham_set_model(ces_ham hh, int correlation, double smearing_kT, int mix_density) {
  CES_TRY(check_ham(hh));
  if (correlation != 0 && correlation != 1)
    return fail(CES_ERR_INVALID_ARG, "correlation must be 0 or 1");
  if (mix_density != 0 && mix_density != 1)
    return fail(CES_ERR_INVALID_ARG, "mix_density must be 0 or 1");
  if (!(smearing_kT >= 0.0) || !std::isfinite(smearing_kT))
    return fail(CES_ERR_INVALID_ARG, "smearing kT must be finite and >= 0");
  hh->h.xc_correlation = correlation;
  hh->h.smear_kT = smearing_kT;
  hh->h.mix_density = mix_density;
  return CES_OK;
}

ces_status ces_ham_set_scf_eigensolver(ces_ham hh, int mode, double res_tol, int max_iter) {
  CES_TRY(check_ham(hh));
  if (mode < 0 || mode > 2) return fail(CES_ERR_INVALID_ARG, "eigensolver mode must be 0, 1 or 2");
  if (!(res_tol > 0) || !std::isfinite(res_tol) || max_iter < 1)
    return fail(CES_ERR_INVALID_ARG, "LOBPCG tolerance must be > 0 and max_iter >= 1");
  hh->h.scf_solver = mode;
  hh->h.lobpcg_tol = res_tol;
  hh->h.lobpcg_max_iter = max_iter;
  return CES_OK;
}

ces_status ces_ham_set_density_basis(ces_ham hh, ces_basis bb) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  if (!bb) {
    h.rho_basis = nullptr;
    return CES_OK;
  }
  Basis& bd = bb->b;
  const Basis& b = *h.basis;
  if (bd.n_r != b.n_r || bd.n_theta != b.n_theta || bd.n_phi != b.n_phi || bd.R != b.R ||
      bd.rule != b.rule)
    return fail(CES_ERR_INVALID_ARG, "the density basis must use the orbitals' grid "
                                     "(same R, n_r, n_theta, n_phi and radial rule)");
  if (bd.L < b.L) return fail(CES_ERR_INVALID_ARG, "the density basis must have lmax >= the "
                                                  "orbitals' lmax");
  CES_TRY(ensure_device(bd));
  if (bd.device != b.device) return fail(CES_ERR_INVALID_ARG, "bases on different devices");
  h.rho_basis = &bd;
  return CES_OK;
}

ces_status ces_pz_correlation(int64_t n, const double* d_rho, double* d_vc, double* d_ec,
                              void* stream) {
  if (n < 0) return fail(CES_ERR_INVALID_ARG, "negative length");
  if (n == 0) return CES_OK;
  if (!d_rho || !d_vc) return fail(CES_ERR_INVALID_ARG, "null density or output");
  if (d_ec && (d_ec == d_vc || d_ec == d_rho))
    return fail(CES_ERR_INVALID_ARG, "energy output must not alias the density or potential");
  launch_pz_correlation(d_rho, d_vc, d_ec, n, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_fermi_dirac(int k, const double* h_eval, double n_electrons, double kT,
                           double* h_occ, double* h_eF) {
  if (k < 1 || !h_eval || !h_occ || !h_eF) return fail(CES_ERR_INVALID_ARG, "bad arguments");
  if (!(kT > 0.0) || !std::isfinite(kT)) return fail(CES_ERR_INVALID_ARG, "kT must be > 0");
  const double half = 0.5 * n_electrons;
  if (!(half > 0.0) || !(half < k))
    return fail(CES_ERR_INVALID_ARG, "need 0 < n_electrons / 2 < k");
  double lo = h_eval[0], hi = h_eval[0];
  for (int i = 0; i < k; ++i) {
    if (!std::isfinite(h_eval[i])) return fail(CES_ERR_INVALID_ARG, "non-finite eigenvalue");
    lo = std::min(lo, h_eval[i]);
    hi = std::max(hi, h_eval[i]);
  }
  auto excess = [&](double mu) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += fermi_factor(h_eval[i], mu, kT);
    return s - half;
  };
  // the count rises monotonically from ~0 to ~k across this bracket
  lo -= 50.0 * kT + 1.0;
  hi += 50.0 * kT + 1.0;
  const double eF = brent_root(excess, lo, hi, excess(lo), excess(hi), 1e-15);
  for (int i = 0; i < k; ++i) h_occ[i] = fermi_factor(h_eval[i], eF, kT);
  *h_eF = eF;
  return CES_OK;
}

ces_status ces_slater_x(int64_t n, const double* d_rho, double* d_vx, void* stream) {
  if (n < 0) return fail(CES_ERR_INVALID_ARG, "negative length");
  if (n == 0) return CES_OK;
  if (!d_rho || !d_vx) return fail(CES_ERR_INVALID_ARG, "null density or output");
  launch_slater_x(d_rho, d_vx, n, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_hartree(ces_ham hh, const double* d_tau, double* d_vh, void* d_work,
                       size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  if (!d_tau || !d_vh) return fail(CES_ERR_INVALID_ARG, "null coefficients or output");
  Layout ly;
  CES_TRY(check_work(h, 1, CES_PREC_FP64, d_work, work_bytes, ly));
  hartree_to_grid(*h.basis, ly, d_work, d_tau, d_vh, static_cast<hipStream_t>(stream));
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_ks_potential(ces_ham hh, const double* d_rho, const double* d_rho_ion,
                            const double* d_vext, double* d_v, double* d_tau, void* d_work,
                            size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  if (!d_rho || !d_rho_ion || !d_vext || !d_v)
    return fail(CES_ERR_INVALID_ARG, "null density, ion density, V_ext or output");
  if (d_v == d_rho || d_v == d_rho_ion || d_v == d_vext)
    return fail(CES_ERR_INVALID_ARG, "output potential aliases an input");
  Layout ly;
  CES_TRY(check_work(h, 1, CES_PREC_FP64, d_work, work_bytes, ly));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the density's coefficients in the orbitals' basis (dualing) or in the
  // larger density basis on the same grid (Section 2.2.5)
  const Basis& b = h.rho_basis ? *h.rho_basis : *h.basis;
  double* tau = d_tau ? d_tau : Ptr<double>::at(d_work, ly.V3);
  double* A = Ptr<double>::at(d_work, ly.A);
  double* gh = Ptr<double>::at(d_work, ly.gbuf);
  launch_sub(d_rho, d_rho_ion, d_v, b.n_grid, s);                  // d_v <- rho - rho_ion
  launch_phi_analysis_one(b, d_v, gh, s);                          // forward transform
  launch_legendre_analysis<double>(b, b.t64, gh, A, kColPad, s);
  launch_radial_forward<double>(b, b.t64, A, nullptr, 0, nullptr, 0, tau, b.d, 1.0, 0.0, 0.0,
                                false, nullptr, 1, kColPad, s);
  hartree_to_grid(b, ly, d_work, tau, d_v, s);                      // d_v <- V_H
  launch_ks_finish(d_vext, d_rho, d_v, b.n_grid, h.xc_correlation, s);   // + V_ext + V_xc
  CES_HIP(hipGetLastError());
  return CES_OK;
}

ces_status ces_anderson_workspace_size(int64_t n, int m, size_t* bytes) {
  if (!bytes || n < 1 || m < 1 || m > kMaxHistory)
    return fail(CES_ERR_INVALID_ARG, "bad Anderson sizes (1 <= m <= 64)");
  *bytes = anderson_bytes(n, m);
  return CES_OK;
}

ces_status ces_anderson_mix(int64_t n, int m, const double* d_V, const double* d_F, int64_t ld,
                            int oldest, double beta, double* d_out, double* h_coef,
                            void* d_work, size_t work_bytes, void* stream) {
  if (n < 1 || m < 1 || m > kMaxHistory || ld < n || oldest < 0 || oldest >= m)
    return fail(CES_ERR_INVALID_ARG, "bad Anderson sizes");
  if (!d_V || !d_F || !d_out) return fail(CES_ERR_INVALID_ARG, "null history or output");
  if (!std::isfinite(beta)) return fail(CES_ERR_INVALID_ARG, "non-finite mixing parameter");
  const size_t need = anderson_bytes(n, m);
  if (!d_work || work_bytes < need)
    return fail(CES_ERR_WORKSPACE, "Anderson workspace too small: need " + std::to_string(need));
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(CES_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(d_work);
  double* part = reinterpret_cast<double*>(w);
  double* Gd = reinterpret_cast<double*>(w + align256(size_t(gram_chunks(n, m)) * m * m * 8));
  double* cd = Gd + align256(size_t(m) * m * 8) / 8;
  launch_gram(d_F, ld, d_F, ld, Gd, part, n, m, s);
  std::vector<double> G(size_t(m) * m), c;
  CES_HIP(hipMemcpyAsync(G.data(), Gd, G.size() * 8, hipMemcpyDeviceToHost, s));
  CES_HIP(hipStreamSynchronize(s));
  // columns by age, oldest first; drop the oldest while the system is singular
  std::vector<int> cols(m);
  for (int t = 0; t < m; ++t) cols[t] = (oldest + t) % m;
  bool ok = false;
  while (!cols.empty()) {
    if (solve_bordered(G, m, cols, c)) {
      ok = true;
      break;
    }
    cols.erase(cols.begin());
  }
  if (!ok) return fail(CES_ERR_INVALID_ARG, "Anderson history is not finite");
  CES_HIP(hipMemcpyAsync(cd, c.data(), size_t(m) * 8, hipMemcpyHostToDevice, s));
  launch_anderson_combine(d_V, d_F, ld, cd, m, beta, d_out, n, s);
  CES_HIP(hipGetLastError());
  CES_HIP(hipStreamSynchronize(s));
  if (h_coef) std::copy(c.begin(), c.end(), h_coef);
  return CES_OK;
}

ces_status ces_sad_density(ces_ham hh, int n_atoms, const double* h_atoms,
                           const double* h_tau00, double* d_rho, void* d_work,
                           size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  const Basis& b = *h.basis;
  if (n_atoms < 0 || (n_atoms > 0 && !h_atoms) || !h_tau00 || !d_rho)
    return fail(CES_ERR_INVALID_ARG, "bad SAD arguments");
  Layout ly;
  CES_TRY(check_work(h, 1, CES_PREC_FP64, d_work, work_bytes, ly));
  const int N0 = b.Nl[0];   // the l = 0 radial functions of the layout
  if (3 * int64_t(n_atoms) + N0 > 3 * b.d) return fail(CES_ERR_INVALID_ARG, "too many atoms");
  // rho_at(r) = Y_00 sum_n tau00[n] R_0n(r); R_0n = sqrt(2/R^3) j0(k_n r) / j1(b_0n)
  std::vector<double> buf(3 * size_t(n_atoms) + N0);
  const double c0 = std::sqrt(2.0 / (b.R * b.R * b.R)) / std::sqrt(4.0 * M_PI);
  for (int n = 0; n < N0; ++n) {
    const double z = b.zeros[n];
    if (std::fabs(z - (n + 1) * M_PI) > 1e-9 * z)
      return fail(CES_ERR_DEVICE, "l = 0 radial zeros are not multiples of pi");
    buf[3 * size_t(n_atoms) + n] = h_tau00[n] * c0 / sph_bessel_j(1, z);
  }
  std::copy(h_atoms, h_atoms + 3 * size_t(n_atoms), buf.begin());
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* dv = Ptr<double>::at(d_work, ly.V3);
  CES_HIP(hipMemcpyAsync(dv, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, s));
  launch_sad_density(b, dv, n_atoms, dv + 3 * size_t(n_atoms), d_rho, s);
  CES_HIP(hipGetLastError());
  CES_HIP(hipStreamSynchronize(s));
  return CES_OK;
}

ces_status ces_scf_workspace_size(ces_ham hh, int k, int prec, int hist, size_t* bytes) {
  if (!hh || !bytes) return fail(CES_ERR_INVALID_ARG, "null argument");
  if (k < 1 || hist < 1 || hist > kMaxHistory) return fail(CES_ERR_INVALID_ARG, "bad k or history");
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  ScfLayout L;
  CES_TRY(scf_layout(hh->h, k, prec, hist, L));
  *bytes = L.total;
  return CES_OK;
}

ces_status ces_scf(ces_ham hh, int k, double* d_X, int64_t ldx, int n_occ, const double* d_vext,
                   const double* d_rho_ion, const double* d_rho0, const double* d_v0, int degree,
                   double beta, int hist, double tol, int max_steps, int first_iters, int prec,
                   double* d_eval, double* d_rho, int* h_steps, double* h_dtheta, void* d_work,
                   size_t work_bytes, void* stream) {
  CES_TRY(check_ham(hh));
  Ham& h = hh->h;
  CES_TRY(check_block(h, k, d_X, ldx, "X"));
  if (!d_vext || !d_rho_ion || !d_rho0 || !d_v0 || !d_eval || !d_rho || !h_steps)
    return fail(CES_ERR_INVALID_ARG, "null SCF argument");
  if (n_occ < 1 || n_occ >= k || k > h.basis->d)
    return fail(CES_ERR_INVALID_ARG, "need 1 <= n_occ < k <= d");
  if (degree < 1 || max_steps < 1 || first_iters < 0 || hist < 1 || hist > kMaxHistory ||
      !(tol > 0) || !std::isfinite(beta))
    return fail(CES_ERR_INVALID_ARG, "bad SCF parameters");
  if (prec != CES_PREC_FP64 && prec != CES_PREC_MIXED)
    return fail(CES_ERR_INVALID_ARG, "unknown precision");
  ScfLayout L;
  CES_TRY(scf_layout(h, k, prec, hist, L));
  if (!d_work || work_bytes < L.total)
    return fail(CES_ERR_WORKSPACE, "SCF workspace too small: need " + std::to_string(L.total));
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(CES_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Basis& b = *h.basis;
  const int64_t ng = b.n_grid;
  void* ew = d_work;                 // eigensolver workspace at offset 0
  const size_t ewb = L.base;
  double* vin = Ptr<double>::at(d_work, L.vin);
  double* vout = Ptr<double>::at(d_work, L.vout);
  double* rho = Ptr<double>::at(d_work, L.rho);
  double* Vh = Ptr<double>::at(d_work, L.Vh);
  double* Fh = Ptr<double>::at(d_work, L.Fh);
  double* occ = Ptr<double>::at(d_work, L.occ);
  double* res = Ptr<double>::at(d_work, L.res);
  void* aw = Ptr<char>::at(d_work, L.anderson);

  std::vector<double> hocc(k, 0.0);
  for (int i = 0; i < n_occ; ++i) hocc[i] = 1.0;
  CES_HIP(hipMemcpyAsync(occ, hocc.data(), size_t(k) * 8, hipMemcpyHostToDevice, s));
  CES_HIP(hipStreamSynchronize(s));

  CES_TRY(ces_ks_potential(hh, d_rho0, d_rho_ion, d_vext, vin, nullptr, ew, ewb, stream));
  // density mixing: the history holds (rho_in, rho_out - rho_in), and V_out is
  // never formed, so its buffer holds rho_in
  const bool mixrho = h.mix_density != 0;
  double* rin = vout;
  if (mixrho)
    CES_HIP(hipMemcpyAsync(rin, d_rho0, size_t(ng) * 8, hipMemcpyDeviceToDevice, s));
  std::vector<double> theta(k), theta_old(k);
  int count = 0;   // pairs pushed into the history ring
  int step = 0;
  for (step = 1; step <= max_steps; ++step) {
    CES_TRY(ces_ham_set_veff(hh, vin, stream));
    double bnd = 0;
    CES_TRY(ces_lanczos_bound(hh, d_v0, kLanczosSteps, &bnd, ew, ewb, stream));
    auto filter_rr = [&]() -> ces_status {
      CES_TRY(ces_cheb_filter(hh, k, d_X, ldx, degree, theta[k - 1], bnd, theta[0], prec, ew, ewb,
                              stream));
      CES_TRY(ces_rayleigh_ritz(hh, k, d_X, ldx, nullptr, d_eval, res, theta.data(), nullptr,
                                CES_PREC_FP64, ew, ewb, stream));
      return CES_OK;
    };
    // LOBPCG to the handle's residual tolerance on all k states (Section 3.1):
    // in the first step only (h.scf_solver == 1), or in every step (2)
    auto lobpcg = [&]() -> ces_status {
      int its = 0;
      CES_TRY(ces_lobpcg(hh, k, d_X, ldx, 0, nullptr, 0, k, h.lobpcg_max_iter, h.lobpcg_tol, 1.0,
                         1, prec, d_eval, res, &its, nullptr, ew, ewb, stream));
      CES_HIP(hipMemcpy(theta.data(), d_eval, size_t(k) * 8, hipMemcpyDeviceToHost));
      return CES_OK;
    };
    if (h.scf_solver == 2 || (step == 1 && h.scf_solver == 1)) {
      CES_TRY(lobpcg());
    } else if (step == 1) {
      CES_TRY(ces_rayleigh_ritz(hh, k, d_X, ldx, nullptr, d_eval, res, theta.data(), nullptr,
                                CES_PREC_FP64, ew, ewb, stream));
      for (int it = 0; it < first_iters; ++it) CES_TRY(filter_rr());
    } else {
      CES_TRY(filter_rr());
    }
    if (h.smear_kT > 0.0) {   // Fermi-Dirac occupations of this step's Ritz values
      double eF = 0.0;
      CES_TRY(ces_fermi_dirac(k, theta.data(), 2.0 * n_occ, h.smear_kT, hocc.data(), &eF));
      CES_HIP(hipMemcpyAsync(occ, hocc.data(), size_t(k) * 8, hipMemcpyHostToDevice, s));
      CES_HIP(hipStreamSynchronize(s));   // hocc is reused next step
    }
    CES_TRY(ces_density(hh, k, d_X, ldx, occ, rho, nullptr, CES_PREC_FP64, ew, ewb, stream));
    if (!mixrho)
      CES_TRY(ces_ks_potential(hh, rho, d_rho_ion, d_vext, vout, nullptr, ew, ewb, stream));
    double dmax = std::numeric_limits<double>::infinity();
    if (step > 1) {
      dmax = 0.0;
      for (int i = 0; i < n_occ; ++i) dmax = std::max(dmax, std::fabs(theta[i] - theta_old[i]));
    }
    if (h_dtheta) h_dtheta[step - 1] = dmax;
    if (dmax < tol) break;
    theta_old = theta;
    if (step == max_steps) break;
    const int slot = count % hist;
    double* xin = mixrho ? rin : vin;            // the mixed quantity, in
    const double* xout = mixrho ? rho : vout;    // and out
    launch_copy2d(xin, ng, Vh + size_t(slot) * ng, ng, ng, 1, s);
    launch_sub(xout, xin, Fh + size_t(slot) * ng, ng, s);
    ++count;
    const int m = std::min(count, hist);
    const int oldest = count <= hist ? 0 : count % hist;
    CES_TRY(ces_anderson_mix(ng, m, Vh, Fh, ng, oldest, beta, xin, nullptr, aw, L.anderson_bytes,
                             stream));
    if (mixrho)
      CES_TRY(ces_ks_potential(hh, rin, d_rho_ion, d_vext, vin, nullptr, ew, ewb, stream));
  }
  *h_steps = std::min(step, max_steps);
  CES_HIP(hipMemcpyAsync(d_rho, rho, size_t(ng) * 8, hipMemcpyDeviceToDevice, s));
  CES_HIP(hipStreamSynchronize(s));
  return CES_OK;
}

}  // extern "C"
