// Host FP64 special functions and quadrature rules for the basis tables.
// See setup_tables.h for what each routine computes and where the paper
// defines it.
#include "setup_tables.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace ces {

double sph_bessel_j(int l, double x) {
  if (x == 0.0) return l == 0 ? 1.0 : 0.0;
  const double s = std::sin(x), c = std::cos(x);
  const double j0 = s / x;
  if (l == 0) return j0;
  const double j1 = s / (x * x) - c / x;
  if (l == 1 && x > 1.0) return j1;
  if (x > static_cast<double>(l) && x > 1.0) {
    // Upward three-term recurrence j_{n+1} = (2n+1)/x j_n - j_{n-1}: stable
    // while the order stays below the argument.
    double jm = j0, jc = j1;
    for (int n = 1; n < l; ++n) {
      const double jn = (2.0 * n + 1.0) / x * jc - jm;
      jm = jc;
      jc = jn;
    }
    return jc;
  }
  // Miller: run the same recurrence downward from far above l with an
  // arbitrary start; the sequence becomes proportional to j_n.  The scale is
  // fixed by sum_n (2n+1) j_n(x)^2 = 1 and the sign by j_0 or j_1.
  const int nstart = l + 30 + static_cast<int>(6.0 * std::sqrt(l + 1.0));
  double fp = 0.0, fc = 1.0, fl = 0.0, sum = 0.0, f0 = 0.0, f1 = 0.0;
  for (int n = nstart; n >= 1; --n) {
    // fc = f_n, fp = f_{n+1}; produce f_{n-1}
    sum += (2.0 * n + 1.0) * fc * fc;
    if (n == l) fl = fc;
    if (n == 1) f1 = fc;
    const double fm = (2.0 * n + 1.0) / x * fc - fp;
    fp = fc;
    fc = fm;
    if (std::fabs(fc) > 1e150) {
      fc *= 1e-150;
      fp *= 1e-150;
      fl *= 1e-150;
      f1 *= 1e-150;
      sum *= 1e-300;
    }
  }
  f0 = fc;
  sum += f0 * f0;
  const double norm = 1.0 / std::sqrt(sum);
  double sign;
  if (std::fabs(j0) >= std::fabs(j1))
    sign = (j0 * f0 >= 0.0) ? 1.0 : -1.0;
  else
    sign = (j1 * f1 >= 0.0) ? 1.0 : -1.0;
  return sign * fl * norm;
}

namespace {

// j_l and its first two derivatives (from the spherical Bessel equation
// x^2 y'' + 2 x y' + (x^2 - l(l+1)) y = 0), for Halley's method.
void bessel_with_derivs(int l, double x, double& f, double& fp, double& fpp) {
  f = sph_bessel_j(l, x);
  const double fm1 = sph_bessel_j(l - 1, x);
  fp = fm1 - (l + 1.0) / x * f;
  fpp = -2.0 / x * fp - (1.0 - l * (l + 1.0) / (x * x)) * f;
}

double halley_in_bracket(int l, double lo, double hi) {
  double flo = sph_bessel_j(l, lo);
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double f, fp, fpp;
    bessel_with_derivs(l, x, f, fp, fpp);
    if (f == 0.0) return x;
    // keep the bracket around the sign change
    if ((f > 0) == (flo > 0)) {
      lo = x;
      flo = f;
    } else {
      hi = x;
    }
    const double den = 2.0 * fp * fp - f * fpp;
    double xn = (den != 0.0) ? x - 2.0 * f * fp / den : 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const double step = std::fabs(xn - x);
    x = xn;
    if (step <= 2e-16 * x || hi - lo <= 4e-16 * x) break;
  }
  return x;
}

}  // namespace

std::vector<double> bessel_zeros(int L, int N) {
  if (L < 1 || N < 1) throw std::invalid_argument("bessel_zeros: L, N >= 1");
  std::vector<double> out(static_cast<size_t>(L) * N);
  // Zeros of j_l and j_{l-1} interlace: z_{l-1,n} < z_{l,n} < z_{l-1,n+1}.
  // Order l needs N + (L-1-l) zeros so that every higher order is bracketed.
  std::vector<double> prev(N + L - 1), cur;
  for (int n = 0; n < N + L - 1; ++n) prev[n] = (n + 1) * M_PI;  // j_0 = sin x / x
  for (int n = 0; n < N; ++n) out[n] = prev[n];
  for (int l = 1; l < L; ++l) {
    const int cnt = N + (L - 1 - l);
    cur.assign(cnt, 0.0);
    for (int n = 0; n < cnt; ++n) cur[n] = halley_in_bracket(l, prev[n], prev[n + 1]);
    for (int n = 0; n < N; ++n) out[static_cast<size_t>(l) * N + n] = cur[n];
    prev.swap(cur);
  }
  return out;
}

namespace {

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..n) and off-diagonal b[0..n-1) (Sturm sequence via LDL^T).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double dd = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double e2 = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    dd = (a[i] - x) - ((i > 0) ? e2 / dd : 0.0);
    if (dd == 0.0) dd = -1e-300;
    if (dd < 0.0) ++cnt;
  }
  return cnt;
}

}  // namespace

void gauss_jacobi(int n, double al, double be, std::vector<double>& x,
                  std::vector<double>& w) {
  if (n < 1) throw std::invalid_argument("gauss_jacobi: n >= 1");
  // Three-term recurrence of the monic Jacobi polynomials:
  // p_{k+1} = (x - alpha_k) p_k - beta_k p_{k-1}.
  std::vector<double> alpha(n), beta(n + 1, 0.0);
  const double ab = al + be;
  for (int k = 0; k < n; ++k) {
    if (k == 0)
      alpha[k] = (be - al) / (ab + 2.0);
    else
      alpha[k] = (be * be - al * al) / ((2.0 * k + ab) * (2.0 * k + ab + 2.0));
  }
  for (int k = 1; k <= n; ++k) {
    const double t = 2.0 * k + ab;
    beta[k] = 4.0 * k * (k + al) * (k + be) * (k + ab) / (t * t * (t + 1.0) * (t - 1.0));
  }
  const double mu0 = std::exp((ab + 1.0) * std::log(2.0) + std::lgamma(al + 1.0) +
                              std::lgamma(be + 1.0) - std::lgamma(ab + 2.0));
  // Golub-Welsch: nodes are the eigenvalues of the Jacobi matrix; found here
  // one by one by Sturm bisection, then polished by Newton on q_n.
  std::vector<double> offd(n > 1 ? n - 1 : 0);
  for (int k = 0; k + 1 < n; ++k) offd[k] = std::sqrt(beta[k + 1]);
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double rad = (i > 0 ? std::fabs(offd[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(offd[i]) : 0.0);
    lo = std::min(lo, alpha[i] - rad);
    hi = std::max(hi, alpha[i] + rad);
  }
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-16 * std::max(1.0, std::fabs(a)); ++it) {
      const double mid = 0.5 * (a + b);
      if (sturm_count(alpha, offd, mid) > i)
        b = mid;
      else
        a = mid;
    }
    x[i] = 0.5 * (a + b);
  }
  // Orthonormal polynomials q_k (q_0 = 1/sqrt(mu0)); Newton on q_n, then
  // Christoffel numbers w = 1 / sum_{k<n} q_k(x)^2.
  auto eval = [&](double t, double& qn, double& dqn, double& ssum) {
    double qm = 0.0, qc = 1.0 / std::sqrt(mu0), dm = 0.0, dc = 0.0;
    ssum = 0.0;
    for (int k = 0; k < n; ++k) {
      ssum += qc * qc;
      const double sb1 = std::sqrt(beta[k + 1]);
      const double sbk = (k > 0) ? std::sqrt(beta[k]) : 0.0;
      const double qn1 = ((t - alpha[k]) * qc - sbk * qm) / sb1;
      const double dn1 = (qc + (t - alpha[k]) * dc - sbk * dm) / sb1;
      qm = qc;
      qc = qn1;
      dm = dc;
      dc = dn1;
    }
    qn = qc;
    dqn = dc;
  };
  for (int i = 0; i < n; ++i) {
    double t = x[i], qn, dqn, ssum;
    for (int it = 0; it < 3; ++it) {
      eval(t, qn, dqn, ssum);
      if (dqn != 0.0) t -= qn / dqn;
    }
    eval(t, qn, dqn, ssum);
    x[i] = t;
    w[i] = 1.0 / ssum;
  }
}

void legendre_normalized(int L, double t, double* out) {
  // Fully normalised recurrences for c_lm P_l^m (no Condon-Shortley phase):
  //   P_00 = 1/sqrt(4 pi),  P_mm = sqrt((2m+1)/(2m)) sin(theta) P_{m-1,m-1},
  //   P_{m+1,m} = sqrt(2m+3) t P_mm,
  //   P_lm = sqrt((4l^2-1)/(l^2-m^2)) [t P_{l-1,m}
  //          - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) P_{l-2,m}].
  const double s = std::sqrt(std::max(0.0, (1.0 - t) * (1.0 + t)));
  auto idx = [](int l, int m) { return l * (l + 1) / 2 + m; };
  double pmm = 1.0 / std::sqrt(4.0 * M_PI);
  for (int m = 0; m < L; ++m) {
    if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    out[idx(m, m)] = pmm;
    if (m + 1 < L) out[idx(m + 1, m)] = std::sqrt(2.0 * m + 3.0) * t * pmm;
    for (int l = m + 2; l < L; ++l) {
      const double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
      const double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) /
                                 (4.0 * (l - 1) * (l - 1) - 1.0));
      out[idx(l, m)] = a * (t * out[idx(l - 1, m)] - b * out[idx(l - 2, m)]);
    }
  }
}

}  // namespace ces
