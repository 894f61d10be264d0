// Host (CPU, FP64) setup tables for the spectral basis on a ball.
//
// Section 2.2.1: radial functions R_ln(r) = sqrt(2/R^3) j_l(b_ln r/R) /
// j_{l+1}(b_ln) (the spherical-Bessel form of eq. spherical_bessel_1), with
// b_ln the (n+1)-th positive zero of j_l; normalised associated Legendre
// functions c_lm P_l^m without the Condon-Shortley phase.
// Section 2.2.2: Gauss-Jacobi (weight r^2) or Gauss-Legendre radial nodes and
// Gauss-Legendre nodes in cos(theta), computed by the Golub-Welsch method.
// Section 4 (implementation notes): Bessel zeros by Halley's method.
#pragma once
#include <vector>

namespace ces {

// Spherical Bessel function j_l(x), x >= 0: upward recurrence where it is
// stable (x > l), Miller's downward recurrence normalised by
// sum_n (2n+1) j_n(x)^2 = 1 otherwise.
double sph_bessel_j(int l, double x);

// zeros[l*N + n] = (n+1)-th positive zero of j_l, l < L, n < N.
std::vector<double> bessel_zeros(int L, int N);

// Gauss-Jacobi rule for the weight (1-x)^alpha (1+x)^beta on [-1,1]:
// nodes ascending, weights summing to the weight's integral.
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x,
                  std::vector<double>& w);

// Normalised associated Legendre functions at one point t:
// out[l*(l+1)/2 + m] = c_lm P_l^m(t), 0 <= m <= l < L, no Condon-Shortley phase.
void legendre_normalized(int L, double t, double* out);

}  // namespace ces
