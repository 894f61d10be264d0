"""Basis set, grid and coefficient layout of the spectral scheme (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows Section 2.2.1 (Laplacian eigenbasis on the ball) and Section 2.2.2
(quadrature grid) of the paper, in the paper's complex form:
  F_lmn(r,theta,phi) = R_ln(r) Y_l^m(theta,phi)                 eq. eigfunction_1
  R_ln(r) = sqrt(2/r) J_{l+1/2}(b_ln r / R) / (R J_{l+3/2}(b_ln))  eq. spherical_bessel_1
  Y_l^m   = c_lm P_l^m(cos theta) e^{i m phi},
  c_lm    = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                  eq. spherical_harmonics_1
  Lambda_lmn = (b_ln / R)^2                                    eq. laplacian_eigenvalue
with b_ln the (n+1)-th positive zero of J_{l+1/2}, no Condon-Shortley phase
(footnote to the real-function symmetry in Section 2.2.1) and
Y_l^{-m} = conj(Y_l^m), which is the reading that makes the paper's
real-function symmetry f_{l,-m,n} = conj(f_{l,m,n}) hold.

Index map (footnote in Section 2.2.3, minus one for 0-based arrays):
  alpha(l,m,n) = (l^2 + l + m) * N + n.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np
from scipy import optimize, special

RADIAL_GAUSS_JACOBI_R2 = 0
RADIAL_GAUSS_LEGENDRE = 1


# ------------------------------------------------------------ Bessel zeros

@functools.lru_cache(maxsize=64)
def bessel_zeros(L: int, N: int) -> np.ndarray:
    """b[l, n] = (n+1)-th positive zero of J_{l+1/2} (equivalently of j_l),
    l < L, n < N.  Found by a sign-change scan (zero spacing exceeds pi, so a
    0.1 step cannot skip a pair) and refined with Brent's method."""
    out = np.empty((L, N))
    for l in range(L):
        hi = (N + 0.5 * l + 4) * math.pi + 10.0   # z_{l,n} ~ (n + l/2 + 1) pi
        xs = np.arange(0.1, hi, 0.1)
        ys = special.spherical_jn(l, xs)
        idx = np.nonzero(np.sign(ys[:-1]) * np.sign(ys[1:]) < 0)[0]
        assert len(idx) >= N, (l, len(idx))
        for n in range(N):
            a, b = xs[idx[n]], xs[idx[n] + 1]
            out[l, n] = optimize.brentq(lambda x: special.spherical_jn(l, x),
                                        a, b, xtol=1e-15, rtol=1e-15, maxiter=200)
    return out


def radial_function(l: int, b: np.ndarray, r: np.ndarray, R: float) -> np.ndarray:
    """R_ln(r) for the zeros b (any shape) at radii r, written as in
    eq. spherical_bessel_1 with ordinary Bessel functions J_nu.
    Returns shape b.shape + r.shape."""
    b = np.asarray(b, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    bb = b.reshape(b.shape + (1,) * r.ndim)
    num = np.sqrt(2.0 / r) * special.jv(l + 0.5, bb * r / R)
    den = R * special.jv(l + 1.5, bb)
    return num / den


# -------------------------------------------------------------------- grid

def radial_nodes(n_r: int, R: float, rule: int):
    """Radial nodes (ascending) and weights that include the r^2 volume factor,
    so that sum_k w_k f(r_k) ~ int_0^R f(r) r^2 dr (eq. Arlm_to_coeff).
    Gauss-Jacobi: nodes of the weight r^2 on [0,R] (Section 2.2.2).
    Gauss-Legendre: plain Gauss nodes on [0,R], r^2 multiplied into weights."""
    if rule == RADIAL_GAUSS_JACOBI_R2:
        x, w = special.roots_jacobi(n_r, 0.0, 2.0)   # weight (1+x)^2 on [-1,1]
        r = R * (1.0 + x) / 2.0
        wr = w * (R / 2.0) ** 3
    elif rule == RADIAL_GAUSS_LEGENDRE:
        x, w = special.roots_legendre(n_r)
        r = R * (1.0 + x) / 2.0
        wr = w * (R / 2.0) * r * r
    else:
        raise ValueError(rule)
    order = np.argsort(r)
    return r[order], wr[order]


def theta_nodes(n_theta: int):
    """Gauss-Legendre nodes in t = cos(theta) on [-1,1] (Section 2.2.2), ordered
    by increasing theta (decreasing t); returns (theta, t, w)."""
    t, w = special.roots_legendre(n_theta)
    order = np.argsort(-t)
    t, w = t[order], w[order]
    return np.arccos(t), t, w


def phi_nodes(n_phi: int):
    """Equally spaced azimuths phi_p = 2 pi p / N_phi (Section 2.2.2)."""
    return 2.0 * math.pi * np.arange(n_phi) / n_phi


# --------------------------------------------------------------- harmonics

def legendre_table(L: int, t: np.ndarray) -> np.ndarray:
    """P[l, m, j] = c_lm P_l^m(t_j) for 0 <= m <= l < L, no Condon-Shortley
    phase (zero for m > l).  Evaluated through SciPy's normalised spherical
    harmonic, whose built-in (-1)^m phase is removed."""
    theta = np.arccos(np.clip(t, -1.0, 1.0))
    P = np.zeros((L, L, len(t)))
    for l in range(L):
        for m in range(l + 1):
            y = special.sph_harm_y(l, m, theta, 0.0).real
            P[l, m] = (-1.0) ** m * y
    return P


def c_lm(l: int, m: int) -> float:
    """Normalisation constant of eq. spherical_harmonics_1 (m >= 0)."""
    return math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.exp(math.lgamma(l - m + 1) - math.lgamma(l + m + 1)))


def Y_complex(l: int, m: int, theta, phi):
    """Y_l^m(theta, phi) of eq. spherical_harmonics_1 without the CS phase;
    negative m via Y_l^{-m} = conj(Y_l^m)."""
    am = abs(m)
    y = (-1.0) ** am * special.sph_harm_y(l, am, theta, phi)
    return y if m >= 0 else np.conj(y)


# ------------------------------------------------------------ index layout

def index(l: int, m: int, n: int, N: int) -> int:
    """alpha = (l^2 + l + m) N + n (0-based form of the paper's indexing map)."""
    return (l * l + l + m) * N + n


def complex_to_real(F: np.ndarray, L: int, N: int) -> np.ndarray:
    """Map complex-harmonic coefficients to real-harmonic ones (unitary):
    s_{l,m} = (f_m + f_{-m})/sqrt2, s_{l,-m} = i (f_m - f_{-m})/sqrt2 (m > 0),
    s_{l,0} = f_0.  Real basis: S_lm = sqrt2 c_lm P_l^m cos(m phi) (m>0),
    S_l0 = c_l0 P_l, S_{l,-m} = sqrt2 c_lm P_l^m sin(m phi)."""
    F = np.asarray(F)
    S = np.zeros_like(F, dtype=np.complex128)
    s2 = math.sqrt(2.0)
    for l in range(L):
        base = l * l + l
        S[base * N:(base + 1) * N] = F[base * N:(base + 1) * N]
        for m in range(1, l + 1):
            fp = F[(base + m) * N:(base + m + 1) * N]
            fm = F[(base - m) * N:(base - m + 1) * N]
            S[(base + m) * N:(base + m + 1) * N] = (fp + fm) / s2
            S[(base - m) * N:(base - m + 1) * N] = 1j * (fp - fm) / s2
    return S


def real_to_complex(S: np.ndarray, L: int, N: int) -> np.ndarray:
    """Inverse of complex_to_real: f_m = (s_m - i s_{-m})/sqrt2,
    f_{-m} = (s_m + i s_{-m})/sqrt2."""
    S = np.asarray(S)
    F = np.zeros(S.shape, dtype=np.complex128)
    s2 = math.sqrt(2.0)
    for l in range(L):
        base = l * l + l
        F[base * N:(base + 1) * N] = S[base * N:(base + 1) * N]
        for m in range(1, l + 1):
            sp = S[(base + m) * N:(base + m + 1) * N]
            sm = S[(base - m) * N:(base - m + 1) * N]
            F[(base + m) * N:(base + m + 1) * N] = (sp - 1j * sm) / s2
            F[(base - m) * N:(base - m + 1) * N] = (sp + 1j * sm) / s2
    return F


# ----------------------------------------------------------- basis object

@dataclasses.dataclass
class Basis:
    L: int
    N: int
    R: float
    n_r: int
    n_theta: int
    n_phi: int
    rule: int
    b: np.ndarray = None          # [L, N] Bessel zeros
    lam: np.ndarray = None        # [d] Laplacian eigenvalues (b/R)^2 per alpha
    r: np.ndarray = None
    wr: np.ndarray = None
    theta: np.ndarray = None
    t: np.ndarray = None
    wt: np.ndarray = None
    phi: np.ndarray = None
    Rtab: np.ndarray = None       # [L, N, n_r]  R_ln(r_k)
    Ptab: np.ndarray = None       # [L, L, n_theta]  c_lm P_l^m(t_j)

    @property
    def d(self) -> int:
        return self.L * self.L * self.N

    @property
    def n_grid(self) -> int:
        return self.n_r * self.n_theta * self.n_phi

    def weights(self) -> np.ndarray:
        """Quadrature weight per grid point, [r][theta][phi]:
        w_r * w_theta * 2 pi / N_phi."""
        return (self.wr[:, None, None] * self.wt[None, :, None]
                * np.full((1, 1, self.n_phi), 2.0 * math.pi / self.n_phi))


def make_basis(L, N, R, n_r, n_theta, n_phi, rule=RADIAL_GAUSS_JACOBI_R2) -> Basis:
    bs = Basis(L, N, float(R), n_r, n_theta, n_phi, rule)
    bs.b = bessel_zeros(L, N)
    lam = np.empty(bs.d)
    for l in range(L):
        for m in range(-l, l + 1):
            for n in range(N):
                lam[index(l, m, n, N)] = (bs.b[l, n] / R) ** 2
    bs.lam = lam
    bs.r, bs.wr = radial_nodes(n_r, R, rule)
    bs.theta, bs.t, bs.wt = theta_nodes(n_theta)
    bs.phi = phi_nodes(n_phi)
    bs.Rtab = np.stack([radial_function(l, bs.b[l], bs.r, R) for l in range(L)])
    bs.Ptab = legendre_table(L, bs.t)
    return bs


def basis_for(w) -> Basis:
    """Basis of a synth_inputs.Workload."""
    return make_basis(w.L, w.N, w.R, w.n_r, w.n_theta, w.n_phi, w.radial_rule)


def ke_cutoff_counts(bs: Basis, e_cut: float) -> np.ndarray:
    """Radial functions kept per l by a kinetic-energy cutoff (the non-uniform
    basis of the footnote in Section 2.2.1): N_l = #{n < N : Lambda_ln / 2 <=
    e_cut}.  Lambda_ln grows with n, so the kept ones are n = 0 .. N_l - 1."""
    return np.array([int(np.sum(0.5 * (bs.b[l] / bs.R) ** 2 <= e_cut)) for l in range(bs.L)])


def ke_cutoff_index(bs: Basis, e_cut: float) -> np.ndarray:
    """Positions, in the uniform layout, of the functions the cutoff keeps, in
    the order of the cutoff basis's own layout (l, then m, then n, as in the
    uniform one): a coefficient vector of the cutoff basis is the uniform one
    restricted to these entries."""
    Nl = ke_cutoff_counts(bs, e_cut)
    return np.array([index(l, m, n, bs.N) for l in range(bs.L) for m in range(-l, l + 1)
                     for n in range(Nl[l])], dtype=np.int64)


def basis_matrix_complex(bs: Basis) -> np.ndarray:
    """B[g, alpha] = F_alpha(x_g) on the grid (flattened [r][theta][phi]);
    small bases only."""
    TH, PH = np.meshgrid(bs.theta, bs.phi, indexing="ij")
    B = np.zeros((bs.n_r, bs.n_theta, bs.n_phi, bs.d), dtype=np.complex128)
    for l in range(bs.L):
        for m in range(-l, l + 1):
            Y = Y_complex(l, m, TH, PH)
            for n in range(bs.N):
                B[..., index(l, m, n, bs.N)] = bs.Rtab[l, n][:, None, None] * Y[None]
    return B.reshape(bs.n_grid, bs.d)


def real_harmonic(l: int, m: int, theta, phi):
    """Real orthonormal harmonic S_lm of the C interface's coefficient layout."""
    am = abs(m)
    y = Y_complex(l, am, theta, phi)
    if m > 0:
        return math.sqrt(2.0) * y.real
    if m < 0:
        return math.sqrt(2.0) * y.imag
    return y.real
