"""Electron density, Hartree potential and exchange (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Density (eq. density_expression, Section 2.2.5): rho = 2 sum_i f_i |psi_i|^2,
computed by inverse transforms to the grid, pointwise squares, and a forward
transform for the coefficients tau: in the orbitals' own basis (the dualing
choice) or in the larger density basis with l' <= 2(L-1) that the product of
two orbitals needs (Section 2.2.5's first comment, density_basis_for).

Hartree (Section 2.3.1, eqs. Laplace_expansion, hartree_calc1, zeta_definition):
V_H(x) = sum tau_lmn (4 pi / (2l+1)) Y_lm(x) Z_ln(r), with Z_ln the radial
integral of r_<^l / r_>^{l+1} against R_ln(s) s^2, evaluated here by direct
Gauss quadrature of that definition (split at s = r).  In the real layout the
same sum runs over the real harmonics S_lm (the addition theorem is basis
independent).

Exchange: Slater (LDA exchange only), V_x = -(3 rho / pi)^{1/3}.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .basis import Basis, index, radial_function, real_harmonic
from .hamiltonian import from_grid_real, to_grid_real


def density_grid(bs: Basis, X: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """rho(x_g) = 2 sum_i f_i psi_i(x_g)^2, psi_i the inverse transform of x_i;
    returns (n_r, n_theta, n_phi)."""
    psi = to_grid_real(bs, X)
    return 2.0 * np.einsum("rtpi,i->rtp", psi * psi, np.asarray(occ, dtype=np.float64))


def density_coefficients(bs: Basis, rho: np.ndarray) -> np.ndarray:
    """tau = forward transform of rho (same basis as the orbitals)."""
    return from_grid_real(bs, rho[..., None])[:, 0]


def density_basis_for(bs: Basis, N_rho: int | None = None) -> Basis:
    """The larger basis for the density of Section 2.2.5 (the non-dualing
    choice): the product of two orbitals holds angular degrees up to 2(L-1),
    so l' <= 2(L-1), i.e. L' = 2L - 1; N_rho radial functions (default N), on
    the orbitals' grid (same R, nodes and radial rule).  The grid integrates
    the density against these functions exactly in angle when n_theta >=
    2L - 1 and n_phi >= 4L - 3, which the usual n_theta = 2L, n_phi = 4L
    satisfy."""
    from .basis import make_basis
    Lr = 2 * bs.L - 1
    assert bs.n_theta >= Lr and bs.n_phi >= 2 * Lr - 1, "grid too coarse for the density basis"
    return make_basis(Lr, bs.N if N_rho is None else N_rho, bs.R, bs.n_r, bs.n_theta,
                      bs.n_phi, bs.rule)


def integrate_grid(bs: Basis, f: np.ndarray) -> float:
    """sum_g W_g f(x_g)  ~  int over the ball."""
    return float(np.sum(bs.weights() * f))


def zeta_table(bs: Basis, n_quad: int = 160) -> np.ndarray:
    """Z[l, n, k] = int_0^R (r_<^l / r_>^{l+1}) R_ln(s) s^2 ds at r = r_k,
    by Gauss-Legendre quadrature on [0, r] and [r, R] (eq. zeta_definition)."""
    x, w = special.roots_legendre(n_quad)
    Z = np.zeros((bs.L, bs.N, bs.n_r))
    R = bs.R
    for kk, r in enumerate(bs.r):
        s1 = 0.5 * r * (x + 1.0)
        w1 = 0.5 * r * w
        s2 = r + 0.5 * (R - r) * (x + 1.0)
        w2 = 0.5 * (R - r) * w
        for l in range(bs.L):
            f1 = radial_function(l, bs.b[l], s1, R)       # [n, q]
            f2 = radial_function(l, bs.b[l], s2, R)
            inner = (f1 * (s1 ** (l + 2))[None, :]) @ w1 / r ** (l + 1)
            outer = (f2 * (s2 ** (1 - l))[None, :]) @ w2 * r ** l
            Z[l, :, kk] = inner + outer
    return Z


def hartree_grid(bs: Basis, tau: np.ndarray, zeta: np.ndarray | None = None) -> np.ndarray:
    """V_H on the grid from real-layout density coefficients tau, eq. hartree_calc1."""
    if zeta is None:
        zeta = zeta_table(bs)
    TH, PH = np.meshgrid(bs.theta, bs.phi, indexing="ij")
    V = np.zeros((bs.n_r, bs.n_theta, bs.n_phi))
    for l in range(bs.L):
        pref = 4.0 * math.pi / (2 * l + 1)
        for m in range(-l, l + 1):
            S = real_harmonic(l, m, TH, PH)
            a0 = index(l, m, 0, bs.N)
            radial = pref * (tau[a0:a0 + bs.N] @ zeta[l])   # [r]
            V += radial[:, None, None] * S[None]
    return V


def slater_exchange(rho: np.ndarray) -> np.ndarray:
    """V_x = -(3 rho / pi)^{1/3} (LDA exchange)."""
    return -np.cbrt(3.0 * np.maximum(rho, 0.0) / math.pi)


# Perdew-Zunger (1981) fit of the Ceperley-Alder correlation energy per
# electron of the unpolarised electron gas: the LDA parametrisation Section
# 2.1 adopts.  Published constants (Hartree atomic units).
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334        # r_s >= 1
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116      # r_s < 1


def pz81_correlation(rho: np.ndarray):
    """Correlation energy per electron eps_c and potential v_c = d(rho eps_c)/drho
    of the Perdew-Zunger parametrisation, r_s = (3 / (4 pi rho))^{1/3}:
        r_s >= 1:  eps_c = gamma / (1 + beta1 sqrt(r_s) + beta2 r_s)
        r_s < 1:   eps_c = A ln r_s + B + C r_s ln r_s + D r_s
    and v_c = eps_c - (r_s / 3) d eps_c / d r_s (the chain rule through
    d r_s / d rho = -r_s / (3 rho)), written out per branch.  rho <= 0 gives
    0 for both (the r_s -> infinity limit).  Returns (eps_c, v_c)."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    v = np.zeros_like(rho)
    pos = rho > 0.0
    rs = np.cbrt(3.0 / (4.0 * math.pi * rho[pos]))
    lo = rs >= 1.0
    # low density: eps = gamma / den, d eps / d r_s = -gamma (beta1 / (2 sqrt r_s) + beta2) / den^2
    sq = np.sqrt(rs[lo])
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * rs[lo]
    e_lo = PZ_GAMMA / den
    de_lo = -PZ_GAMMA * (PZ_BETA1 / (2.0 * sq) + PZ_BETA2) / den ** 2
    # high density: d eps / d r_s = A / r_s + C (ln r_s + 1) + D
    r_hi = rs[~lo]
    ln = np.log(r_hi)
    e_hi = PZ_A * ln + PZ_B + PZ_C * r_hi * ln + PZ_D * r_hi
    de_hi = PZ_A / r_hi + PZ_C * (ln + 1.0) + PZ_D
    e_pos = np.empty_like(rs)
    v_pos = np.empty_like(rs)
    e_pos[lo], e_pos[~lo] = e_lo, e_hi
    v_pos[lo] = e_lo - rs[lo] / 3.0 * de_lo
    v_pos[~lo] = e_hi - r_hi / 3.0 * de_hi
    eps[pos], v[pos] = e_pos, v_pos
    return eps, v
