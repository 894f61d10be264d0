"""Self-consistent field loop of the cluster model (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The model follows the paper's SCF (Sections 2.1, 3.2, 3.4.1): an effective
potential V_eff = V_ext + V_H[rho - rho_ion] + V_x[rho] (Hartree by the Laplace
expansion of Section 2.3.1, LDA exchange only), Chebyshev-filtered subspace
iteration for the orbitals (one filter + Rayleigh-Ritz per SCF step after a
first step that filters the random start), density from the occupied
orbitals (Section 2.2.5, dualing basis), Anderson mixing of the potential
(Section 3.4.1, full history up to `hist`), a superposition-of-atomic-
densities start (Section 3.2).  Each atom carries valence charge 2 with a
neutralising Gaussian ion charge, so the cluster is neutral.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis as ob
from . import density as od
from . import eigensolver as oe
from . import hamiltonian as oh


def fermi_dirac_occupations(eigs, n_electrons, kT):
    """Fermi-Dirac smearing (Section 3.4.1, eq. Fermi_constraint):
    f_i = 1 / (1 + exp((lambda_i - eF) / kT)), with eF fixed by
    sum_i f_i = N_e / 2 over all the given states (each orbital doubly
    occupied).  The sum runs over every computed state: with only N_e / 2
    terms the constraint would force every f_i = 1.  eF is the root of the
    monotone constraint, found by Brent's method (scipy.optimize.brentq)
    on a bracket where the sum goes from below to above N_e / 2.
    Returns (f, eF)."""
    from scipy import optimize, special
    lam = np.asarray(eigs, dtype=np.float64)
    half = 0.5 * n_electrons
    assert kT > 0 and 0 < half < lam.size

    def excess(mu):
        return special.expit((mu - lam) / kT).sum() - half

    lo = lam.min() - 50.0 * kT - 1.0
    hi = lam.max() + 50.0 * kT + 1.0
    eF = optimize.brentq(excess, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
    return special.expit((eF - lam) / kT), eF


def anderson_step(V_hist, F_hist, beta):
    """Anderson mixing of potentials: with F = V_out - V_in and differences
    dV_i = V_{i+1} - V_i, dF_i = F_{i+1} - F_i over the stored history,
    gamma = argmin || F_k - sum_i gamma_i dF_i ||  (plain l2 over the grid),
    V_bar = V_k - sum gamma_i dV_i, F_bar = F_k - sum gamma_i dF_i,
    V_next = V_bar + beta F_bar.  With one entry: V_k + beta F_k."""
    Vk, Fk = V_hist[-1], F_hist[-1]
    m = len(V_hist) - 1
    if m == 0:
        return Vk + beta * Fk
    dV = np.stack([V_hist[i + 1] - V_hist[i] for i in range(m)], axis=1)
    dF = np.stack([F_hist[i + 1] - F_hist[i] for i in range(m)], axis=1)
    gamma, *_ = np.linalg.lstsq(dF, Fk, rcond=None)
    Vbar = Vk - dV @ gamma
    Fbar = Fk - dF @ gamma
    return Vbar + beta * Fbar


class ClusterSCF:
    """Oracle SCF for one cluster: atoms (n x 3), the workload's basis."""

    def __init__(self, bs: ob.Basis, atoms: np.ndarray, V_ext: np.ndarray,
                 rho_ion: np.ndarray, n_occ: int, n_guard: int, degree: int = 12,
                 beta: float = 0.2, hist: int = 20, zeta: np.ndarray | None = None,
                 correlation: bool = False, kT: float = 0.0, mix_density: bool = False,
                 density_basis: ob.Basis | None = None):
        """correlation: add the Perdew-Zunger LDA correlation potential to
        V_eff (Section 2.1); kT > 0: Fermi-Dirac occupations of all k states
        at that temperature for 2 n_occ electrons, recomputed from each
        step's Ritz values (Section 3.4.1), instead of n_occ filled states.
        mix_density: Anderson mixing of the electron density instead of the
        potential (Section 3.4.1 allows either): the history holds
        (rho_in, rho_out - rho_in) and each step's V_in is V_eff[rho_in].
        density_basis: expand rho - rho_ion for the Hartree potential in this
        larger basis on the same grid (the non-dualing choice of Section
        2.2.5) instead of the orbitals' basis."""
        self.rho_bs = bs if density_basis is None else density_basis
        self.mix_density = mix_density
        self.correlation = correlation
        self.kT = kT
        self.bs = bs
        self.atoms = atoms
        self.V_ext = V_ext
        self.rho_ion = rho_ion
        self.n_occ = n_occ
        self.k = n_occ + n_guard
        self.degree = degree
        self.beta = beta
        self.hist = hist
        self.zeta = od.zeta_table(self.rho_bs) if zeta is None else zeta
        self.occ = np.zeros(self.k)
        self.occ[:n_occ] = 1.0

    def potential(self, rho):
        """V_eff[rho] = V_ext + V_H[rho - rho_ion] + V_x[rho] (+ V_c[rho])."""
        tau = od.density_coefficients(self.rho_bs, rho - self.rho_ion)
        V = self.V_ext + od.hartree_grid(self.rho_bs, tau, self.zeta) + od.slater_exchange(rho)
        if self.correlation:
            V = V + od.pz81_correlation(rho)[1]
        return V

    def run(self, rho0, X0, v0=None, tol=1e-6, max_steps=60, first_iters=12, log=None):
        """Returns (eigenvalues, steps, rho, X); v0 starts the Lanczos bound
        (all ones if None)."""
        bs = self.bs
        v0 = np.ones(bs.d) if v0 is None else v0
        rho_in = rho0
        V_in = self.potential(rho0)
        X = X0.copy()
        V_hist, F_hist = [], []
        theta_old = None
        for step in range(1, max_steps + 1):
            app = lambda Y, V=V_in: oh.apply_H_real(bs, V, Y)  # noqa: E731
            b = oe.lanczos_upper_bound(app, v0)
            if step == 1:
                theta, X, _, _ = oe.rayleigh_ritz(app, X)
                for _ in range(first_iters):
                    Y = oe.chebyshev_filter(app, X, self.degree, theta[-1], b, theta[0])
                    theta, X, _, _ = oe.rayleigh_ritz(app, Y)
            else:
                Y = oe.chebyshev_filter(app, X, self.degree, theta[-1], b, theta[0])
                theta, X, _, _ = oe.rayleigh_ritz(app, Y)
            if self.kT > 0.0:
                self.occ = fermi_dirac_occupations(theta, 2 * self.n_occ, self.kT)[0]
            rho = od.density_grid(bs, X, self.occ)
            if log is not None:
                log(step, theta)
            if theta_old is not None and \
                    np.max(np.abs(theta[:self.n_occ] - theta_old[:self.n_occ])) < tol:
                return theta, step, rho, X
            theta_old = theta
            if self.mix_density:
                V_hist.append(rho_in.reshape(-1))
                F_hist.append((rho - rho_in).reshape(-1))
                V_hist, F_hist = V_hist[-self.hist:], F_hist[-self.hist:]
                rho_in = anderson_step(V_hist, F_hist, self.beta).reshape(rho.shape)
                V_in = self.potential(rho_in)
            else:
                V_out = self.potential(rho)
                V_hist.append(V_in.reshape(-1))
                F_hist.append((V_out - V_in).reshape(-1))
                V_hist, F_hist = V_hist[-self.hist:], F_hist[-self.hist:]
                V_in = anderson_step(V_hist, F_hist, self.beta).reshape(V_in.shape)
        return theta, max_steps, rho, X


def atomic_density_profile(bs: ob.Basis, rho_atom_grid: np.ndarray) -> np.ndarray:
    """l = 0 coefficients of an atom-centred density: tau_00n (n < N), from the
    forward transform (dualing basis)."""
    tau = od.density_coefficients(bs, rho_atom_grid)
    return tau[:bs.N].copy()


def radial_density(bs: ob.Basis, tau00: np.ndarray, r: np.ndarray) -> np.ndarray:
    """rho_atom(r) = Y_00 sum_n tau_00n R_0n(r) for r < R, 0 beyond."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    inside = (r < bs.R) & (r > 0)
    Rf = ob.radial_function(0, bs.b[0], r[inside], bs.R)   # [n, pts]
    out[inside] = (tau00 @ Rf) / math.sqrt(4 * math.pi)
    # r = 0: limit of R_0n, sqrt(2/R^3) * 1 / j_1(b)
    zero = r == 0
    if np.any(zero):
        from scipy import special
        lim = math.sqrt(2.0 / bs.R ** 3) / special.spherical_jn(1, bs.b[0])
        out[zero] = (tau00 @ lim) / math.sqrt(4 * math.pi)
    return out


def sad_density(bs: ob.Basis, tau00: np.ndarray, atoms: np.ndarray) -> np.ndarray:
    """Superposition of atomic densities on the grid (Section 3.2)."""
    pts = np.stack(np.broadcast_arrays(*_cart(bs)), axis=-1)
    rho = np.zeros(pts.shape[:-1])
    for a in atoms:
        rho += radial_density(bs, tau00, np.linalg.norm(pts - a, axis=-1))
    return rho


def _cart(bs):
    r = bs.r[:, None, None]
    st = np.sin(bs.theta)[None, :, None]
    ct = np.cos(bs.theta)[None, :, None]
    cp = np.cos(bs.phi)[None, None, :]
    sp = np.sin(bs.phi)[None, None, :]
    return r * st * cp, r * st * sp, r * ct * np.ones_like(cp)
