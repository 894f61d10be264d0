"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: closed forms,
tabulated values, textbook spectra, invariants and brute force on tiny bases.
"""
import math

import numpy as np
import pytest
from scipy import special

import synth_inputs as si
from oracle import basis as ob
from oracle import density as od
from oracle import eigensolver as oe
from oracle import hamiltonian as oh
from conftest import golden_path


def _load(name):
    return np.loadtxt(golden_path(name), comments="#")


# ------------------------------------------------------------ basis tables

def test_bessel_zeros_tabulated_and_closed_forms():
    b = ob.bessel_zeros(6, 8)
    for l, n, val in _load("bessel_zeros_tabulated.txt"):
        assert abs(b[int(l), int(n)] - val) < 2e-9
    # j_0 = sin x / x: zeros (n+1) pi
    assert np.allclose(b[0], np.pi * np.arange(1, 9), rtol=0, atol=1e-13)
    # j_1 = 0  <=>  tan x = x
    x = b[1]
    assert np.max(np.abs(np.sin(x) - x * np.cos(x)) / x) < 1e-13
    # j_2 = 0  <=>  (3 - x^2) sin x = 3 x cos x
    x = b[2]
    assert np.max(np.abs((3 - x * x) * np.sin(x) - 3 * x * np.cos(x)) / x ** 2) < 1e-13
    # interlacing b[l,n] < b[l+1,n] < b[l,n+1]
    assert np.all(b[:-1, :] < b[1:, :])
    assert np.all(b[1:, :-1] < b[:-1, 1:])


def test_radial_functions_orthonormal_and_closed_form():
    L, N, R = 5, 6, 7.0
    b = ob.bessel_zeros(L, N)
    r, wr = ob.radial_nodes(4 * N + 8, R, ob.RADIAL_GAUSS_JACOBI_R2)
    for l in range(L):
        Rt = ob.radial_function(l, b[l], r, R)
        G = (Rt * wr) @ Rt.T
        assert np.max(np.abs(G - np.eye(N))) < 1e-12
        # sqrt(2/r) J_{l+1/2}(kr) / (R J_{l+3/2}(b)) == sqrt(2/R^3) j_l(kr) / j_{l+1}(b)
        k = b[l] / R
        alt = (math.sqrt(2.0 / R ** 3) * special.spherical_jn(l, k[:, None] * r[None, :])
               / special.spherical_jn(l + 1, b[l])[:, None])
        assert np.max(np.abs(Rt - alt)) < 1e-12 * np.max(np.abs(alt))
    # the two radial rules integrate r^2 polynomials exactly
    for rule in (ob.RADIAL_GAUSS_JACOBI_R2, ob.RADIAL_GAUSS_LEGENDRE):
        r, wr = ob.radial_nodes(12, R, rule)
        for p in range(0, 15):
            assert abs(np.sum(wr * r ** p) - R ** (p + 3) / (p + 3)) < 1e-12 * R ** (p + 3)


def test_harmonics_closed_forms_no_condon_shortley():
    th, ph = 0.7, 0.3
    Y = ob.Y_complex
    assert abs(Y(0, 0, th, ph) - 1 / math.sqrt(4 * math.pi)) < 1e-15
    assert abs(Y(1, 0, th, ph) - math.sqrt(3 / (4 * math.pi)) * math.cos(th)) < 1e-15
    # no CS phase: Y_1^1 = +sqrt(3/8pi) sin(theta) e^{i phi}
    assert abs(Y(1, 1, th, ph) - math.sqrt(3 / (8 * math.pi)) * math.sin(th)
               * np.exp(1j * ph)) < 1e-15
    assert abs(Y(2, 1, th, ph) - math.sqrt(15 / (8 * math.pi)) * math.sin(th)
               * math.cos(th) * np.exp(1j * ph)) < 1e-15
    assert abs(Y(2, 2, th, ph) - math.sqrt(15 / (32 * math.pi)) * math.sin(th) ** 2
               * np.exp(2j * ph)) < 1e-15
    assert abs(Y(2, -2, th, ph) - np.conj(Y(2, 2, th, ph))) < 1e-15
    # real harmonics of the C layout: l = 1 gives sqrt(3/4pi) (x, y, z)/r
    c = math.sqrt(3 / (4 * math.pi))
    assert abs(ob.real_harmonic(1, 1, th, ph) - c * math.sin(th) * math.cos(ph)) < 1e-15
    assert abs(ob.real_harmonic(1, -1, th, ph) - c * math.sin(th) * math.sin(ph)) < 1e-15
    assert abs(ob.real_harmonic(1, 0, th, ph) - c * math.cos(th)) < 1e-15


def test_legendre_table_against_lpmv():
    L = 18
    _, t, _ = ob.theta_nodes(23)
    P = ob.legendre_table(L, t)
    for l in range(L):
        for m in range(l + 1):
            # lpmv carries the (-1)^m phase; the paper's P_l^m does not
            ref = ob.c_lm(l, m) * (-1.0) ** m * special.lpmv(m, l, t)
            assert np.max(np.abs(P[l, m] - ref)) < 1e-11, (l, m)


def test_harmonics_orthonormal_on_grid():
    L = 7
    theta, t, wt = ob.theta_nodes(L + 1)
    phi = ob.phi_nodes(2 * L)
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    W = wt[:, None] * (2 * math.pi / len(phi))
    Ys = [ob.Y_complex(l, m, TH, PH) for l in range(L) for m in range(-l, l + 1)]
    G = np.array([[np.sum(W * a * np.conj(b)) for b in Ys] for a in Ys])
    assert np.max(np.abs(G - np.eye(len(Ys)))) < 1e-13
    Ss = [ob.real_harmonic(l, m, TH, PH) for l in range(L) for m in range(-l, l + 1)]
    G = np.array([[np.sum(W * a * b) for b in Ss] for a in Ss])
    assert np.max(np.abs(G - np.eye(len(Ss)))) < 1e-13


def test_complex_real_map_unitary_and_real_functions():
    L, N = 4, 3
    d = L * L * N
    rng = np.random.default_rng(0)
    F = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    S = ob.complex_to_real(F, L, N)
    assert abs(np.linalg.norm(S) - np.linalg.norm(F)) < 1e-13
    assert np.max(np.abs(ob.real_to_complex(S, L, N) - F)) < 1e-14
    # a real function has f_{l,-m,n} = conj(f_{l,m,n}) and real s coefficients
    bs = ob.make_basis(L, N, 5.0, 4 * N, L + 1, 2 * L, ob.RADIAL_GAUSS_JACOBI_R2)
    TH, PH = np.meshgrid(bs.theta, bs.phi, indexing="ij")
    f = (np.exp(-bs.r[:, None, None] ** 2) * np.cos(TH)[None] ** 2
         * (1 + np.sin(TH) * np.cos(PH - 0.4))[None])
    Fc = oh.forward_transform(bs, f[..., None].astype(complex))[:, 0]
    for l in range(L):
        for m in range(1, l + 1):
            for n in range(N):
                assert abs(Fc[ob.index(l, -m, n, N)] - np.conj(Fc[ob.index(l, m, n, N)])) < 1e-13
    assert np.max(np.abs(ob.complex_to_real(Fc, L, N).imag)) < 1e-13


# ---------------------------------------------------------------- operator

def test_round_trip_identity_exact_quadrature():
    # B^H W B = I once N_theta >= L, N_phi >= 2L-1 (angular quadrature exact)
    # and N_r well above N (radial products of Bessel functions are not
    # polynomials; at N_r = 6N the radial rule is exact to rounding).
    L, N = 4, 5
    bs = ob.make_basis(L, N, 6.0, 6 * N, L, 2 * L - 1, ob.RADIAL_GAUSS_JACOBI_R2)
    B = ob.basis_matrix_complex(bs)
    G = B.conj().T @ (bs.weights().reshape(-1)[:, None] * B)
    assert np.max(np.abs(G - np.eye(bs.d))) < 1e-12
    X = si.random_block(bs.d, 3, 1)
    Fc = ob.real_to_complex(X, L, N)
    back = oh.forward_transform(bs, oh.inverse_transform(bs, Fc))
    assert np.max(np.abs(back - Fc)) < 1e-12


def test_dense_equals_separable_and_symmetric():
    w = si.small(5, 6, R=8.0, k=3)
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    H = oh.dense_H_real(bs, V)
    assert np.max(np.abs(H - H.T)) < 1e-13 * np.max(np.abs(H))
    X = si.random_block(bs.d, 3, 2)
    Z = oh.apply_H_real(bs, V, X)
    assert np.max(np.abs(Z - H @ X)) < 1e-12 * np.max(np.abs(Z))
    # the real-layout operator equals the one built from real harmonics directly
    TH, PH = np.meshgrid(bs.theta, bs.phi, indexing="ij")
    Br = np.zeros((bs.n_r, bs.n_theta, bs.n_phi, bs.d))
    for l in range(bs.L):
        for m in range(-l, l + 1):
            S = ob.real_harmonic(l, m, TH, PH)
            for n in range(bs.N):
                Br[..., ob.index(l, m, n, bs.N)] = bs.Rtab[l, n][:, None, None] * S[None]
    Br = Br.reshape(bs.n_grid, bs.d)
    Hr = Br.T @ ((bs.weights() * V).reshape(-1)[:, None] * Br) + np.diag(0.5 * bs.lam)
    assert np.max(np.abs(Hr - H)) < 1e-12 * np.max(np.abs(H))


def test_particle_in_sphere_and_constant_shift():
    L, N, R = 4, 4, 10.0
    bs = ob.make_basis(L, N, R, 6 * N, L, 2 * L - 1, ob.RADIAL_GAUSS_JACOBI_R2)
    ev = np.linalg.eigvalsh(oh.dense_H_real(bs, np.zeros((bs.n_r, bs.n_theta, bs.n_phi))))
    table = _load("particle_in_sphere_R10.txt")
    levels = sorted((val, 2 * int(l) + 1) for l, n, val in table)
    pos = 0
    for val, deg in levels:
        assert np.all(np.abs(ev[pos:pos + deg] - val) < 1e-9)
        pos += deg
    # a constant potential c shifts every level by c when the quadrature is exact
    c = -0.37
    ev2 = np.linalg.eigvalsh(oh.dense_H_real(bs, np.full((bs.n_r, bs.n_theta, bs.n_phi), c)))
    assert np.max(np.abs(ev2 - (ev + c))) < 1e-12


@pytest.mark.parametrize("rule", [si.RADIAL_GAUSS_LEGENDRE, si.RADIAL_GAUSS_JACOBI_R2])
def test_harmonic_oscillator_levels(rule):
    w = si.C1
    bs = ob.make_basis(w.L, w.N, w.R, w.n_r, w.n_theta, w.n_phi, rule)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    ev = np.linalg.eigvalsh(oh.dense_H_real(bs, V))
    pos = 0
    for n, e, deg in _load("harmonic_oscillator_w0.5.txt"):
        assert np.all(np.abs(ev[pos:pos + int(deg)] - e) < 1e-8)
        pos += int(deg)


def test_hydrogen_l0_polynomial_convergence():
    # Section 4.1: l = 0 only, V = -1/r, ground state -> -0.5 Ha (slowly).
    errs = []
    for N in (10, 20, 40, 80):
        bs = ob.make_basis(1, N, 20.0, 2 * N, 1, 1, ob.RADIAL_GAUSS_JACOBI_R2)
        V = np.broadcast_to(-1.0 / bs.r[:, None, None], (bs.n_r, 1, 1)).copy()
        ev = np.linalg.eigvalsh(oh.dense_H_real(bs, V))
        errs.append(abs(ev[0] + 0.5))
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 1e-3
    # polynomial, not spectral: doubling N gains a bounded factor
    assert all(2.0 < errs[i] / errs[i + 1] < 16.0 for i in range(3))


# -------------------------------------------------------------- eigensolver

def _tiny_operator():
    w = si.small(4, 5, R=8.0, k=6)
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    return w, bs, V, oh.dense_H_real(bs, V)


def test_chebyshev_filter_equals_polynomial_of_H():
    w, bs, V, H = _tiny_operator()
    lam, U = np.linalg.eigh(H)
    X = si.random_block(bs.d, 4, 3)
    a, b, a0 = lam[10], lam[-1] * 1.01, lam[0]
    for deg in (1, 2, 7):
        Y = oe.chebyshev_filter(lambda Z: H @ Z, X, deg, a, b, a0)
        p = oe.chebyshev_filter_scalar(lam, deg, a, b, a0)
        ref = U @ (p[:, None] * (U.T @ X))
        assert np.max(np.abs(Y - ref)) < 1e-11 * np.max(np.abs(ref))


def test_cholesky_qr_and_rayleigh_ritz():
    w, bs, V, H = _tiny_operator()
    lam, U = np.linalg.eigh(H)
    X = si.random_block(bs.d, 5, 4) * np.array([1e-3, 1, 10, 1e2, 1])
    Q = oe.cholesky_qr(X)
    assert np.max(np.abs(Q.T @ Q - np.eye(5))) < 1e-12
    # Q spans the same space as X
    assert np.max(np.abs(Q @ (Q.T @ X) - X)) < 1e-10 * np.max(np.abs(X))
    # an invariant subspace reproduces exact eigenvalues
    Z = U[:, 3:8] @ si.random_block(5, 5, 7)
    theta, Xo, HXo, res = oe.rayleigh_ritz(lambda Y: H @ Y, Z)
    assert np.max(np.abs(theta - lam[3:8])) < 1e-12
    assert np.max(res) < 1e-11


def test_chefsi_converges_to_dense_eigenvalues():
    w, bs, V, H = _tiny_operator()
    lam = np.linalg.eigvalsh(H)
    app = lambda Y: H @ Y
    b = oe.lanczos_upper_bound(app, si.lanczos_start(bs.d))
    assert b >= lam[-1]
    X0 = si.x0_block(w, k=8, d=bs.d)
    theta, X, res, it = oe.chefsi(app, X0, 10, b, n_check=6, max_iter=200)
    assert np.max(np.abs(theta[:6] - lam[:6])) < 1e-7      # default stop rule
    theta, X, res, it = oe.chefsi(app, X0, 10, b, n_check=6, max_iter=400,
                                  res_tol=1e-10, dtheta_tol=1e-13)
    assert np.max(np.abs(theta[:6] - lam[:6])) < 1e-12


# ------------------------------------------------------- KB nonlocal term

def test_kb_rank_one_secular_equation():
    # V = 0 plus one projector: eigenvalues solve 1 + h sum_a p_a^2/(e_a - lam) = 0
    L, N = 3, 4
    bs = ob.make_basis(L, N, 8.0, 4 * N, L, 2 * L, ob.RADIAL_GAUSS_JACOBI_R2)
    zero = np.zeros((bs.n_r, bs.n_theta, bs.n_phi))
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    pg, _ = si.kb_projector_values(pts, np.array([[0.5, -0.3, 0.8]]))
    P = oh.kb_projectors(bs, pg.reshape(bs.n_r, bs.n_theta, bs.n_phi, -1))[:, :1]
    h = np.array([1.5])
    Hm = np.column_stack([oh.apply_H_real(bs, zero, e, proj=P, h=h) for e in np.eye(bs.d)])
    assert np.max(np.abs(Hm - Hm.T)) < 1e-13
    ev = np.linalg.eigvalsh(Hm)
    eps = 0.5 * bs.lam
    p2 = P[:, 0] ** 2
    for lam_ in ev:
        if np.min(np.abs(eps - lam_)) < 1e-8:
            continue           # eigenvalue shared with an unperturbed level
        assert abs(1.0 + h[0] * np.sum(p2 / (eps - lam_))) < 1e-8


# ------------------------------------------------------- density, Hartree

def test_density_integrates_to_electron_count():
    L, N = 4, 5
    bs = ob.make_basis(L, N, 6.0, 6 * N, L + 1, 4 * L, ob.RADIAL_GAUSS_JACOBI_R2)
    X = oe.cholesky_qr(si.random_block(bs.d, 4, 9))
    occ = np.array([1.0, 1.0, 0.5, 0.25])
    rho = od.density_grid(bs, X, occ)
    assert abs(od.integrate_grid(bs, rho) - 2 * occ.sum()) < 1e-12
    # for any block, int rho = 2 sum_i f_i ||x_i||^2 (Parseval with exact quadrature)
    Y = si.random_block(bs.d, 4, 10)
    rho = od.density_grid(bs, Y, occ)
    ref = 2 * np.sum(occ * np.sum(Y * Y, axis=0))
    assert abs(od.integrate_grid(bs, rho) - ref) < 1e-11 * ref


def test_zeta_quadrature_matches_closed_form():
    # Z_ln(r) = C [(2l+1) j_l(kr)/k^2 + j_{l+1}(kR) r^l / (k R^{l-1})],
    # C = sqrt(2/R^3) / j_{l+1}(kR): the regular solution of the radial Poisson
    # equation with source (2l+1) R_ln whose exterior continuation decays.
    bs = ob.make_basis(6, 4, 9.0, 10, 1, 1, ob.RADIAL_GAUSS_JACOBI_R2)
    Z = od.zeta_table(bs)
    R = bs.R
    for l in range(6):
        for n in range(4):
            k = bs.b[l, n] / R
            C = math.sqrt(2 / R ** 3) / special.spherical_jn(l + 1, k * R)
            ref = C * ((2 * l + 1) * special.spherical_jn(l, k * bs.r) / k ** 2
                       + special.spherical_jn(l + 1, k * R) * bs.r ** l / (k * R ** (l - 1)))
            assert np.max(np.abs(Z[l, n] - ref)) < 1e-11 * np.max(np.abs(ref))


def test_hartree_of_gaussian_charge_is_erf():
    sigma, Q = 1.0, 2.0
    bs = ob.make_basis(1, 40, 10.0, 60, 2, 2, ob.RADIAL_GAUSS_JACOBI_R2)
    rho = Q * (2 * math.pi * sigma ** 2) ** -1.5 * np.exp(-bs.r ** 2 / (2 * sigma ** 2))
    rho = np.broadcast_to(rho[:, None, None], (bs.n_r, 2, 2)).copy()
    tau = od.density_coefficients(bs, rho)
    VH = od.hartree_grid(bs, tau)
    ref = Q * special.erf(bs.r / (math.sqrt(2) * sigma)) / bs.r
    assert np.max(np.abs(VH[:, 0, 0] - ref)) < 1e-8
