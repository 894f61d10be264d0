"""Pins of the oracle's LOBPCG and Teter-Payne-Allan preconditioner (Section
3.1) against results fixed independently of it: dense diagonalisation,
the harmonic oscillator's levels, the preconditioner's stated limits, and
exact eigenvectors for the locking rules."""
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import lobpcg as ol


@pytest.fixture(scope="module")
def small():
    w = si.small(6, 8, R=9.0, k=8)
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    Hd = oh.dense_H_real(bs, V)
    lam, U = np.linalg.eigh(Hd)
    return bs, Hd, lam, U


def test_tpa_factor_limits():
    """T(g) = 1 with zero first three derivatives at g = 0 (T - 1 = -(16/27)
    g^4 + O(g^5)), decreases monotonically in (0, 1] for g >= 0, and tends to
    1/(2g), the inverse of the Laplacian up to a constant, for large g."""
    assert ol.tpa_factor(0.0) == 1.0
    for g in (1e-2, 3e-3, 1e-3):
        assert abs((ol.tpa_factor(g) - 1.0) / g ** 4 + 16.0 / 27.0) < 50 * g
    g = np.linspace(0.0, 50.0, 5001)
    t = ol.tpa_factor(g)
    assert np.all(t > 0) and np.all(t <= 1.0) and np.all(np.diff(t) < 0)
    for g in (1e3, 1e5):
        assert abs(ol.tpa_factor(g) * 2.0 * g - 1.0) < 2.0 / g


def test_tpa_preconditioner_is_diagonal_and_scale_free():
    """Each column is scaled coefficient-wise by T(g_alpha) with g_alpha =
    Lambda_alpha / KE, KE the kinetic energy per unit norm: the result is
    linear in the column's scale and low-Lambda coefficients pass unchanged
    when KE is large."""
    rng = np.random.default_rng(5)
    lam = np.linspace(0.01, 40.0, 200)
    R = rng.standard_normal((200, 3))
    P1 = ol.tpa_precondition(R, lam)
    assert np.allclose(ol.tpa_precondition(7.0 * R, lam), 7.0 * P1, rtol=1e-14, atol=0)
    ke = 0.5 * np.sum(lam[:, None] * R ** 2, axis=0) / np.sum(R ** 2, axis=0)
    ref = R * ol.tpa_factor(lam[:, None] / ke[None, :])
    assert np.allclose(P1, ref, rtol=1e-14, atol=0)
    # TPA's own variable: half the Laplacian eigenvalue
    ref2 = R * ol.tpa_factor(0.5 * lam[:, None] / ke[None, :])
    assert np.allclose(ol.tpa_precondition(R, lam, g_scale=0.5), ref2, rtol=1e-14, atol=0)


@pytest.mark.parametrize("g_scale", [1.0, 0.5])
def test_lobpcg_matches_dense_eigenvalues(small, g_scale):
    """Lowest 6 eigenvalues of the dense operator (k = 8 with 2 guard states),
    for the printed preconditioner variable and TPA's own."""
    bs, Hd, lam, U = small
    th, X, res, it, _ = ol.lobpcg(lambda Y: Hd @ Y, si.random_block(bs.d, 8, 3), bs.lam,
                                  res_tol=1e-10, max_iter=400, n_check=6, g_scale=g_scale)
    assert it < 400
    assert np.max(np.abs(th[:6] - lam[:6])) < 1e-12 * np.max(np.abs(lam))
    assert np.max(np.abs(X.T @ X - np.eye(8))) < 1e-12
    # converged columns: Ritz vectors span the eigenvectors (subspace projector)
    Pg = X[:, :6] @ X[:, :6].T
    Pr = U[:, :6] @ U[:, :6].T
    assert np.max(np.abs(Pg - Pr)) < 1e-8


def test_lobpcg_preconditioner_speeds_up_convergence(small):
    """Section 3.1.2: the diagonal preconditioner markedly speeds up LOBPCG;
    here the unpreconditioned run needs more than twice the iterations."""
    bs, Hd, lam, U = small
    X0 = si.random_block(bs.d, 8, 3)
    _, _, _, it_p, _ = ol.lobpcg(lambda Y: Hd @ Y, X0, bs.lam, res_tol=1e-8, max_iter=500,
                                 n_check=6)
    _, _, res, it_n, _ = ol.lobpcg(lambda Y: Hd @ Y, X0, bs.lam, res_tol=1e-8,
                                   max_iter=500, n_check=6, precondition=False)
    assert it_p < 500 and it_n > 2 * it_p


def test_lobpcg_harmonic_oscillator_levels():
    """omega (n + 3/2) with degeneracies (n+1)(n+2)/2: the lowest ten are
    0.75, 1.25 x 3, 1.75 x 6 (omega = 0.5); one guard state."""
    w = si.C1
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    th, X, res, it, _ = ol.lobpcg(lambda Y: oh.apply_H_real(bs, V, Y),
                                  si.x0_block(w, k=11), bs.lam, res_tol=1e-9, max_iter=300,
                                  n_check=10)
    ref = np.array([0.75] + [1.25] * 3 + [1.75] * 6)
    assert it < 300
    assert np.max(np.abs(th[:10] - ref)) < 1e-8


def test_lobpcg_hard_locking_deflates_constraints(small):
    """With the three lowest exact eigenvectors as constraints, the block finds
    eigenvalues 4..9 and stays orthogonal to the constraints."""
    bs, Hd, lam, U = small
    Y = U[:, :3]
    th, X, res, it, _ = ol.lobpcg(lambda Z: Hd @ Z, si.random_block(bs.d, 8, 4), bs.lam,
                                  res_tol=1e-10, max_iter=400, n_check=6, constraints=Y)
    assert np.max(np.abs(th[:6] - lam[3:9])) < 1e-12 * np.max(np.abs(lam))
    assert np.max(np.abs(Y.T @ X)) < 1e-12


def test_lobpcg_soft_locking_of_converged_columns(small):
    """A start block holding three exact eigenvectors: those columns are
    converged at iteration 0 and leave the search (the active count starts at
    k - 3), the rest converge, and the locked eigenvalues stay exact."""
    bs, Hd, lam, U = small
    X0 = si.random_block(bs.d, 8, 5)
    X0[:, :3] = U[:, :3]
    hist = []
    th, X, res, it, _ = ol.lobpcg(lambda Z: Hd @ Z, X0, bs.lam, res_tol=1e-10, max_iter=400,
                                  n_check=6, log=lambda i, t, r, n: hist.append(n))
    assert hist[0] == 5
    assert np.max(np.abs(th[:6] - lam[:6])) < 1e-12 * np.max(np.abs(lam))
