"""Chebyshev-filtered subspace iteration (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.2 of the paper uses the polynomial-filtered subspace iteration of
Zhou, Saad, Tiago and Chelikowsky, with Cholesky factorisation in place of DGKS
for the orthonormalisation and a Rayleigh-Ritz step after each filter;
Section 3.1.1 asks for column scaling before the Cholesky factorisation.  The
paper gives no filter formulas, so the steps below are the published scaled
three-term Chebyshev recurrence of that method, written here from its
definition: p_m(t) = T_m((t - c)/e) / T_m((a0 - c)/e) with e = (b - a)/2,
c = (b + a)/2, which damps [a, b] and keeps values below a near the scale of
p_m(a0) = 1.  The run starts from random vectors with no first
diagonalisation (the paper's footnote on Zhou 2014).
`apply` is any callable Y -> H Y on d x k blocks.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def chebyshev_filter(apply, X: np.ndarray, degree: int, a: float, b: float,
                     a0: float) -> np.ndarray:
    """Y_m = p_m(H) X by the scaled recurrence
        sigma_1 = e / (a0 - c),  Y_1 = (sigma_1 / e) (H X - c X),
        sigma_j = 1 / (2 / sigma_1 - sigma_{j-1}),
        Y_j = (2 sigma_j / e) (H Y_{j-1} - c Y_{j-1}) - sigma_{j-1} sigma_j Y_{j-2}."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma1 = e / (a0 - c)
    y_prev = X
    y = (sigma1 / e) * (apply(X) - c * X)
    sigma = sigma1
    for _ in range(2, degree + 1):
        sigma_new = 1.0 / (2.0 / sigma1 - sigma)
        y_new = (2.0 * sigma_new / e) * (apply(y) - c * y) - (sigma * sigma_new) * y_prev
        y_prev, y, sigma = y, y_new, sigma_new
    return y


def chebyshev_filter_scalar(t, degree: int, a: float, b: float, a0: float):
    """The filter polynomial p_m(t) itself, T_m((t-c)/e) / T_m((a0-c)/e),
    evaluated with NumPy's Chebyshev series (used to pin the recurrence)."""
    from numpy.polynomial import chebyshev as C
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    coef = np.zeros(degree + 1)
    coef[-1] = 1.0
    return C.chebval((np.asarray(t) - c) / e, coef) / C.chebval((a0 - c) / e, coef)


def cholesky_qr(X: np.ndarray):
    """Orthonormalise the columns of X: S = X^T X, D = diag(S)^{-1/2},
    R^T R = D S D (Cholesky), Q = X D R^{-1}.  Returns Q."""
    S = X.T @ X
    dg = np.sqrt(np.diag(S))
    D = 1.0 / dg
    Ss = D[:, None] * S * D[None, :]
    Rf = np.linalg.cholesky(Ss).T                    # upper, Ss = R^T R
    Y = X * D[None, :]
    return sla.solve_triangular(Rf, Y.T, trans="T", lower=False).T


def rayleigh_ritz(apply, X: np.ndarray):
    """Cholesky-QR, then the projected eigenproblem:
    Q = cholqr(X); theta, S = eigh(Q^T H Q) (ascending); X_out = Q S;
    r_i = || H x_i - theta_i x_i ||_2.  Returns (theta, X_out, HX_out, r)."""
    Q = cholesky_qr(X)
    HQ = apply(Q)
    Hs = Q.T @ HQ
    Hs = 0.5 * (Hs + Hs.T)
    theta, S = np.linalg.eigh(Hs)
    Xo = Q @ S
    HXo = HQ @ S
    res = np.linalg.norm(HXo - Xo * theta[None, :], axis=0)
    return theta, Xo, HXo, res


def lanczos_upper_bound(apply, v0: np.ndarray, steps: int = 20,
                        safety: float = 1.01) -> float:
    """Upper bound of the spectrum: `steps` Lanczos steps from v0 give the
    tridiagonal T; bound = (largest Ritz value of T + ||f||) * safety, f the
    final residual vector."""
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    f = None
    for j in range(steps):
        w = apply(v[:, None])[:, 0]
        alpha = float(v @ w)
        f = w - alpha * v - beta * v_prev
        alphas.append(alpha)
        beta = float(np.linalg.norm(f))
        if j < steps - 1:
            betas.append(beta)
            v_prev, v = v, f / beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    tmax = float(np.linalg.eigvalsh(T)[-1])
    ub = tmax + beta
    return ub * safety if ub > 0 else ub / safety


def chefsi(apply, X0: np.ndarray, degree: int, b: float, n_check: int,
           max_iter: int = 60, fixed_iter: int = 0, res_tol: float = 1e-4,
           dtheta_tol: float = 1e-7, final_apply=None, log=None):
    """Chebyshev-filtered subspace iteration from a random block.

    1. Initial Rayleigh-Ritz on X0 gives theta; a0 = theta_1, a = theta_k.
    2. Repeat: filter with (a, b, a0); Rayleigh-Ritz; update a, a0.
    3. Stop after `fixed_iter` iterations if given, else when for i <= n_check
       r_i <= res_tol * max(1, |theta_i|) and |delta theta_i| < dtheta_tol.
    4. A final Rayleigh-Ritz with `final_apply` (FP64 operator) if given.
    Returns (theta, X, residuals, iterations)."""
    theta, X, _, res = rayleigh_ritz(apply, X0)
    it = 0
    while True:
        it += 1
        a0, a = theta[0], theta[-1]
        Y = chebyshev_filter(apply, X, degree, a, b, a0)
        theta_old = theta
        theta, X, _, res = rayleigh_ritz(apply, Y)
        if log is not None:
            log(it, theta, res)
        if fixed_iter:
            if it >= fixed_iter:
                break
            continue
        nc = n_check
        ok_res = np.all(res[:nc] <= res_tol * np.maximum(1.0, np.abs(theta[:nc])))
        ok_th = np.max(np.abs(theta[:nc] - theta_old[:nc])) < dtheta_tol
        if (ok_res and ok_th) or it >= max_iter:
            break
    if final_apply is not None:
        theta, X, _, res = rayleigh_ritz(final_apply, X)
    return theta, X, res, it
