"""Block LOBPCG with the Teter-Payne-Allan preconditioner (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 3.1 of the paper uses the locally optimal block preconditioned
conjugate gradient method in the form of Knyazev, Argentati, Lashuk and
Ovtchinnikov (BLOPEX, 2007), with
  * soft locking: columns whose residual has converged take no part in the
    search directions of later iterations (their Ritz vectors still move with
    the Rayleigh-Ritz step),
  * hard locking: deflation against fixed orthonormal constraint vectors Y
    (every search block is kept orthogonal to them),
  * Cholesky orthonormalisation of the residual and conjugate-direction
    blocks with column scaling first (Section 3.1's remark on poorly scaled
    Gram matrices),
  * on a failed factorisation or Rayleigh-Ritz step, a restart that discards
    the conjugate directions (and, if needed, the residual block) and goes
    on from the current Ritz vectors,
and (Section 3.1.2) the diagonal preconditioner
    T(g) = (27 + 18 g + 12 g^2 + 8 g^3) / (27 + 18 g + 12 g^2 + 8 g^3 + 16 g^4)
applied to each residual vector y with, per coefficient alpha,
    g_alpha = g_scale * Lambda_alpha / KE(y),  KE(y) = (1/2) sum Lambda |y|^2 / sum |y|^2,
the ratio of the Laplacian eigenvalue to the kinetic energy of the residual.
The printed formula corresponds to g_scale = 1 (KE read per unit norm of
y); Teter, Payne and Allan's own variable uses half the Laplacian
eigenvalue, g_scale = 1/2.  Both are supported.

The algorithm steps follow the published method; no code from BLOPEX is used.
`apply` is any callable Y -> H Y on d x k blocks.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def tpa_factor(g):
    """T(g) of Section 3.1.2 (elementwise)."""
    g = np.asarray(g, dtype=np.float64)
    num = 27.0 + g * (18.0 + g * (12.0 + 8.0 * g))
    return num / (num + 16.0 * g ** 4)


def tpa_precondition(R: np.ndarray, lam: np.ndarray, g_scale: float = 1.0) -> np.ndarray:
    """Apply the diagonal preconditioner to each column of R (d x n)."""
    nrm2 = np.sum(R * R, axis=0)
    ke = 0.5 * np.sum(lam[:, None] * R * R, axis=0) / nrm2
    g = g_scale * lam[:, None] / ke[None, :]
    return tpa_factor(g) * R


def _scaled_cholesky_orth(V: np.ndarray):
    """Orthonormalise the columns of V by Cholesky of the column-scaled Gram
    matrix: S = V^T V, D = diag(S)^{-1/2}, R^T R = D S D, Q = V D R^{-1}.
    Returns the right factor M = D R^{-1} (so Q = V M), or None if the
    factorisation fails or meets a pivot at rounding level (2 n eps)."""
    S = V.T @ V
    dg = np.diag(S)
    if np.any(dg <= 0.0):
        return None
    D = 1.0 / np.sqrt(dg)
    Ss = D[:, None] * S * D[None, :]
    try:
        Rf = np.linalg.cholesky(Ss).T
    except np.linalg.LinAlgError:
        return None
    n = V.shape[1]
    if np.min(np.diag(Rf)) ** 2 <= 2.0 * n * np.finfo(np.float64).eps:
        return None
    Rinv = sla.solve_triangular(Rf, np.eye(n), lower=False)
    return D[:, None] * Rinv


def _project_out(V: np.ndarray, Y):
    """V <- V - Y (Y^T V) for orthonormal constraint columns Y (hard locking)."""
    if Y is None or Y.shape[1] == 0:
        return V
    return V - Y @ (Y.T @ V)


def lobpcg(apply, X0: np.ndarray, lam: np.ndarray, res_tol: float = 1e-6,
           max_iter: int = 200, n_check: int | None = None, g_scale: float = 1.0,
           precondition: bool = True, constraints: np.ndarray | None = None, log=None):
    """Lowest eigenpairs of H by block LOBPCG from the block X0 (d x k).

    Convergence of column i: r_i = ||H x_i - theta_i x_i|| <= res_tol *
    max(1, |theta_i|); a converged column leaves the search (soft locking);
    the run stops when the first n_check columns (default all) have
    converged.  constraints: d x c orthonormal columns the eigenvectors must
    be orthogonal to (hard locking).  Returns (theta, X, residuals, iters,
    restarts)."""
    d, k = X0.shape
    n_check = k if n_check is None else n_check
    Y = constraints
    # initial block: deflate, orthonormalise, Rayleigh-Ritz
    X = _project_out(X0, Y)
    M = _scaled_cholesky_orth(X)
    if M is None:
        raise np.linalg.LinAlgError("start block is numerically rank deficient")
    X = X @ M
    AX = apply(X)
    Hs = X.T @ AX
    theta, C = np.linalg.eigh(0.5 * (Hs + Hs.T))
    X, AX = X @ C, AX @ C
    P = AP = None
    restarts = 0
    it = 0
    while True:
        R = AX - X * theta[None, :]
        res = np.linalg.norm(R, axis=0)
        conv = res <= res_tol * np.maximum(1.0, np.abs(theta))
        if log is not None:
            log(it, theta, res, int(np.count_nonzero(~conv)))
        if np.all(conv[:n_check]) or it >= max_iter:
            break
        it += 1
        act = np.flatnonzero(~conv)
        W = R[:, act]
        if precondition:
            W = tpa_precondition(W, lam, g_scale)
        W = _project_out(W, Y)
        C = None
        Mw = _scaled_cholesky_orth(W)
        if Mw is not None:
            Wq = W @ Mw
            AW = apply(Wq)
            # Rayleigh-Ritz on span[X, W, P]; on a failed factorisation of the
            # conjugate directions or of the projected pencil, restart without P
            for use_p in ((True, False) if P is not None else (False,)):
                blocks, ablocks = [X, Wq], [AX, AW]
                if use_p:
                    Mp = _scaled_cholesky_orth(P[:, act])
                    if Mp is None:
                        restarts += 1
                        continue
                    blocks.append(P[:, act] @ Mp)
                    ablocks.append(AP[:, act] @ Mp)
                S = np.hstack(blocks)
                AS = np.hstack(ablocks)
                gA = S.T @ AS
                gB = S.T @ S
                try:
                    theta_all, C = sla.eigh(0.5 * (gA + gA.T), 0.5 * (gB + gB.T))
                    break
                except np.linalg.LinAlgError:
                    restarts += 1
                    C = None
        if C is None:
            # restart from the current Ritz vectors: drop W and P entirely
            restarts += 1
            P = AP = None
            X = X @ _scaled_cholesky_orth(X)
            AX = apply(X)
            Hs = X.T @ AX
            theta, C = np.linalg.eigh(0.5 * (Hs + Hs.T))
            X, AX = X @ C, AX @ C
            continue
        theta = theta_all[:k]
        Cx = C[:k, :k]
        Cr = C[k:, :k]                           # coefficients on [W, P]
        P = S[:, k:] @ Cr
        AP = AS[:, k:] @ Cr
        X = X @ Cx + P
        AX = AX @ Cx + AP
    return theta, X, res, it, restarts
