"""The discretised Kohn-Sham operator H and its product with a block (oracle).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definition (Section 2.2.4, eq. matvec_final with the quadratures of
eqs. Ar_lm and Arlm_to_coeff):
    Z = 1/2 Lambda o Y + forward_transform( V_eff * inverse_transform(Y) )
         [ + P diag(h) P^T Y   for Kleinman-Bylander projectors, Section 2.3.2 ]
In matrix form H = 1/2 diag(Lambda) + B^H W diag(V) B, B[g,alpha] = F_alpha(x_g)
and W the tensor quadrature weights: the quadrature (pseudospectral) operator
that the transforms compute.

`dense_H_*` build that matrix explicitly (small bases); `apply_H_*` follow the
paper's separable route step by step: radial sum (eq. G_lmr), Legendre sum per
m, inverse FFT in phi; multiply by V; FFT in phi, Legendre quadrature in
t = cos(theta) (eq. Ar_lm), radial quadrature (eq. Arlm_to_coeff).
"""
from __future__ import annotations

import math

import numpy as np

from .basis import (Basis, basis_matrix_complex, complex_to_real, index,
                    real_to_complex)


# ----------------------------------------------------------- dense (small)

def dense_H_complex(bs: Basis, V: np.ndarray) -> np.ndarray:
    """H = 1/2 diag(Lambda) + B^H diag(W V) B in the complex basis."""
    B = basis_matrix_complex(bs)
    wv = (bs.weights() * V).reshape(-1)
    H = B.conj().T @ (wv[:, None] * B)
    H[np.diag_indices(bs.d)] += 0.5 * bs.lam
    return H


def dense_H_real(bs: Basis, V: np.ndarray) -> np.ndarray:
    """The same operator in the real-harmonic layout: U H_c U^H."""
    Hc = dense_H_complex(bs, V)
    T = complex_to_real(Hc, bs.L, bs.N)                 # U H
    H = complex_to_real(T.conj().T, bs.L, bs.N).conj().T  # (U (U H)^H)^H = U H U^H
    assert np.max(np.abs(H.imag)) <= 1e-12 * max(1.0, np.max(np.abs(H.real)))
    return np.ascontiguousarray(H.real)


# --------------------------------------------------------- separable route

def _coeff_blocks(bs: Basis, F: np.ndarray):
    """Split a d x k coefficient block into per-l arrays C_l[m+l, n, i]."""
    N = bs.N
    return [F[(l * l) * N:((l + 1) ** 2) * N].reshape(2 * l + 1, N, -1)
            for l in range(bs.L)]


def inverse_transform(bs: Basis, F: np.ndarray) -> np.ndarray:
    """Coefficients (d x k, complex) -> values on the grid (n_r, n_theta, n_phi, k).

    Step 1, eq. G_lmr: G(l,m; r_k) = sum_n f_lmn R_ln(r_k).
    Step 2, inverse SHT per radial node: per m, sum over l >= |m| of
    c_l|m| P_l^|m|(t_j) G(l,m; r), then sum over m of e^{i m phi_p} (inverse FFT).
    """
    L, Np = bs.L, bs.n_phi
    assert Np >= 2 * L - 1, "phi grid too coarse for the band limit"
    k = F.shape[1]
    C = _coeff_blocks(bs, F)
    G = [np.einsum("mni,nr->mri", C[l], bs.Rtab[l]) for l in range(L)]
    S = np.zeros((bs.n_r, bs.n_theta, Np, k), dtype=np.complex128)
    for m in range(-(L - 1), L):
        am = abs(m)
        Gm = np.stack([G[l][m + l] for l in range(am, L)])        # [l, r, i]
        Fm = np.tensordot(bs.Ptab[am:, am], Gm, axes=([0], [0]))   # [j, r, i]
        S[:, :, m % Np, :] += Fm.transpose(1, 0, 2)
    return np.fft.ifft(S, axis=2) * Np


def forward_transform(bs: Basis, f: np.ndarray) -> np.ndarray:
    """Values on the grid (n_r, n_theta, n_phi, k) -> coefficients (d x k).

    eq. Ar_lm: A(r; l,m) = c_lm int P_l^m(t) [ int f e^{-i m phi} dphi ] dt with
    the phi integral by the FFT (2 pi / N_phi sum) and the t integral by the
    Gauss rule; eq. Arlm_to_coeff: f_lmn = sum_k w_k A(r_k; l,m) R_ln(r_k).
    """
    L, N, Np = bs.L, bs.N, bs.n_phi
    k = f.shape[3]
    Fh = np.fft.fft(f, axis=2) * (2.0 * math.pi / Np)   # [r, j, bin, i]
    out = np.zeros((bs.d, k), dtype=np.complex128)
    for m in range(-(L - 1), L):
        am = abs(m)
        Pw = bs.Ptab[am:, am] * bs.wt[None, :]                     # [l, j]
        A = np.tensordot(Pw, Fh[:, :, m % Np, :], axes=([1], [1]))  # [l, r, i]
        for l in range(am, L):
            coef = (bs.Rtab[l] * bs.wr[None, :]) @ A[l - am]        # [n, i]
            a0 = index(l, m, 0, N)
            out[a0:a0 + N] = coef
    return out


def apply_H_complex(bs: Basis, V: np.ndarray, F: np.ndarray,
                    chunk: int | None = None) -> np.ndarray:
    """Z = 1/2 Lambda o F + forward(V * inverse(F)), eq. matvec_final."""
    F = np.asarray(F, dtype=np.complex128)
    if F.ndim == 1:
        return apply_H_complex(bs, V, F[:, None], chunk)[:, 0]
    k = F.shape[1]
    if chunk is None:
        chunk = max(1, int(2.0e8 // (bs.n_grid * 16 * 3)))
    out = np.empty_like(F)
    for s in range(0, k, chunk):
        Fs = F[:, s:s + chunk]
        f = inverse_transform(bs, Fs)
        out[:, s:s + chunk] = forward_transform(bs, V[..., None] * f)
    out += 0.5 * bs.lam[:, None] * F
    return out


def apply_H_real(bs: Basis, V: np.ndarray, X: np.ndarray,
                 proj: np.ndarray | None = None, h: np.ndarray | None = None,
                 chunk: int | None = None) -> np.ndarray:
    """H X in the real-harmonic layout (X real, d x k), with optional
    Kleinman-Bylander term P diag(h) P^T X (P real-layout coefficients,
    d x n_proj), Section 2.3.2."""
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    if one:
        X = X[:, None]
    Fc = real_to_complex(X, bs.L, bs.N)
    Zc = apply_H_complex(bs, V, Fc, chunk)
    Z = complex_to_real(Zc, bs.L, bs.N)
    assert np.max(np.abs(Z.imag)) <= 1e-10 * max(1.0, np.max(np.abs(Z.real)))
    Z = Z.real
    if proj is not None and proj.shape[1] > 0:
        Z = Z + proj @ (h[:, None] * (proj.T @ X))
    return Z[:, 0] if one else Z


def apply_H_subset(bs: Basis, V: np.ndarray, kept: np.ndarray, X: np.ndarray,
                   proj: np.ndarray | None = None, h=None) -> np.ndarray:
    """H X in the basis of the functions `kept` (uniform-layout positions, e.g.
    a kinetic-energy cutoff): the operator of a subset of an orthonormal basis
    is the submatrix of H, so X is placed at those positions, H is applied and
    the same positions are read back.  proj: uniform-layout projector
    coefficients (their restriction is the subset's own)."""
    Xf = np.zeros((bs.d, X.shape[1]))
    Xf[kept] = X
    return apply_H_real(bs, V, Xf, proj=proj, h=h)[kept]


def to_grid_real(bs: Basis, X: np.ndarray) -> np.ndarray:
    """Real-layout coefficients -> real grid values (n_r, n_theta, n_phi, k)."""
    f = inverse_transform(bs, real_to_complex(np.atleast_2d(X.T).T, bs.L, bs.N))
    return f.real


def from_grid_real(bs: Basis, f: np.ndarray) -> np.ndarray:
    """Real grid values (n_r, n_theta, n_phi, k) -> real-layout coefficients."""
    F = forward_transform(bs, f.astype(np.complex128))
    return complex_to_real(F, bs.L, bs.N).real


def kb_projectors(bs: Basis, p_grid: np.ndarray) -> np.ndarray:
    """Projector coefficients: sample each projector on the grid and
    forward-transform it (Section 2.3.2); p_grid is (n_r, n_theta, n_phi, n_proj)."""
    return from_grid_real(bs, p_grid)
