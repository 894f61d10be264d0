"""Learned start density (oracle side): per-atom descriptors, atom-centred
correction functions, the per-cluster quadratic loss and a plain MLP with
hand-derived gradients, all in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This part is not in the paper: it predicts a correction to the
superposition-of-atomic-densities start (Section 3.2) so that the SCF needs
fewer steps; the converged answer does not depend on it.

  rho_0(x) = rho_SAD(x) + sum_j sum_q c_jq Phi_q(x - a_j; u_j),
  c_j = MLP(descriptors of atom j),

with Phi_q spherical Gaussians (q < 5) and dipoles along the atom's
environment direction u_j (q >= 5), so rho_0 rotates with the cluster and does
not depend on the order of the atoms.  Loss per cluster: the quadrature L2
distance between rho_0 and the converged density rho*,
  L = || sum c Phi - (rho* - rho_SAD) ||_W^2 = c^T M c - 2 p^T c + t,
M = Phi W Phi^T, p = Phi W (rho* - rho_SAD), t = ||rho* - rho_SAD||_W^2.
"""
from __future__ import annotations

import math

import numpy as np

# descriptor parameters
RC = 10.0                                  # cutoff radius of fc
G2_MU = 2.0 + 0.5 * np.arange(16)           # radial shells (bohr)
G2_ETA = 2.0
G4_ETA = 0.02
G4_ZL = ((1, 1.0), (1, -1.0), (4, 1.0), (4, -1.0))
ENV_SIGMA = 3.0
N_FEATURES = 24
# correction functions
SPH_SIGMA = (0.6, 0.9, 1.3, 1.9, 2.8)
DIP_SIGMA = (0.9, 1.4, 2.2)
N_CHANNELS = len(SPH_SIGMA) + len(DIP_SIGMA)


def cutoff(r):
    """fc(r) = (cos(pi r / RC) + 1) / 2 for r < RC, else 0."""
    return np.where(r < RC, 0.5 * (np.cos(math.pi * r / RC) + 1.0), 0.0)


def environment(atoms: np.ndarray):
    """u_j = sum_{i != j} exp(-r_ij^2 / (2 ENV_SIGMA^2)) (a_i - a_j) / r_ij;
    returns (u, unit directions (zero where |u| <= 1e-6))."""
    n = len(atoms)
    u = np.zeros((n, 3))
    for j in range(n):
        for i in range(n):
            if i == j:
                continue
            v = atoms[i] - atoms[j]
            r = np.linalg.norm(v)
            u[j] += math.exp(-r * r / (2 * ENV_SIGMA ** 2)) * v / r
    norm = np.linalg.norm(u, axis=1)
    dirs = np.where(norm[:, None] > 1e-6, u / np.maximum(norm, 1e-300)[:, None], 0.0)
    return u, dirs


def descriptors(atoms: np.ndarray) -> np.ndarray:
    """(n, 24): 16 radial symmetry functions G2 (Gaussian shells at G2_MU),
    4 angular G4 (zeta, lambda) in G4_ZL, |a_j| / 8, n / 40, the Gaussian
    coordination sum_i exp(-r_ij^2 / 18) / 10, and |u_j|."""
    n = len(atoms)
    F = np.zeros((n, N_FEATURES))
    u, _ = environment(atoms)
    for j in range(n):
        for i in range(n):
            if i == j:
                continue
            r = np.linalg.norm(atoms[i] - atoms[j])
            F[j, :16] += np.exp(-G2_ETA * (r - G2_MU) ** 2) * cutoff(r)
            F[j, 22] += math.exp(-r * r / (2 * ENV_SIGMA ** 2)) / 10.0
        for i in range(n):
            for k in range(i + 1, n):
                if i == j or k == j:
                    continue
                vi, vk = atoms[i] - atoms[j], atoms[k] - atoms[j]
                ri, rk = np.linalg.norm(vi), np.linalg.norm(vk)
                cos = vi @ vk / (ri * rk)
                g = math.exp(-G4_ETA * (ri * ri + rk * rk)) * cutoff(ri) * cutoff(rk)
                for q, (zeta, lam) in enumerate(G4_ZL):
                    F[j, 16 + q] += 2.0 ** (1 - zeta) * (1 + lam * cos) ** zeta * g
        F[j, 20] = np.linalg.norm(atoms[j]) / 8.0
        F[j, 21] = n / 40.0
        F[j, 23] = np.linalg.norm(u[j])
    return F


def correction_functions(points: np.ndarray, atoms: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Phi at the points: (n_atoms, N_CHANNELS, *points.shape[:-1]).
    q < 5: (2 pi s^2)^{-3/2} exp(-r^2 / (2 s^2)), s = SPH_SIGMA[q];
    q >= 5: (2 pi s^2)^{-3/2} ((x - a_j) . u_j / s) exp(-r^2 / (2 s^2))."""
    shape = points.shape[:-1]
    out = np.zeros((len(atoms), N_CHANNELS) + shape)
    for j, a in enumerate(atoms):
        d = points - a
        r2 = np.sum(d * d, axis=-1)
        proj = d @ dirs[j]
        for q, s in enumerate(SPH_SIGMA):
            out[j, q] = (2 * math.pi * s * s) ** -1.5 * np.exp(-r2 / (2 * s * s))
        for q, s in enumerate(DIP_SIGMA):
            out[j, len(SPH_SIGMA) + q] = ((2 * math.pi * s * s) ** -1.5 * proj / s
                                          * np.exp(-r2 / (2 * s * s)))
    return out


def quadratic_form(Phi: np.ndarray, weights: np.ndarray, target: np.ndarray):
    """M = Phi W Phi^T, p = Phi W target, t = target W target over the grid
    (Phi flattened to (n_atoms * N_CHANNELS, n_grid), atom-major)."""
    P = Phi.reshape(-1, weights.size)
    w = weights.reshape(-1)
    tg = target.reshape(-1)
    return (P * w) @ P.T, (P * w) @ tg, float(np.sum(w * tg * tg))


def cluster_loss(M, p, t, C):
    """L = c^T M c - 2 p^T c + t (c = C flattened atom-major) and dL/dC."""
    c = C.reshape(-1)
    L = c @ M @ c - 2 * p @ c + t
    return L, (2 * (M @ c) - 2 * p).reshape(C.shape)


# ------------------------------------------------------------------- MLP

def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, seed):
    """Weights N(0, 1/fan_in), zero biases; W_l has shape (in, out)."""
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((a, b)) / math.sqrt(a), np.zeros(b))
            for a, b in zip(sizes[:-1], sizes[1:])]


def forward(params, X, mean, std):
    """Standardise X, then hidden layers z = h W + b, h = silu(z), and a
    linear output layer.  Returns (output, cache)."""
    h = (X - mean) / std
    cache = [(h, None)]
    for li, (W, b) in enumerate(params):
        z = h @ W + b
        h = silu(z) if li + 1 < len(params) else z
        cache.append((h, z))
    return h, cache


def backward(params, cache, dout):
    """Gradients (dW, db) of sum(dout * output) by the chain rule."""
    grads = [None] * len(params)
    g = dout
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_prev = cache[li][0]
        if li + 1 < len(params):
            g = g * silu_grad(cache[li + 1][1])
        grads[li] = (h_prev.T @ g, g.sum(axis=0))
        g = g @ W.T
    return grads


def adam_update(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on every weight and bias, in place."""
    for li in range(len(params)):
        for a in range(2):
            g = grads[li][a]
            m[li][a] = b1 * m[li][a] + (1 - b1) * g
            v[li][a] = b2 * v[li][a] + (1 - b2) * g * g
            mh = m[li][a] / (1 - b1 ** step)
            vh = v[li][a] / (1 - b2 ** step)
            params[li][a][...] -= lr * mh / (np.sqrt(vh) + eps)
