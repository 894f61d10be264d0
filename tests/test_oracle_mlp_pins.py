"""Pins of the learned-start oracle (oracle/mlp.py).

- MLP gradients match central finite differences of the loss in FP64.
- Descriptors are invariant under rotations about the ball centre and under
  permutations of the atoms, and reduce to closed forms for two and three atoms.
- Spherical correction functions carry unit charge; dipoles carry none and
  have first moment sigma along u; the predicted correction rotates with the
  cluster.
- The quadratic form equals the brute-force grid norm of rho_0 - rho*.
- A first Adam step moves every parameter by lr * sign(gradient).
"""
import math

import numpy as np

import synth_inputs as si
from oracle import basis as ob
from oracle import mlp as om


def _rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q * np.sign(np.linalg.det(q))


def test_descriptors_two_and_three_atom_closed_forms():
    r = 3.1
    F = om.descriptors(np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]]))
    ref = np.exp(-om.G2_ETA * (r - om.G2_MU) ** 2) * 0.5 * (math.cos(math.pi * r / om.RC) + 1)
    assert np.max(np.abs(F[0, :16] - ref)) < 1e-15 and np.all(F[:, 16:20] == 0)
    # equilateral triangle: each angle is 60 degrees
    a = np.array([[0, 0, 0], [r, 0, 0], [r / 2, r * math.sqrt(3) / 2, 0]])
    F = om.descriptors(a)
    fc = 0.5 * (math.cos(math.pi * r / om.RC) + 1)
    for q, (zeta, lam) in enumerate(om.G4_ZL):
        ref = 2.0 ** (1 - zeta) * (1 + lam * 0.5) ** zeta * math.exp(-2 * om.G4_ETA * r * r) * fc ** 2
        assert abs(F[0, 16 + q] - ref) < 1e-14


def test_descriptors_rotation_and_permutation_invariant():
    atoms = si.scf_cluster(11)[:9]
    F = om.descriptors(atoms)
    Q = _rotation(1)
    assert np.max(np.abs(om.descriptors(atoms @ Q.T) - F)) < 1e-12
    perm = np.random.default_rng(2).permutation(len(atoms))
    assert np.max(np.abs(om.descriptors(atoms[perm]) - F[perm])) < 1e-12
    _, d = om.environment(atoms)
    _, dr = om.environment(atoms @ Q.T)
    assert np.max(np.abs(dr - d @ Q.T)) < 1e-12


def test_correction_functions_moments():
    bs = ob.make_basis(8, 40, 24.0, 160, 16, 32, ob.RADIAL_GAUSS_JACOBI_R2)   # tails inside
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    u = np.array([[0.0, 0.6, 0.8]])
    Phi = om.correction_functions(pts, np.zeros((1, 3)), u)[0]
    W = bs.weights()
    for q, s in enumerate(om.SPH_SIGMA):
        assert abs(np.sum(W * Phi[q]) - 1.0) < 1e-9
    proj = pts @ u[0]
    for q, s in enumerate(om.DIP_SIGMA):
        ph = Phi[len(om.SPH_SIGMA) + q]
        assert abs(np.sum(W * ph)) < 1e-12
        assert abs(np.sum(W * ph * proj) - s) < 1e-9


def test_correction_rotates_with_cluster():
    atoms = si.scf_cluster(12)[:6]
    Q = _rotation(3)
    pts = np.random.default_rng(4).uniform(-6, 6, (50, 3))
    _, d = om.environment(atoms)
    _, dq = om.environment(atoms @ Q.T)
    C = np.random.default_rng(5).standard_normal((len(atoms), om.N_CHANNELS))
    f = np.einsum("jq,jqp->p", C, om.correction_functions(pts, atoms, d))
    fq = np.einsum("jq,jqp->p", C, om.correction_functions(pts @ Q.T, atoms @ Q.T, dq))
    assert np.max(np.abs(f - fq)) < 1e-12


def test_quadratic_form_equals_grid_norm():
    bs = ob.make_basis(6, 12, 10.0, 18, 12, 24, ob.RADIAL_GAUSS_JACOBI_R2)
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    atoms = si.scf_cluster(13)[:4] * 0.6
    _, d = om.environment(atoms)
    Phi = om.correction_functions(pts, atoms, d)
    target = np.random.default_rng(6).standard_normal(pts.shape[:-1])
    W = bs.weights()
    M, p, t = om.quadratic_form(Phi, W, target)
    C = np.random.default_rng(7).standard_normal((len(atoms), om.N_CHANNELS))
    L, G = om.cluster_loss(M, p, t, C)
    diff = np.einsum("jq,jq...->...", C, Phi) - target
    assert abs(L - np.sum(W * diff * diff)) < 1e-10 * abs(L)
    # gradient: 2 <Phi_jq, diff>_W
    G_ref = 2 * np.tensordot(Phi, W * diff, axes=([2, 3, 4], [0, 1, 2]))
    assert np.max(np.abs(G - G_ref)) < 1e-9


def test_mlp_gradients_match_finite_differences():
    rng = np.random.default_rng(8)
    sizes = [om.N_FEATURES, 7, 6, 5, om.N_CHANNELS]
    params = om.init_params(sizes, 9)
    X = rng.standard_normal((11, om.N_FEATURES))
    mean, std = X.mean(0), X.std(0) + 0.5
    A = rng.standard_normal((11 * om.N_CHANNELS, 11 * om.N_CHANNELS))
    M = A @ A.T
    p = rng.standard_normal(11 * om.N_CHANNELS)

    def loss():
        out, cache = om.forward(params, X, mean, std)
        L, G = om.cluster_loss(M, p, 0.0, out)
        return L, G, cache

    L, G, cache = loss()
    grads = om.backward(params, cache, G)
    h = 1e-6
    for li in range(len(params)):
        for a in range(2):
            P = params[li][a]
            for idx in [tuple(rng.integers(0, s) for s in P.shape) for _ in range(4)]:
                old = P[idx]
                P[idx] = old + h
                Lp = loss()[0]
                P[idx] = old - h
                Lm = loss()[0]
                P[idx] = old
                fd = (Lp - Lm) / (2 * h)
                assert abs(grads[li][a][idx] - fd) < 1e-6 * max(1.0, abs(fd)), (li, a, idx)


def test_first_adam_step_is_sign_step():
    params = om.init_params([4, 3, 2], 10)
    grads = [(np.random.default_rng(11).standard_normal(W.shape),
              np.random.default_rng(12).standard_normal(b.shape)) for W, b in params]
    before = [(W.copy(), b.copy()) for W, b in params]
    m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    om.adam_update(params, grads, m, v, 1, 0.01, eps=0.0)
    for li in range(len(params)):
        for a in range(2):
            step = before[li][a] - params[li][a]
            assert np.max(np.abs(step - 0.01 * np.sign(grads[li][a]))) < 1e-15
