"""ces_lobpcg (Section 3.1: block LOBPCG with soft and hard locking and the
Teter-Payne-Allan preconditioner) against the FP64 oracle: the oracle's own
LOBPCG on the same start block, dense eigenvalues, the oscillator levels and
the 13-atom workload's stored oracle eigenvalues.  Eigenvectors are compared
through subspace projectors (degenerate levels have no unique vectors)."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import lobpcg as ol
from conftest import golden_path

torch = pytest.importorskip("torch")
from paper_1404_3773_amd import ces  # noqa: E402

pytestmark = pytest.mark.gpu

FP64, MIXED = ces.CES_PREC_FP64, ces.CES_PREC_MIXED
SMALL = si.small(6, 8, R=9.0, k=8)


def _say(msg):
    print(msg, flush=True)


class Case:
    def __init__(self, w):
        self.w = w
        self.B = ces.Basis.for_workload(w)
        r, wr, th, wt, ph = self.B.grid()
        self.H = ces.Ham(self.B, torch.from_numpy(si.potential_on_grid(w, r, th, ph).reshape(-1)).cuda())
        self.bs = ob.basis_for(w)
        self.Vo = si.potential_on_grid(w, self.bs.r, self.bs.theta, self.bs.phi)

    def run(self, X0, n_check, res_tol, prec=FP64, Y=None, **kw):
        k = X0.shape[1]
        X = torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
        Yt = None if Y is None else torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()
        ev = torch.empty(k, dtype=torch.float64, device="cuda")
        rs = torch.empty(k, dtype=torch.float64, device="cuda")
        work = self.H.lobpcg_workspace(k, 0 if Y is None else Y.shape[1], prec)
        it, restarts = self.H.lobpcg(X, ev, rs, work, n_check=n_check, res_tol=res_tol,
                                     prec=prec, Y=Yt, **kw)
        return ev.cpu().numpy(), X.cpu().numpy().T, rs.cpu().numpy(), it, restarts


_cases = {}


def case(w):
    if w not in _cases:
        _cases[w] = Case(w)
    return _cases[w]


def projector_diff(A, B):
    return np.max(np.abs(A @ A.T - B @ B.T))


@pytest.mark.parametrize("g_scale", [1.0, 0.5])
def test_lobpcg_matches_oracle_lobpcg_and_dense(g_scale):
    c = case(SMALL)
    _say(f"case lobpcg small g_scale={g_scale}")
    Hd = oh.dense_H_real(c.bs, c.Vo)
    lam, U = np.linalg.eigh(Hd)
    X0 = si.random_block(c.B.d, 8, 3)
    th_o, X_o, _, it_o, _ = ol.lobpcg(lambda Z: oh.apply_H_real(c.bs, c.Vo, Z), X0, c.bs.lam,
                                      res_tol=1e-9, max_iter=400, n_check=6, g_scale=g_scale)
    th, X, res, it, rst = c.run(X0, 6, 1e-9, g_scale=g_scale, max_iter=400)
    scale = np.max(np.abs(lam))
    _say(f"  iterations gpu {it} oracle {it_o}, restarts {rst}; "
         f"eig err vs dense {np.max(np.abs(th[:6] - lam[:6])) / scale:.2e}")
    assert it < 400
    assert np.max(np.abs(th[:6] - lam[:6])) < 1e-11 * scale
    assert np.max(np.abs(th[:6] - th_o[:6])) < 1e-11 * scale
    assert np.all(res[:6] <= 1e-9 * np.maximum(1.0, np.abs(th[:6])) * 1.01)
    assert np.max(np.abs(X.T @ X - np.eye(8))) < 1e-12
    assert projector_diff(X[:, :6], U[:, :6]) < 1e-7
    assert projector_diff(X[:, :6], X_o[:, :6]) < 1e-7
    # the same algorithm from the same start: iteration counts close
    assert abs(it - it_o) <= max(3, it_o // 5)


def test_lobpcg_large_block_uses_both_factorisation_paths():
    """k = 64: the residual blocks start above the one-workgroup limit (60
    columns) and shrink below it as columns lock."""
    c = case(SMALL)
    _say("case lobpcg small k=64")
    lam = np.linalg.eigvalsh(oh.dense_H_real(c.bs, c.Vo))
    th, X, res, it, _ = c.run(si.random_block(c.B.d, 64, 4), 56, 1e-9, max_iter=400)
    assert it < 400
    assert np.max(np.abs(th[:56] - lam[:56])) < 1e-11 * np.max(np.abs(lam))
    assert np.max(np.abs(X.T @ X - np.eye(64))) < 1e-12


def test_lobpcg_harmonic_oscillator_levels():
    c = case(si.C1)
    _say("case lobpcg oscillator")
    th, X, res, it, _ = c.run(si.x0_block(si.C1, k=11), 10, 1e-9, max_iter=300)
    ref = np.array([0.75] + [1.25] * 3 + [1.75] * 6)
    assert it < 300
    assert np.max(np.abs(th[:10] - ref)) < 1e-8


def test_lobpcg_hard_and_soft_locking():
    c = case(SMALL)
    _say("case lobpcg locking")
    lam, U = np.linalg.eigh(oh.dense_H_real(c.bs, c.Vo))
    scale = np.max(np.abs(lam))
    # hard locking: constraints = the three lowest eigenvectors
    th, X, res, it, _ = c.run(si.random_block(c.B.d, 8, 4), 6, 1e-10, Y=U[:, :3],
                              max_iter=400)
    assert np.max(np.abs(th[:6] - lam[3:9])) < 1e-11 * scale
    assert np.max(np.abs(U[:, :3].T @ X)) < 1e-11
    # soft locking: a start block holding three exact eigenvectors converges
    # and keeps them
    X0 = si.random_block(c.B.d, 8, 5)
    X0[:, :3] = U[:, :3]
    th, X, res, it, _ = c.run(X0, 6, 1e-10, max_iter=400)
    assert np.max(np.abs(th[:6] - lam[:6])) < 1e-11 * scale
    assert projector_diff(X[:, :3], U[:, :3]) < 1e-9


def test_lobpcg_mixed_precision_products():
    """H W in FP32 (FP64 Gram products, factorisations and final
    Rayleigh-Ritz): eigenvalues within 1e-7 of the dense ones at residual
    tolerance 1e-5."""
    c = case(SMALL)
    lam = np.linalg.eigvalsh(oh.dense_H_real(c.bs, c.Vo))
    th, X, res, it, _ = c.run(si.random_block(c.B.d, 8, 3), 6, 1e-5, prec=MIXED, max_iter=400)
    _say(f"case lobpcg mixed: {it} iterations, err {np.max(np.abs(th[:6] - lam[:6])):.2e}")
    assert it < 400
    assert np.max(np.abs(th[:6] - lam[:6])) < 1e-7


@pytest.mark.timeout(300)
def test_lobpcg_13_atom_workload_matches_stored_oracle_eigenvalues():
    """The 26 bound states of the 13-atom workload (k = 32) from its seeded
    start block, against the oracle CheFSI eigenvalues stored by
    tests/golden/make_golden.py."""
    w = si.C2
    c = case(w)
    ref = np.loadtxt(golden_path(f"{w.name}_eigenvalues.txt"), comments="#")[:, 1]
    th, X, res, it, rst = c.run(si.x0_block(w), w.n_check, 1e-6, max_iter=500)
    err = np.max(np.abs(th[:w.n_check] - ref))
    _say(f"case lobpcg ico13: {it} iterations, {rst} restarts, max eig err {err:.2e} Ha")
    assert it < 500
    assert err < 1e-8
