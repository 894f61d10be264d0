"""Full-size parity of H*X on the large workload shapes (sampled columns).

The 147-atom Mackay cluster runs at its full size (L_max = 60, N = 120,
180 x 122 x 244 grid, k = 400).  The 309-atom fcc workload's basis and grid
(L_max = 80, N = 150, 225 x 162 x 324) are used with the 13 central atoms of
its geometry for V_eff and one atom's projectors, so that the oracle side
stays within minutes; the kernels see the same shapes and tile counts.
Tolerances as in test_gpu_parity.py.
"""
import dataclasses

import numpy as np
import pytest

import synth_inputs as si
from oracle import basis as ob
from oracle import hamiltonian as oh

torch = pytest.importorskip("torch")
from paper_1404_3773_amd import ces  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-11, 5e-5


def _say(msg):
    print(msg, flush=True)


def rel_err(got, ref):
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


def _run(w, atoms, k, cols, proj_atoms=None, proj_cols=None, mixed_vs_fp64_all=False):
    B = ces.Basis.for_workload(w)
    r, wr, th, wt, ph = B.grid()
    V = si.gaussian_wells(si.spherical_to_cartesian(r, th, ph), atoms)
    bs = ob.basis_for(w)
    Vo = si.gaussian_wells(si.spherical_to_cartesian(bs.r, bs.theta, bs.phi), atoms)
    P = h = None
    proj_t = None
    if proj_atoms is not None:
        pg, h = si.kb_projector_values(si.spherical_to_cartesian(bs.r, bs.theta, bs.phi),
                                       proj_atoms)
        pg, h = pg[:, proj_cols], h[proj_cols]
        P = oh.kb_projectors(bs, pg.reshape(*Vo.shape, -1))
        proj_t = torch.from_numpy(np.ascontiguousarray(P.T)).cuda()
    H = ces.Ham(B, torch.from_numpy(V.reshape(-1)).cuda(), proj=proj_t, energies=h)
    X = si.random_block(B.d, k, 17)
    Z = oh.apply_H_real(bs, Vo, X[:, cols], proj=P, h=h)
    Xt = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    del X
    outs = {}
    for prec, tol in ((ces.CES_PREC_FP64, TOL64), (ces.CES_PREC_MIXED, TOL32)):
        work = H.workspace(k, prec)
        Yt = torch.empty_like(Xt)
        H.apply_H(Xt, Yt, prec, work)
        torch.cuda.synchronize()
        Y = Yt[cols].cpu().numpy().T
        for c in range(len(cols)):
            e = rel_err(Y[:, c], Z[:, c])
            _say(f"  prec={prec} column {cols[c]} rel err {e:.2e}")
            assert e < tol, (prec, cols[c], e)
        del work
        if mixed_vs_fp64_all:
            outs[prec] = Yt
        else:
            del Yt
        torch.cuda.empty_cache()
    if mixed_vs_fp64_all:
        # every column: the FP32 path against the FP64 one (the FP64 path is the
        # oracle's to 1e-11 on the sampled columns)
        y64, y32 = outs[ces.CES_PREC_FP64], outs[ces.CES_PREC_MIXED]
        e = ((y32 - y64).abs().amax(dim=1) / y64.abs().amax(dim=1)).max().item()
        _say(f"  mixed vs fp64, all {k} columns: max rel err {e:.2e}")
        assert e < TOL32


@pytest.mark.timeout(600)
def test_apply_H_147_atom_cluster_full_size():
    w = si.C3
    _say(f"case apply_H full size {w.name} k={w.k}")
    _run(w, si.atoms_for(w), w.k, [0, w.k - 1])


@pytest.mark.timeout(600)
def test_apply_H_309_atom_basis_full_size_with_projectors():
    w = si.C4
    atoms = si.atoms_for(w)
    central = atoms[np.argsort(np.linalg.norm(atoms, axis=1))[:13]]
    _say(f"case apply_H full basis {w.name} (13 central wells, 2 projectors) k=64")
    _run(w, central, 64, [5], proj_atoms=central[1:2], proj_cols=[0, 2])


@pytest.mark.timeout(900)
def test_apply_H_309_atom_basis_full_block_k1000():
    """The 309-atom basis and grid at the workload's full block (k = 1000):
    the angular intermediate then holds n_r n_theta (2L - 1) k = 5.9e9
    elements, past 2^31, so every 64-bit index path of the Legendre, phi and
    projector kernels is crossed.  Sampled columns 0 and 999 against the
    oracle in both precisions; all columns mixed against FP64."""
    w = si.C4
    atoms = si.atoms_for(w)
    central = atoms[np.argsort(np.linalg.norm(atoms, axis=1))[:13]]
    n_r, n_t, S = w.n_r, w.n_theta, 2 * w.L - 1
    assert n_r * n_t * S * w.k > 2 ** 31
    _say(f"case apply_H full basis {w.name} (13 central wells, 2 projectors) k={w.k}")
    _run(w, central, w.k, [0, w.k - 1], proj_atoms=central[1:2], proj_cols=[0, 2],
         mixed_vs_fp64_all=True)
