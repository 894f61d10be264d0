"""Pins of the kinetic-energy-cutoff basis (the non-uniform basis the footnote
of Section 2.2.1 proposes: only the spherical waves with Lambda_ln / 2 below a
cutoff), against facts fixed independently of the oracle's transforms: the
cutoff rule itself by brute force, the free particle's spectrum, the
interlacing theorem for a subset of an orthonormal basis, and the
harmonic-oscillator levels."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import basis as ob
from oracle import hamiltonian as oh


def test_cutoff_keeps_exactly_the_waves_below_it():
    bs = ob.make_basis(9, 12, 10.0, 24, 18, 36)
    lam = 0.5 * (bs.b / bs.R) ** 2
    for e_cut in (0.3, 1.0, 2.5, 1e9):
        Nl = ob.ke_cutoff_counts(bs, e_cut)
        assert np.all(np.diff(Nl) <= 0) and Nl[0] <= bs.N      # fewer waves at higher l
        kept = ob.ke_cutoff_index(bs, e_cut)
        assert len(kept) == int(np.sum((2 * np.arange(bs.L) + 1) * Nl))
        assert np.all(np.diff(kept) > 0)                        # the uniform order, restricted
        brute = sorted(ob.index(l, m, n, bs.N) for l in range(bs.L) for m in range(-l, l + 1)
                       for n in range(bs.N) if lam[l, n] <= e_cut)
        assert list(kept) == brute
    assert len(ob.ke_cutoff_index(bs, 1e9)) == bs.d


def test_cutoff_basis_free_particle_spectrum():
    """V = 0: the eigenvalues in the cutoff basis are the kept b_ln^2 / (2 R^2),
    each 2l + 1 times."""
    w = si.small(6, 8, R=9.0, potential="zero")
    bs = ob.basis_for(w)
    e_cut = 1.2
    kept = ob.ke_cutoff_index(bs, e_cut)
    V = np.zeros((bs.n_r, bs.n_theta, bs.n_phi))
    H = oh.apply_H_subset(bs, V, kept, np.eye(len(kept)))
    ref = np.sort(np.concatenate([np.full(2 * l + 1, 0.5 * (bs.b[l, n] / bs.R) ** 2)
                                  for l in range(bs.L) for n in range(bs.N)
                                  if 0.5 * (bs.b[l, n] / bs.R) ** 2 <= e_cut]))
    assert np.max(np.abs(np.linalg.eigvalsh(0.5 * (H + H.T)) - ref)) < 1e-12 * ref[-1]


def test_cutoff_basis_eigenvalues_interlace_the_full_basis():
    """A subset of an orthonormal basis gives a compression of H, so by
    Cauchy's interlacing theorem lambda_j(full) <= lambda_j(cutoff) <=
    lambda_{j + d - d_E}(full) for every j."""
    w = si.small(6, 8, R=9.0)
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    full = np.linalg.eigvalsh(oh.dense_H_real(bs, V))
    for e_cut in (0.8, 2.0):
        kept = ob.ke_cutoff_index(bs, e_cut)
        dE = len(kept)
        HE = oh.apply_H_subset(bs, V, kept, np.eye(dE))
        lamE = np.linalg.eigvalsh(0.5 * (HE + HE.T))
        tol = 1e-12 * np.max(np.abs(full))
        assert np.all(lamE >= full[:dE] - tol)
        assert np.all(lamE <= full[bs.d - dE:] + tol)


def test_cutoff_basis_beats_a_uniform_basis_of_the_same_size():
    """omega (n + 3/2), omega = 0.5: a cutoff basis holding 59 % of the uniform
    basis's functions gives the lowest ten levels to 3e-6, where a uniform
    basis of the same size (7 instead of 12 radial functions per l) misses by
    1e-2: the advantage the footnote of Section 2.2.1 claims for the cutoff."""
    w = si.C1
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    ref = np.array([0.75] + [1.25] * 3 + [1.75] * 6)
    e_cut = 0.7 * 0.5 * (bs.b[0, bs.N - 1] / bs.R) ** 2
    kept = ob.ke_cutoff_index(bs, e_cut)
    HE = oh.apply_H_subset(bs, V, kept, np.eye(len(kept)))
    lamE = np.linalg.eigvalsh(0.5 * (HE + HE.T))[:10]
    w7 = si.Workload("ho_L9_N7", L=9, N=7, R=10.0, n_r=24, n_theta=18, n_phi=36,
                     radial_rule=si.RADIAL_GAUSS_LEGENDRE, k=10, n_check=10, degree=12,
                     x0_seed=0, geom_seed=0, potential="harmonic")
    b7 = ob.basis_for(w7)
    lam7 = np.linalg.eigvalsh(oh.dense_H_real(b7, si.potential_on_grid(w7, b7.r, b7.theta,
                                                                      b7.phi)))[:10]
    assert abs(len(kept) - b7.d) <= 0.02 * bs.d
    assert np.max(np.abs(lamE - ref)) < 3e-6
    assert np.max(np.abs(lam7 - ref)) > 1e-3
