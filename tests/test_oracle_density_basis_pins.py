"""Pins of the non-dualing density basis (Section 2.2.5's first comment: the
density of orbitals with l <= L-1 holds angular degrees up to 2(L-1), so it
needs a larger basis than the orbitals), against facts fixed independently
of the oracle's transforms: the product rules of spherical harmonics, exact
quadrature (grid refinement leaves the coefficients unchanged), and the
closed-form potential of a Gaussian charge."""
import math

import numpy as np
import pytest
from scipy import special

import synth_inputs as si
from oracle import basis as ob
from oracle import density as od
from oracle import hamiltonian as oh
from oracle import scf as osf


def _basis_function_on_grid(bs, l, m, n):
    e = np.zeros((bs.d, 1))
    e[ob.index(l, m, n, bs.N)] = 1.0
    return oh.to_grid_real(bs, e)[..., 0]


def _allowed(la, ma, lb, mb, lr, mr):
    """Real-harmonic product rules: triangle and parity (Gaunt) in l; |m'| is
    |ma| + |mb| or ||ma| - |mb||; sine-type (m < 0) factors combine like
    signs: cos*cos and sin*sin give cosines, cos*sin gives sines."""
    if not (abs(la - lb) <= lr <= la + lb) or (la + lb + lr) % 2:
        return False
    if abs(mr) not in (abs(ma) + abs(mb), abs(abs(ma) - abs(mb))):
        return False
    sin_a, sin_b = ma < 0, mb < 0
    want_sin = sin_a != sin_b
    if abs(mr) == 0:
        return not want_sin
    return (mr < 0) == want_sin


def test_density_basis_holds_products_of_orbitals_exactly_in_angle():
    """rho = F_a F_b with l_a + l_b > L - 1: its density-basis coefficients obey
    the product rules of the harmonics, carry the components with l' above
    the orbitals' cutoff, and do not change when the angular grid is refined
    (the orbitals' grid already integrates them exactly)."""
    L, N = 4, 5
    bs = ob.make_basis(L, N, 8.0, 20, 2 * L, 4 * L)
    br = od.density_basis_for(bs)
    fine = ob.make_basis(L, N, 8.0, 20, 4 * L, 8 * L)
    brf = od.density_basis_for(fine)
    assert br.L == 2 * L - 1 and np.array_equal(br.r, bs.r)
    for (la, ma, na), (lb, mb, nb) in [((3, 2, 0), (3, -1, 1)), ((2, 0, 1), (3, 3, 0)),
                                       ((3, -3, 2), (3, -2, 0)), ((1, 1, 0), (3, 0, 3))]:
        rho = _basis_function_on_grid(bs, la, ma, na) * _basis_function_on_grid(bs, lb, mb, nb)
        rho_f = _basis_function_on_grid(fine, la, ma, na) * _basis_function_on_grid(fine, lb, mb,
                                                                                     nb)
        tau = od.density_coefficients(br, rho)
        tau_f = od.density_coefficients(brf, rho_f)
        big = np.max(np.abs(tau))
        assert np.max(np.abs(tau - tau_f)) < 1e-12 * big
        top = 0.0
        for lr in range(br.L):
            for mr in range(-lr, lr + 1):
                blk = tau[ob.index(lr, mr, 0, N):ob.index(lr, mr, 0, N) + N]
                if _allowed(la, ma, lb, mb, lr, mr):
                    if lr == la + lb:
                        top = max(top, np.max(np.abs(blk)))
                else:
                    assert np.max(np.abs(blk)) < 1e-12 * big, (la, ma, lb, mb, lr, mr)
        # the highest allowed degree, beyond the orbitals' cutoff, is present
        assert la + lb > L - 1 and top > 1e-3 * big


def test_density_basis_hartree_of_an_offcentre_gaussian():
    """V_H of a unit Gaussian charge off the centre is Q erf(s / (sqrt2 sigma))
    / s, s the distance to its centre.  The density basis (l' <= 2(L-1))
    reproduces it to 1e-6 on the grid; the orbitals' own basis (the dualing
    choice) misses by more than 1e-4."""
    L, N, sigma = 8, 24, 1.0
    bs = ob.make_basis(L, N, 12.0, 36, 2 * L, 4 * L)
    br = od.density_basis_for(bs)
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    c = np.array([0.3, -0.2, 2.0])
    d2 = np.sum((pts - c) ** 2, axis=-1)
    rho = (2 * math.pi * sigma ** 2) ** -1.5 * np.exp(-d2 / (2 * sigma ** 2))
    s = np.sqrt(d2)
    exact = special.erf(s / (math.sqrt(2.0) * sigma)) / s
    err = {}
    for name, b in (("dualing", bs), ("density", br)):
        V = od.hartree_grid(b, od.density_coefficients(b, rho))
        err[name] = np.max(np.abs(V - exact))
    assert err["density"] < 1e-6
    assert err["dualing"] > 1e-4


def test_scf_with_density_basis_converges_near_the_dualing_run():
    """The SCF with the density basis for the Hartree potential converges; its
    occupied eigenvalues differ from the dualing run's by the truncation of
    the density that the larger basis removes (about 1e-2 Ha for this
    5-atom cluster at L = 8)."""
    w = si.small(8, 16, R=16.0, n_r=24, n_theta=16, n_phi=32, potential="scf")
    bs = ob.basis_for(w)
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    atoms = si.scf_cluster(1)[:5]
    n_occ, n_guard = si.scf_occupation(len(atoms))
    rion = si.ion_density(pts, atoms)
    out = []
    for dens in (None, od.density_basis_for(bs)):
        scf = osf.ClusterSCF(bs, atoms, si.gaussian_wells(pts, atoms), rion, n_occ, n_guard,
                             degree=w.degree, density_basis=dens)
        th, st, _, _ = scf.run(rion, si.random_block(bs.d, n_occ + n_guard, 502),
                               v0=si.lanczos_start(bs.d), tol=1e-9, max_steps=100)
        assert st < 100
        out.append(th[:n_occ])
    diff = np.max(np.abs(out[0] - out[1]))
    assert 1e-4 < diff < 3e-2
