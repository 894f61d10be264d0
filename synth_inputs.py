"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only *describes workloads*: basis/grid sizes, cluster geometries,
the seeded random start block X0, and closed-form model potentials evaluated at
caller-supplied Cartesian points.  It holds none of the spectral method's
arithmetic (no basis functions, no quadrature, no transforms): each side builds
its own grid and evaluates the potential there.

Workloads stand in for the paper's Al/Ba/fullerene clusters (Section 4), whose
coordinates and pseudopotential parameters are not available; the shapes follow
the paper's icosahedral / fcc cluster families and its rule that the outermost
atom sits 8-16 bohr inside the sphere (start of Section 4).
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

# Radial quadrature rules (same numbering as the C header).
RADIAL_GAUSS_JACOBI_R2 = 0   # Gauss-Jacobi nodes for weight r^2 on [0,R] (Section 2.2.2)
RADIAL_GAUSS_LEGENDRE = 1    # Gauss-Legendre nodes on [0,R], r^2 folded into the weights


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    L: int            # angular cutoff: l = 0..L-1  (L = L_max + 1)
    N: int            # radial functions per l
    R: float          # ball radius (bohr)
    n_r: int
    n_theta: int
    n_phi: int
    radial_rule: int
    k: int            # orbitals in the block
    n_check: int      # eigenpairs that must converge
    degree: int       # Chebyshev degree
    x0_seed: int
    geom_seed: int
    potential: str    # "harmonic" | "wells" | "wells+kb" | "zero"
    omega: float = 0.5
    max_iter: int = 60
    fixed_iter: int = 0   # >0: run exactly this many outer iterations

    @property
    def d(self) -> int:
        return self.L * self.L * self.N

    @property
    def n_grid(self) -> int:
        return self.n_r * self.n_theta * self.n_phi


# Harmonic oscillator in a ball: R=10, L_max=8, 12 radial/l, 24x18x36 grid.
C1 = Workload("ho_L9_N12", L=9, N=12, R=10.0, n_r=24, n_theta=18, n_phi=36,
              radial_rule=RADIAL_GAUSS_LEGENDRE, k=10, n_check=10, degree=12,
              x0_seed=0, geom_seed=0, potential="harmonic", omega=0.5,
              fixed_iter=30)
# 13-atom icosahedral cluster of Gaussian wells: R=14, L_max=30, 60 radial/l.
# n_check = the 26 bound (negative-energy) states; the next 12 states form a
# dense band of box states between 0.016 and 0.045 Ha that the block edge at
# k = 32 would cut, so they serve as the guard states.
C2 = Workload("ico13_L31_N60", L=31, N=60, R=14.0, n_r=90, n_theta=62,
              n_phi=124, radial_rule=RADIAL_GAUSS_JACOBI_R2, k=32, n_check=26,
              degree=16, x0_seed=0, geom_seed=1, potential="wells", max_iter=120)
# 147-atom Mackay icosahedron: R=24, L_max=60, 120 radial/l.
C3 = Workload("mackay147_L61_N120", L=61, N=120, R=24.0, n_r=180,
              n_theta=122, n_phi=244, radial_rule=RADIAL_GAUSS_JACOBI_R2,
              k=400, n_check=360, degree=20, x0_seed=0, geom_seed=2,
              potential="wells")
# 309-atom fcc cuboctahedron with Kleinman-Bylander projectors: R=30, L_max=80.
C4 = Workload("fcc309kb_L81_N150", L=81, N=150, R=30.0, n_r=225,
              n_theta=162, n_phi=324, radial_rule=RADIAL_GAUSS_JACOBI_R2,
              k=1000, n_check=900, degree=20, x0_seed=0, geom_seed=3,
              potential="wells+kb")

# Self-consistent clusters of 8-40 Gaussian-well atoms: R=16, L_max=24, 40
# radial/l, grid 60x50x100, degree 12.  k and n_check here are the largest
# block (40 occupied + 8 guards); each cluster uses its own (scf_occupation).
C5 = Workload("scf_L25_N40", L=25, N=40, R=16.0, n_r=60, n_theta=50, n_phi=100,
              radial_rule=RADIAL_GAUSS_JACOBI_R2, k=48, n_check=40, degree=12,
              x0_seed=0, geom_seed=0, potential="scf")

WORKLOADS = {w.name: w for w in (C1, C2, C3, C4, C5)}

# Gaussian-well model pseudopotential: V_j(r) = -2 exp(-r^2 / (2 * 1.2^2)) Ha.
WELL_DEPTH = 2.0
WELL_SIGMA = 1.2
JITTER_SIGMA = 0.1
# Kleinman-Bylander projectors: Gaussian radial form, width 1.0 bohr,
# channel energies h_0 = +1.5 Ha (l=0), h_1 = -0.8 Ha (l=1).
KB_WIDTH = 1.0
KB_ENERGY = {0: 1.5, 1: -0.8}


# SCF cluster model: each atom is a Gaussian well plus a Gaussian ion charge
# of +2 (width 1.2 bohr) carrying two valence electrons, so clusters are
# neutral; atoms uniform in a ball of radius 8 bohr, pairwise >= 2.5 bohr.
ION_CHARGE = 2.0
ION_SIGMA = 1.2
SCF_BALL = 8.0
SCF_MIN_SEP = 2.5
SCF_ATOMS = (8, 40)
TRAIN_SEED0 = 0          # training cluster i uses seed i
HELDOUT_SEED0 = 10000    # held-out cluster i uses seed 10000 + i


def small(L, N, R=10.0, n_r=None, n_theta=None, n_phi=None, k=4,
          rule=RADIAL_GAUSS_JACOBI_R2, potential="wells", degree=8,
          geom_seed=1, x0_seed=0, name=None) -> Workload:
    """A reduced workload with the same structure, for fast parity tests."""
    n_r = n_r if n_r is not None else (3 * N + 1) // 2
    n_theta = n_theta if n_theta is not None else 2 * L
    n_phi = n_phi if n_phi is not None else 4 * L
    return Workload(name or f"small_L{L}_N{N}", L=L, N=N, R=R, n_r=n_r,
                    n_theta=n_theta, n_phi=n_phi, radial_rule=rule, k=k,
                    n_check=max(1, k - max(2, math.ceil(0.1 * k))),
                    degree=degree, x0_seed=x0_seed, geom_seed=geom_seed,
                    potential=potential)


# ---------------------------------------------------------------- geometry

def _icosahedron_dirs() -> np.ndarray:
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1, s2 in itertools.product((-1.0, 1.0), repeat=2):
        v += [(0.0, s1, s2 * g), (s1, s2 * g, 0.0), (s2 * g, 0.0, s1)]
    v = np.array(v)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _icosahedron_faces(dirs: np.ndarray):
    # Faces = triples of mutually nearest vertices.
    dmin = min(np.linalg.norm(dirs[i] - dirs[j])
               for i in range(12) for j in range(i + 1, 12))
    adj = [[j for j in range(12) if j != i and
            abs(np.linalg.norm(dirs[i] - dirs[j]) - dmin) < 1e-9] for i in range(12)]
    faces = set()
    for i in range(12):
        for j in adj[i]:
            for kk in adj[j]:
                if kk in adj[i]:
                    faces.add(tuple(sorted((i, j, kk))))
    return sorted(faces)


def mackay_icosahedron(shells: int, spacing: float) -> np.ndarray:
    """Centre atom plus flat-faced icosahedral shells s=1..shells, vertex s at
    distance s*spacing; 1, 13, 55, 147, ... atoms."""
    dirs = _icosahedron_dirs()
    faces = _icosahedron_faces(dirs)
    pts = [np.zeros(3)]
    for s in range(1, shells + 1):
        shell = {}
        for (a, b, c) in faces:
            for i in range(s + 1):
                for j in range(s + 1 - i):
                    kk = s - i - j
                    p = spacing * (i * dirs[a] + j * dirs[b] + kk * dirs[c])
                    shell[tuple(np.round(p, 9))] = p
        pts += list(shell.values())
    return np.array(pts)


def fcc_cuboctahedron(shells: int, nn_dist: float) -> np.ndarray:
    """fcc cluster {|x|,|y|,|z| <= n, |x|+|y|+|z| <= 2n, x+y+z even} in units
    of a/2, with nearest-neighbour distance nn_dist; 13, 55, 147, 309 atoms."""
    h = nn_dist / math.sqrt(2.0)
    n = shells
    pts = [(x, y, z) for x in range(-n, n + 1) for y in range(-n, n + 1)
           for z in range(-n, n + 1)
           if (x + y + z) % 2 == 0 and abs(x) + abs(y) + abs(z) <= 2 * n]
    return h * np.array(pts, dtype=np.float64)


def atoms_for(w: Workload) -> np.ndarray:
    """Atom positions (bohr) for a workload, jittered N(0, 0.1^2) per coordinate."""
    if w.potential in ("harmonic", "zero"):
        return np.zeros((0, 3))
    if w.name.startswith("mackay147"):
        base = mackay_icosahedron(3, 4.5)
    elif w.name.startswith("fcc309"):
        base = fcc_cuboctahedron(4, 4.0)
    else:  # 13-atom icosahedron + centre (also used by reduced workloads)
        base = mackay_icosahedron(1, 4.5)
    rng = np.random.default_rng(w.geom_seed)
    return base + rng.normal(0.0, JITTER_SIGMA, size=base.shape)


# --------------------------------------------------------------- potentials

def spherical_to_cartesian(r, theta, phi):
    """Cartesian points for the tensor grid r x theta x phi, shape (n_r, n_t, n_p, 3)."""
    r = np.asarray(r)[:, None, None]
    st = np.sin(np.asarray(theta))[None, :, None]
    ct = np.cos(np.asarray(theta))[None, :, None]
    cp = np.cos(np.asarray(phi))[None, None, :]
    sp = np.sin(np.asarray(phi))[None, None, :]
    x = r * st * cp
    y = r * st * sp
    z = r * ct * np.ones_like(cp)
    return np.stack(np.broadcast_arrays(x, y, z), axis=-1)


def gaussian_wells(points: np.ndarray, atoms: np.ndarray,
                   depth: float = WELL_DEPTH, sigma: float = WELL_SIGMA) -> np.ndarray:
    """V(x) = sum_j -depth * exp(-|x - x_j|^2 / (2 sigma^2)) at the given points.
    Each well is evaluated where it exceeds depth * 1e-40 (|x - x_j| < 13.6
    sigma); beyond that its contribution is set to zero."""
    import torch   # multithreaded CPU elementwise work; float64 throughout
    shape = points.shape[:-1]
    p = torch.from_numpy(np.ascontiguousarray(points.reshape(-1, 3), dtype=np.float64))
    return gaussian_wells_torch(p, atoms, depth, sigma).numpy().reshape(shape)


def gaussian_wells_torch(p, atoms: np.ndarray, depth: float = WELL_DEPTH,
                         sigma: float = WELL_SIGMA):
    """gaussian_wells on a float64 torch tensor of points (n, 3), on the
    tensor's device; returns a float64 tensor (n,)."""
    import torch
    a = torch.from_numpy(np.ascontiguousarray(np.asarray(atoms, dtype=np.float64).reshape(-1, 3)))
    a = a.to(p.device)
    v = torch.zeros(p.shape[0], dtype=torch.float64, device=p.device)
    if a.shape[0] == 0:
        return v
    cut2 = 2.0 * sigma * sigma * 92.1   # exp(-92.1) = 1e-40
    chunk = max(1, int(2.0e8 // a.shape[0]))
    for s in range(0, p.shape[0], chunk):
        pc = p[s:s + chunk]
        d2 = ((pc[:, None, :] - a[None, :, :]) ** 2).sum(-1)
        e = torch.exp(-d2 / (2.0 * sigma * sigma))
        e = torch.where(d2 < cut2, e, torch.zeros_like(e))
        v[s:s + chunk] = -depth * e.sum(1)
    return v


def harmonic(points: np.ndarray, omega: float) -> np.ndarray:
    """V(x) = omega^2 |x|^2 / 2."""
    return 0.5 * omega * omega * np.sum(points ** 2, axis=-1)


def potential_on_grid(w: Workload, r, theta, phi) -> np.ndarray:
    """Model potential on the tensor grid, C-order [r][theta][phi]."""
    pts = spherical_to_cartesian(r, theta, phi)
    if w.potential == "zero":
        return np.zeros(pts.shape[:-1])
    if w.potential == "harmonic":
        return harmonic(pts, w.omega)
    return gaussian_wells(pts, atoms_for(w))


def kb_projector_values(points: np.ndarray, atoms: np.ndarray,
                        width: float = KB_WIDTH) -> tuple[np.ndarray, np.ndarray]:
    """Sample the atom-centred projectors p_{j,l,m}(x) = N_l rho^l
    exp(-rho^2 / (2 w^2)) S_lm(rho_hat), l = 0, 1 (S real harmonics), at the
    given points.  Returns (values [n_points, n_proj], energies [n_proj]).
    Projector order: atom-major, then (l=0), (l=1, m=-1, 0, 1).
    N_l normalises each projector over all of R^3."""
    p = points.reshape(-1, 3)
    cols, energies = [], []
    # int_0^inf r^{2l+2} exp(-r^2/w^2) dr = Gamma(l+3/2) w^{2l+3} / 2
    for a in atoms:
        rho = p - a
        rr = np.sqrt(np.sum(rho ** 2, axis=-1))
        g = np.exp(-rr ** 2 / (2.0 * width ** 2))
        n0 = 1.0 / math.sqrt(math.gamma(1.5) * width ** 3 / 2.0)
        cols.append(n0 * g / math.sqrt(4.0 * math.pi))
        energies.append(KB_ENERGY[0])
        n1 = 1.0 / math.sqrt(math.gamma(2.5) * width ** 5 / 2.0)
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        # real l=1 harmonics times rho:  m=-1 -> y, m=0 -> z, m=+1 -> x
        for comp in (1, 2, 0):
            cols.append(n1 * g * c1 * rho[:, comp])
            energies.append(KB_ENERGY[1])
    if not cols:
        return np.zeros((p.shape[0], 0)), np.zeros(0)
    return np.stack(cols, axis=1), np.array(energies)


def kb_projector_values_torch(p, atoms: np.ndarray, width: float = KB_WIDTH):
    """kb_projector_values on a float64 torch tensor of points (n, 3), on the
    tensor's device, transposed: returns (values [n_proj, n], energies
    [n_proj]) with the same projector order and normalisation."""
    import torch
    n0 = 1.0 / math.sqrt(math.gamma(1.5) * width ** 3 / 2.0) / math.sqrt(4.0 * math.pi)
    n1 = (1.0 / math.sqrt(math.gamma(2.5) * width ** 5 / 2.0)) * math.sqrt(3.0 / (4.0 * math.pi))
    out = torch.empty(4 * len(atoms), p.shape[0], dtype=torch.float64, device=p.device)
    energies = []
    for j, a in enumerate(np.asarray(atoms, dtype=np.float64)):
        rho = p - torch.from_numpy(a).to(p.device)
        g = torch.exp(-(rho * rho).sum(1) / (2.0 * width ** 2))
        out[4 * j] = n0 * g
        for c, comp in enumerate((1, 2, 0)):
            out[4 * j + 1 + c] = n1 * g * rho[:, comp]
        energies += [KB_ENERGY[0]] + [KB_ENERGY[1]] * 3
    return out, np.array(energies)


def x0_row_chunks(w: Workload, chunk: int):
    """The rows of x0_block(w).T (row i = column i of the start block) in
    consecutive chunks of at most `chunk` rows: the same draws in the same
    order, without holding the whole block."""
    rng = np.random.default_rng(w.x0_seed)
    for i0 in range(0, w.k, chunk):
        yield i0, rng.standard_normal((min(chunk, w.k - i0), w.d))


def x0_block(w: Workload, k: int | None = None, d: int | None = None,
             seed: int | None = None) -> np.ndarray:
    """Seeded N(0,1) start block, d x k, column-major (Fortran order);
    column i is draws [i*d, (i+1)*d) of the generator."""
    k = w.k if k is None else k
    d = w.d if d is None else d
    rng = np.random.default_rng(w.x0_seed if seed is None else seed)
    return np.asfortranarray(rng.standard_normal((k, d)).T)


def random_block(d: int, k: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) d x k block, Fortran order (for operator parity tests)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((k, d)).T)


def lanczos_start(d: int, seed: int = 12345) -> np.ndarray:
    """Seeded start vector for the upper-bound Lanczos run."""
    return np.random.default_rng(seed).standard_normal(d)


# ------------------------------------------------------------- SCF clusters

def scf_cluster(seed: int) -> np.ndarray:
    """n ~ U{8..40} atoms uniform in the radius-8 ball, rejection-sampled to a
    minimum pair separation of 2.5 bohr.  Returns (n, 3)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(SCF_ATOMS[0], SCF_ATOMS[1] + 1))
    pts: list[np.ndarray] = []
    while len(pts) < n:
        p = rng.uniform(-SCF_BALL, SCF_BALL, 3)
        if np.dot(p, p) > SCF_BALL * SCF_BALL:
            continue
        if pts and np.min(np.sum((np.asarray(pts) - p) ** 2, axis=1)) < SCF_MIN_SEP ** 2:
            continue
        pts.append(p)
    return np.asarray(pts)


def scf_occupation(n_atoms: int) -> tuple[int, int]:
    """(doubly occupied orbitals, guard states) for a neutral cluster."""
    return n_atoms, max(4, math.ceil(0.2 * n_atoms))


def ion_density(points: np.ndarray, atoms: np.ndarray, charge: float = ION_CHARGE,
                sigma: float = ION_SIGMA) -> np.ndarray:
    """Positive background: sum_j charge (2 pi sigma^2)^{-3/2}
    exp(-|x - x_j|^2 / (2 sigma^2)), evaluated like gaussian_wells."""
    depth = -charge * (2.0 * math.pi * sigma * sigma) ** -1.5
    return gaussian_wells(points, atoms, depth=depth, sigma=sigma)
