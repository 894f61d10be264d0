"""Write the stored expected eigenvalues used by the GPU tests.

Calls only the oracle (oracle/) and the seeded inputs (synth_inputs).  Run:
    python tests/golden/make_golden.py ico13      (13-atom cluster, L_max=30)
    python tests/golden/make_golden.py scf        (SCF of held-out cluster 0, L_max=24)
Output: tests/golden/<workload>_eigenvalues.txt, tests/golden/scf_L25_N40_heldout0.txt
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402
from oracle import basis as ob  # noqa: E402
from oracle import density as od  # noqa: E402
from oracle import scf as osf  # noqa: E402
from oracle import eigensolver as oe  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402


def converge(w, k, degree, res_tol=1e-8, dtheta_tol=1e-12, max_iter=400):
    """Oracle CheFSI with its own block size and degree (any convergent run
    gives the same lowest eigenvalues of H)."""
    bs = ob.basis_for(w)
    V = si.potential_on_grid(w, bs.r, bs.theta, bs.phi)
    app = lambda Y: oh.apply_H_real(bs, V, Y)  # noqa: E731
    b = oe.lanczos_upper_bound(app, si.lanczos_start(bs.d))
    X0 = si.x0_block(w, k=k)
    t0 = time.time()

    def log(it, theta, res):
        print(f"it {it:3d}  t={time.time() - t0:7.1f}s  max_res[:n_check]="
              f"{np.max(res[:w.n_check]):.3e}  theta0={theta[0]:.12f}", flush=True)

    theta, X, res, it = oe.chefsi(app, X0, degree, b, w.n_check, max_iter=max_iter,
                                  res_tol=res_tol, dtheta_tol=dtheta_tol, log=log)
    return b, theta, res, it


# seeds of the random start blocks of the SCF runs (GPU tests use the same)
SCF_ATOM_X0_SEED = 501
SCF_X0_SEED = 502


def scf_golden():
    """Oracle SCF of the cluster model on the full SCF basis: the single atom
    (for the SAD start), then held-out cluster 0 from SAD, both to
    max |delta theta_occ| < 1e-10."""
    w = si.C5
    bs = ob.basis_for(w)
    pts = si.spherical_to_cartesian(bs.r, bs.theta, bs.phi)
    v0 = si.lanczos_start(bs.d)
    t0 = time.time()
    zeta = od.zeta_table(bs)
    print(f"zeta table {time.time() - t0:.1f}s", flush=True)

    def log(tag):
        return lambda s, th: print(f"{tag} step {s:3d} t={time.time() - t0:7.1f}s "
                                   f"theta0={th[0]:.12f}", flush=True)

    a1 = np.zeros((1, 3))
    rion1 = si.ion_density(pts, a1)
    scf1 = osf.ClusterSCF(bs, a1, si.gaussian_wells(pts, a1), rion1, 1, 4, degree=w.degree,
                          zeta=zeta)
    th1, st1, rho1, _ = scf1.run(rion1, si.random_block(bs.d, 5, SCF_ATOM_X0_SEED), v0=v0,
                                 tol=1e-10, max_steps=100, log=log("atom"))
    tau00 = od.density_coefficients(bs, rho1)[:bs.N]
    atoms = si.scf_cluster(si.HELDOUT_SEED0)
    n_occ, n_guard = si.scf_occupation(len(atoms))
    rion = si.ion_density(pts, atoms)
    scf = osf.ClusterSCF(bs, atoms, si.gaussian_wells(pts, atoms), rion, n_occ, n_guard,
                         degree=w.degree, zeta=zeta)
    rho0 = osf.sad_density(bs, tau00, atoms)
    th, st, rho, _ = scf.run(rho0, si.random_block(bs.d, n_occ + n_guard, SCF_X0_SEED), v0=v0,
                             tol=1e-10, max_steps=100, log=log("cluster"))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{w.name}_heldout0.txt")
    with open(out, "w") as f:
        f.write(f"# SCF of the cluster model on workload {w.name} (synth_inputs): FP64 oracle,\n"
                f"# Anderson beta 0.2, history 20, degree {w.degree}, converged to max\n"
                f"# |delta theta_occ| < 1e-10.  Written by tests/golden/make_golden.py.\n"
                f"# atom: single atom at the origin ({st1} steps); cluster: held-out cluster 0\n"
                f"# (seed {si.HELDOUT_SEED0}, {len(atoms)} atoms, {n_occ} occupied, SAD start,"
                f" {st} steps)\n# columns: system index eigenvalue\n")
        for i in range(5):
            f.write(f"atom {i} {th1[i]:.15f}\n")
        for i in range(n_occ + n_guard):
            f.write(f"cluster {i} {th[i]:.15f}\n")
    print("wrote", out)


def main(which):
    if which == "scf":
        return scf_golden()
    if which == "ico13":
        w = si.C2
    else:
        raise SystemExit(f"unknown workload {which}")
    k, degree = 40, 20
    b, theta, res, it = converge(w, k, degree)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"{w.name}_eigenvalues.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest eigenvalues (Ha) of the quadrature Hamiltonian for workload "
                f"{w.name}\n# (synth_inputs), from the FP64 oracle's Chebyshev-filtered "
                f"subspace iteration\n# run to max residual <= 1e-8 (block {k}, degree "
                f"{degree}, {it} iterations,\n# Lanczos bound b={b:.10f}).  Written by "
                f"tests/golden/make_golden.py.\n# columns: index eigenvalue residual\n")
        for i in range(w.n_check):
            f.write(f"{i} {theta[i]:.15f} {res[i]:.3e}\n")
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "ico13")
