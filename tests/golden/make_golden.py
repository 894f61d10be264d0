"""Write the stored expected eigenvalues used by the GPU tests.

Calls only the oracle (oracle/) and the seeded inputs (synth_inputs).  Run:
    python tests/golden/make_golden.py ico13      (13-atom cluster, L_max=30)
Output: tests/golden/<workload>_eigenvalues.txt
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402
from oracle import basis as ob  # noqa: E402
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


def main(which):
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
