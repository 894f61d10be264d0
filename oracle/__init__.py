"""FP64 CPU oracle for the spectral Kohn-Sham hot path (Banerjee, Elliott, James,
"A spectral scheme for Kohn-Sham density functional theory of clusters").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
anything in this package: only tests/, the smoke check in __graft_entry__ and
the cpu_baseline leg of bench.py use it.  It shares no code with the HIP
library; the only module both sides read is synth_inputs (seeded workloads,
no method arithmetic).

The oracle works in the paper's own complex basis F_lmn = R_ln(r) Y_l^m(theta,
phi) (Section 2.2.1, eqs. eigfunction_1 / spherical_bessel_1 /
spherical_harmonics_1) and converts to and from the real-harmonic coefficient
layout of the C interface with the unitary map in `basis.complex_to_real`.
Special functions come from SciPy, quadrature nodes from SciPy/NumPy.

Modules
  basis        Bessel zeros, radial functions, grids, harmonics, index map
  hamiltonian  dense H (definition) and the paper's separable H*X
  eigensolver  Chebyshev filter, Cholesky-QR, Rayleigh-Ritz, CheFSI driver
  density      electron density, Hartree potential (closed form), Slater exchange
  scf          Kohn-Sham potential, Anderson mixing, SAD start, SCF driver
  mlp          the learned start's descriptors, network, loss and Adam step

The tests in tests/test_oracle_*pins.py tie the oracle to things other than
itself: closed forms, analytic spectra, invariants, finite differences, an
independent radial solver, brute force on small cases.  Parity unpinned: the absolute eigenvalues
of the cluster workloads (the paper prints none for these synthetic clusters;
they rest on the operator pins and on oracle-GPU agreement), SCF iteration
counts, and the learned start's reduction of them (measured, not pinned).
"""
