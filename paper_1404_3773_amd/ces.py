"""Thin ctypes binding of libces (include/ces.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.

Block convention: a d x k column-major block with leading dimension ld is a
torch tensor of shape (k, ld) (row i = orbital i), float64, on the GPU.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libces.so")

CES_PREC_FP64 = 0
CES_PREC_MIXED = 1
CES_RADIAL_GAUSS_JACOBI_R2 = 0
CES_RADIAL_GAUSS_LEGENDRE = 1

EXPORTS = [
    "ces_basis_create", "ces_basis_create_ke", "ces_basis_radial_counts",
    "ces_basis_destroy", "ces_basis_info", "ces_basis_grid",
    "ces_basis_tables", "ces_ham_create", "ces_ham_set_veff", "ces_ham_destroy",
    "ces_workspace_size", "ces_apply_H", "ces_apply_H_noalloc", "ces_cheb_filter",
    "ces_rayleigh_ritz",
    "ces_lanczos_bound", "ces_chefsi", "ces_lobpcg_workspace_size", "ces_lobpcg",
    "ces_density", "ces_to_grid", "ces_from_grid",
    "ces_coeffs_complex_to_real", "ces_coeffs_real_to_complex", "ces_slater_x",
    "ces_pz_correlation", "ces_fermi_dirac", "ces_ham_set_model", "ces_ham_set_density_basis",
    "ces_ham_set_scf_eigensolver",
    "ces_hartree", "ces_ks_potential", "ces_anderson_workspace_size", "ces_anderson_mix",
    "ces_sad_density", "ces_scf_workspace_size", "ces_scf",
    "ces_atom_descriptors", "ces_density_fit_workspace_size", "ces_density_fit_gram",
    "ces_density_correction", "ces_mlp_create", "ces_mlp_destroy", "ces_mlp_num_params",
    "ces_mlp_get_params", "ces_mlp_set_params", "ces_mlp_get_grads", "ces_mlp_workspace_size",
    "ces_mlp_forward", "ces_mlp_backward", "ces_mlp_adam_step", "ces_cluster_quad_loss",
    "ces_profile_enable", "ces_profile_read", "ces_status_string", "ces_last_error",
]

_lib = None


class CesError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libces.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libces.so not built at {LIB_PATH}; run "
                          "`python -m paper_1404_3773_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                        ctypes.c_size_t)
    sig = {
        "ces_basis_create": [I, I, D, I, I, I, I, ctypes.POINTER(P)],
        "ces_basis_create_ke": [I, I, D, I, I, I, I, D, ctypes.POINTER(P)],
        "ces_basis_radial_counts": [P, P],
        "ces_basis_destroy": [P],
        "ces_basis_info": [P, ctypes.POINTER(I64), ctypes.POINTER(I64)],
        "ces_basis_grid": [P, P, P, P, P, P],
        "ces_basis_tables": [P, P, P, P],
        "ces_ham_create": [P, P, I, P, P, P, ctypes.POINTER(P)],
        "ces_ham_set_veff": [P, P, P],
        "ces_ham_destroy": [P],
        "ces_workspace_size": [P, I, I, ctypes.POINTER(SZ)],
        "ces_apply_H": [P, I, P, I64, P, I64, I, P, SZ, P],
        "ces_apply_H_noalloc": [P, I, P, I64, P, I64, I, P],
        "ces_cheb_filter": [P, I, P, I64, I, D, D, D, I, P, SZ, P],
        "ces_rayleigh_ritz": [P, I, P, I64, P, P, P, P, ctypes.POINTER(I), I, P, SZ, P],
        "ces_lanczos_bound": [P, P, I, ctypes.POINTER(D), P, SZ, P],
        "ces_chefsi": [P, I, P, I64, I, D, I, I, I, D, D, I, P, P, ctypes.POINTER(I), P, SZ, P],
        "ces_lobpcg_workspace_size": [P, I, I, I, ctypes.POINTER(SZ)],
        "ces_lobpcg": [P, I, P, I64, I, P, I64, I, I, D, D, I, I, P, P, ctypes.POINTER(I),
                       ctypes.POINTER(I), P, SZ, P],
        "ces_density": [P, I, P, I64, P, P, P, I, P, SZ, P],
        "ces_to_grid": [P, I, P, I64, P, P, SZ, P],
        "ces_from_grid": [P, I, P, P, I64, P, SZ, P],
        "ces_coeffs_complex_to_real": [P, I, P, I64, P, I64, P],
        "ces_coeffs_real_to_complex": [P, I, P, I64, P, I64, P],
        "ces_slater_x": [I64, P, P, P],
        "ces_pz_correlation": [I64, P, P, P, P],
        "ces_ham_set_model": [P, I, D, I],
        "ces_ham_set_density_basis": [P, P],
        "ces_ham_set_scf_eigensolver": [P, I, D, I],
        "ces_fermi_dirac": [I, P, D, D, P, ctypes.POINTER(D)],
        "ces_hartree": [P, P, P, P, SZ, P],
        "ces_ks_potential": [P, P, P, P, P, P, P, SZ, P],
        "ces_anderson_workspace_size": [I64, I, ctypes.POINTER(SZ)],
        "ces_anderson_mix": [I64, I, P, P, I64, I, D, P, P, P, SZ, P],
        "ces_sad_density": [P, I, P, P, P, P, SZ, P],
        "ces_scf_workspace_size": [P, I, I, I, ctypes.POINTER(SZ)],
        "ces_scf": [P, I, P, I64, I, P, P, P, P, I, D, I, D, I, I, I, P, P,
                    ctypes.POINTER(I), P, P, SZ, P],
        "ces_atom_descriptors": [I, P, P, P],
        "ces_density_fit_workspace_size": [P, I, ctypes.POINTER(SZ)],
        "ces_density_fit_gram": [P, I, P, P, P, P, P, SZ, P],
        "ces_density_correction": [P, I, P, P, P, P, P, SZ, P],
        "ces_mlp_create": [I, I, I, I, ctypes.c_uint64, ctypes.POINTER(P)],
        "ces_mlp_destroy": [P],
        "ces_mlp_num_params": [P, ctypes.POINTER(I64)],
        "ces_mlp_get_params": [P, P, P, P],
        "ces_mlp_set_params": [P, P, P, P],
        "ces_mlp_get_grads": [P, P],
        "ces_mlp_workspace_size": [P, I, ctypes.POINTER(SZ)],
        "ces_mlp_forward": [P, I, P, P, P, SZ, P],
        "ces_mlp_backward": [P, I, P, P, SZ, P],
        "ces_mlp_adam_step": [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              I, P],
        "ces_cluster_quad_loss": [I, I, P, P, P, P, P, P, P, P, ctypes.c_float, P],
        "ces_profile_enable": [I, I],
        "ces_profile_read": [I, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ces_status_string.argtypes = [ctypes.c_int]
    lib.ces_status_string.restype = ctypes.c_char_p
    lib.ces_last_error.argtypes = []
    lib.ces_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        lib = load()
        raise CesError(status, where, lib.ces_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ld(X):
    """Leading dimension of a (k, ld) block tensor."""
    assert X.dtype.is_floating_point and X.dim() == 2 and X.stride(1) == 1
    return X.stride(0)


_STAGE_NAMES = ("radial_inverse", "legendre_synth", "phi_stage", "legendre_analysis",
                "radial_forward", "kb_project", "kb_apply")
STAGES = tuple(f"{n}_fp32" for n in _STAGE_NAMES) + tuple(f"{n}_fp64" for n in _STAGE_NAMES)


def profile_enable(on: bool, max_records: int = 65536):
    _check(load().ces_profile_enable(1 if on else 0, int(max_records) if on else 0),
           "ces_profile_enable")


def profile_read():
    """{stage: (total_ms, launches)} since profile_enable."""
    n = len(STAGES)
    ms = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    _check(load().ces_profile_read(n, ms.ctypes.data_as(ctypes.c_void_p),
                                   cnt.ctypes.data_as(ctypes.c_void_p)), "ces_profile_read")
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def slater_x(rho, vx, stream=None):
    """vx = -(3 max(rho, 0) / pi)^(1/3) elementwise (contiguous float64 tensors)."""
    assert rho.dtype == vx.dtype and rho.is_contiguous() and vx.is_contiguous()
    assert rho.numel() == vx.numel()
    _check(load().ces_slater_x(rho.numel(), _ptr(rho), _ptr(vx), _stream(stream)),
           "ces_slater_x")


def pz_correlation(rho, vc, ec=None, stream=None):
    """vc <- Perdew-Zunger v_c(rho), ec <- eps_c(rho) when given (contiguous
    float64 tensors of equal length)."""
    assert rho.is_contiguous() and vc.is_contiguous() and rho.numel() == vc.numel()
    assert ec is None or (ec.is_contiguous() and ec.numel() == rho.numel())
    _check(load().ces_pz_correlation(rho.numel(), _ptr(rho), _ptr(vc), _ptr(ec),
                                     _stream(stream)), "ces_pz_correlation")


def fermi_dirac(eigs, n_electrons, kT):
    """Occupations f (numpy array) and Fermi level eF for the eigenvalues."""
    lam = np.ascontiguousarray(eigs, dtype=np.float64)
    f = np.zeros_like(lam)
    eF = ctypes.c_double()
    _check(load().ces_fermi_dirac(lam.size, lam.ctypes.data_as(ctypes.c_void_p),
                                  float(n_electrons), float(kT),
                                  f.ctypes.data_as(ctypes.c_void_p), ctypes.byref(eF)),
           "ces_fermi_dirac")
    return f, eF.value


def _ldc(Z):
    """Leading dimension (complex entries) of a (k, ld) complex128 block tensor."""
    import torch
    assert Z.dtype == torch.complex128 and Z.dim() == 2 and Z.stride(1) == 1
    return Z.stride(0)


def anderson_mix(V, F, oldest, beta, out, h_coef=None, stream=None):
    """V, F: (m, ld) float64 history tensors (row i = pair i); out: n values."""
    m, ld = V.shape
    n = out.numel()
    sz = ctypes.c_size_t()
    lib = load()
    _check(lib.ces_anderson_workspace_size(n, m, ctypes.byref(sz)), "ces_anderson_workspace_size")
    import torch
    work = torch.empty(sz.value, dtype=torch.uint8, device=V.device)
    coef = np.zeros(m)
    _check(lib.ces_anderson_mix(n, m, _ptr(V), _ptr(F), ld, int(oldest), float(beta), _ptr(out),
                                coef.ctypes.data_as(ctypes.c_void_p), _ptr(work), sz.value,
                                _stream(stream)), "ces_anderson_mix")
    return coef


MLP_FEATURES = 24
MLP_CHANNELS = 8


def _host3(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, 3))


def atom_descriptors(atoms):
    """(descriptors (n, 24) float32, unit environment directions (n, 3))."""
    a = _host3(atoms)
    desc = np.zeros((a.shape[0], MLP_FEATURES), dtype=np.float32)
    dirs = np.zeros((a.shape[0], 3))
    _check(load().ces_atom_descriptors(a.shape[0], a.ctypes.data_as(ctypes.c_void_p),
                                       desc.ctypes.data_as(ctypes.c_void_p),
                                       dirs.ctypes.data_as(ctypes.c_void_p)),
           "ces_atom_descriptors")
    return desc, dirs


def cluster_quad_loss(row_off, m_off, M, p, t, out, gout, loss, max_atoms, scale=1.0,
                      stream=None):
    _check(load().ces_cluster_quad_loss(int(loss.numel()), int(max_atoms), _ptr(row_off),
                                        _ptr(m_off), _ptr(M), _ptr(p), _ptr(t), _ptr(out),
                                        _ptr(gout), _ptr(loss), float(scale), _stream(stream)),
           "ces_cluster_quad_loss")


class MLP:
    """Handle of ces_mlp (per-atom network, FP32 on the device)."""

    def __init__(self, n_in=MLP_FEATURES, width=256, depth=3, n_out=MLP_CHANNELS, seed=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.ces_mlp_create(int(n_in), int(width), int(depth), int(n_out), int(seed),
                                  ctypes.byref(h)), "ces_mlp_create")
        self._h = h
        self.n_in, self.n_out = n_in, n_out
        self.sizes = [n_in] + [width] * depth + [n_out]
        n = ctypes.c_int64()
        _check(lib.ces_mlp_num_params(h, ctypes.byref(n)), "ces_mlp_num_params")
        self.n_params = n.value

    def get(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        mean = np.zeros(self.n_in, dtype=np.float32)
        std = np.zeros(self.n_in, dtype=np.float32)
        _check(load().ces_mlp_get_params(self._h, *[x.ctypes.data_as(ctypes.c_void_p)
                                                    for x in (p, mean, std)]),
               "ces_mlp_get_params")
        return p, mean, std

    def set(self, params=None, mean=None, std=None):
        args = []
        keep = []
        for x in (params, mean, std):
            if x is None:
                args.append(None)
            else:
                a = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))
                keep.append(a)
                args.append(a.ctypes.data_as(ctypes.c_void_p))
        _check(load().ces_mlp_set_params(self._h, *args), "ces_mlp_set_params")

    def grads(self):
        g = np.zeros(self.n_params, dtype=np.float32)
        _check(load().ces_mlp_get_grads(self._h, g.ctypes.data_as(ctypes.c_void_p)),
               "ces_mlp_get_grads")
        return g

    def workspace(self, rows):
        import torch
        sz = ctypes.c_size_t()
        _check(load().ces_mlp_workspace_size(self._h, int(rows), ctypes.byref(sz)),
               "ces_mlp_workspace_size")
        return torch.empty(sz.value, dtype=torch.uint8, device="cuda")

    def forward(self, X, out, work, stream=None):
        _check(load().ces_mlp_forward(self._h, X.shape[0], _ptr(X), _ptr(out), _ptr(work),
                                      work.numel(), _stream(stream)), "ces_mlp_forward")

    def backward(self, gout, work, stream=None):
        _check(load().ces_mlp_backward(self._h, gout.shape[0], _ptr(gout), _ptr(work),
                                       work.numel(), _stream(stream)), "ces_mlp_backward")

    def adam_step(self, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(load().ces_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2),
                                        float(eps), int(step), _stream(stream)),
               "ces_mlp_adam_step")

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ces_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Basis:
    """Handle of ces_basis (host tables; device upload on first Ham)."""

    def __init__(self, lmax, n_rad, R, n_r, n_theta, n_phi, rule=CES_RADIAL_GAUSS_JACOBI_R2,
                 e_cut=None):
        """e_cut (Hartree): keep only the radial functions with Lambda / 2 <=
        e_cut (the kinetic-energy-cutoff basis); None keeps all n_rad."""
        lib = load()
        h = ctypes.c_void_p()
        if e_cut is None:
            _check(lib.ces_basis_create(int(lmax), int(n_rad), float(R), int(n_r), int(n_theta),
                                        int(n_phi), int(rule), ctypes.byref(h)),
                   "ces_basis_create")
        else:
            _check(lib.ces_basis_create_ke(int(lmax), int(n_rad), float(R), int(n_r),
                                           int(n_theta), int(n_phi), int(rule), float(e_cut),
                                           ctypes.byref(h)), "ces_basis_create_ke")
        self._h = h
        self.L, self.N = lmax + 1, n_rad
        self.R = R
        self.n_r, self.n_theta, self.n_phi = n_r, n_theta, n_phi
        d, g = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.ces_basis_info(h, ctypes.byref(d), ctypes.byref(g)), "ces_basis_info")
        self.d, self.n_grid = d.value, g.value
        self.e_cut = e_cut
        self.Nl = self.radial_counts()

    @classmethod
    def for_workload(cls, w, e_cut=None):
        return cls(w.L - 1, w.N, w.R, w.n_r, w.n_theta, w.n_phi, w.radial_rule, e_cut=e_cut)

    def radial_counts(self):
        """N_l for each l (numpy int array)."""
        out = np.zeros(self.L, dtype=np.int32)
        _check(load().ces_basis_radial_counts(self._h, out.ctypes.data_as(ctypes.c_void_p)),
               "ces_basis_radial_counts")
        return out

    def grid(self):
        r, wr = np.zeros(self.n_r), np.zeros(self.n_r)
        th, wt = np.zeros(self.n_theta), np.zeros(self.n_theta)
        ph = np.zeros(self.n_phi)
        args = [a.ctypes.data_as(ctypes.c_void_p) for a in (r, wr, th, wt, ph)]
        _check(load().ces_basis_grid(self._h, *args), "ces_basis_grid")
        return r, wr, th, wt, ph

    def tables(self):
        z = np.zeros(self.L * self.N)
        rad = np.zeros(self.L * self.n_r * self.N)
        leg = np.zeros(self.n_theta * self.L * (self.L + 1) // 2)
        _check(load().ces_basis_tables(self._h, *[a.ctypes.data_as(ctypes.c_void_p)
                                                  for a in (z, rad, leg)]), "ces_basis_tables")
        return (z.reshape(self.L, self.N), rad.reshape(self.L, self.n_r, self.N),
                leg.reshape(self.n_theta, -1))

    def coeffs_complex_to_real(self, F, S, stream=None):
        """S <- real-basis coefficients of the complex-basis block F; both
        (k, ld) complex128 tensors on the GPU (row i = orbital i)."""
        _check(load().ces_coeffs_complex_to_real(self._h, F.shape[0], _ptr(F), _ldc(F), _ptr(S),
                                                 _ldc(S), _stream(stream)),
               "ces_coeffs_complex_to_real")

    def coeffs_real_to_complex(self, S, F, stream=None):
        """F <- complex-basis coefficients of the real-basis block S."""
        _check(load().ces_coeffs_real_to_complex(self._h, S.shape[0], _ptr(S), _ldc(S), _ptr(F),
                                                 _ldc(F), _stream(stream)),
               "ces_coeffs_real_to_complex")

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ces_basis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ham:
    """Handle of ces_ham: V_eff on the grid (torch float64, n_grid), optional
    projector coefficients (torch float64 of shape (n_proj, d)) and energies."""

    def __init__(self, basis: Basis, veff, proj=None, energies=None, stream=None):
        lib = load()
        self.basis = basis
        n_proj = 0 if proj is None else int(proj.shape[0])
        if proj is not None:
            assert proj.is_contiguous() and proj.shape[1] == basis.d
        e = None
        if n_proj:
            e = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
        h = ctypes.c_void_p()
        _check(lib.ces_ham_create(basis._h, _ptr(veff.contiguous()), n_proj, _ptr(proj),
                                  None if e is None else e.ctypes.data_as(ctypes.c_void_p),
                                  _stream(stream), ctypes.byref(h)), "ces_ham_create")
        self._h = h
        self.n_proj = n_proj

    def set_model(self, correlation=False, smearing_kT=0.0, mix_density=False):
        """SCF model options: Perdew-Zunger correlation in V_eff, Fermi-Dirac
        occupations at smearing_kT (Hartree; 0 = n_occ filled states), and
        Anderson mixing of the density instead of the potential."""
        _check(load().ces_ham_set_model(self._h, int(correlation), float(smearing_kT),
                                        int(mix_density)), "ces_ham_set_model")

    def set_scf_eigensolver(self, mode=0, res_tol=1e-6, max_iter=200):
        """ces_scf eigensolver: 0 CheFSI, 1 LOBPCG in the first step, 2 LOBPCG
        in every step."""
        _check(load().ces_ham_set_scf_eigensolver(self._h, int(mode), float(res_tol),
                                                  int(max_iter)), "ces_ham_set_scf_eigensolver")

    def set_density_basis(self, basis):
        """Expand the density for the Hartree potential in `basis` (a Basis on
        the same grid, typically lmax = 2 lmax of this one); None restores the
        orbitals' basis.  The handle keeps a reference to the basis."""
        _check(load().ces_ham_set_density_basis(self._h, None if basis is None else basis._h),
               "ces_ham_set_density_basis")
        self._rho_basis = basis

    def set_veff(self, veff, stream=None):
        _check(load().ces_ham_set_veff(self._h, _ptr(veff.contiguous()), _stream(stream)),
               "ces_ham_set_veff")

    def workspace_size(self, k, prec=CES_PREC_FP64) -> int:
        n = ctypes.c_size_t()
        _check(load().ces_workspace_size(self._h, int(k), int(prec), ctypes.byref(n)),
               "ces_workspace_size")
        return n.value

    def workspace(self, k, prec=CES_PREC_FP64):
        import torch
        n = self.workspace_size(k, prec)
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    def apply_H(self, X, Y, prec, work, stream=None):
        k = X.shape[0]
        _check(load().ces_apply_H(self._h, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y), int(prec),
                                  _ptr(work), work.numel(), _stream(stream)), "ces_apply_H")

    def apply_H_noalloc(self, X, Y, prec, stream=None):
        """Y = H X with the library's fixed scratch (no workspace argument)."""
        k = X.shape[0]
        _check(load().ces_apply_H_noalloc(self._h, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y),
                                          int(prec), _stream(stream)), "ces_apply_H_noalloc")

    def cheb_filter(self, X, degree, a, b, a0, prec, work, stream=None):
        _check(load().ces_cheb_filter(self._h, X.shape[0], _ptr(X), _ld(X), int(degree),
                                      float(a), float(b), float(a0), int(prec), _ptr(work),
                                      work.numel(), _stream(stream)), "ces_cheb_filter")

    def rayleigh_ritz(self, X, evals, res, work, HX=None, hx_prec=CES_PREC_FP64, stream=None,
                      return_path=False):
        """Returns the eigenvalues as a host array (copied in the call's own
        synchronisation); evals / res receive them on the device.  With
        return_path, returns (eigenvalues, path): 0 plain Cholesky-QR, 1 the
        shifted CholeskyQR3 fallback."""
        h = np.zeros(X.shape[0])
        path = ctypes.c_int(-1)
        _check(load().ces_rayleigh_ritz(self._h, X.shape[0], _ptr(X), _ld(X), _ptr(HX),
                                        _ptr(evals), _ptr(res), h.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(path), int(hx_prec), _ptr(work),
                                        work.numel(), _stream(stream)),
               "ces_rayleigh_ritz")
        return (h, path.value) if return_path else h

    def lanczos_bound(self, v0, work, steps=20, stream=None) -> float:
        out = ctypes.c_double()
        _check(load().ces_lanczos_bound(self._h, _ptr(v0), int(steps), ctypes.byref(out),
                                        _ptr(work), work.numel(), _stream(stream)),
               "ces_lanczos_bound")
        return out.value

    def chefsi(self, X, degree, b, n_check, evals, res, work, prec, max_iter=60,
               fixed_iter=0, res_tol=1e-4, dtheta_tol=1e-7, stream=None) -> int:
        it = ctypes.c_int()
        _check(load().ces_chefsi(self._h, X.shape[0], _ptr(X), _ld(X), int(degree), float(b),
                                 int(n_check), int(max_iter), int(fixed_iter), float(res_tol),
                                 float(dtheta_tol), int(prec), _ptr(evals), _ptr(res),
                                 ctypes.byref(it), _ptr(work), work.numel(), _stream(stream)),
               "ces_chefsi")
        return it.value

    def lobpcg_workspace(self, k, n_lock=0, prec=CES_PREC_FP64):
        import torch
        n = ctypes.c_size_t()
        _check(load().ces_lobpcg_workspace_size(self._h, int(k), int(n_lock), int(prec),
                                                ctypes.byref(n)), "ces_lobpcg_workspace_size")
        return torch.empty(n.value, dtype=torch.uint8, device="cuda")

    def lobpcg(self, X, evals, res, work, n_check=None, max_iter=200, res_tol=1e-6,
               g_scale=1.0, precondition=True, prec=CES_PREC_FP64, Y=None, stream=None):
        """Block LOBPCG in place on X ((k, ld) block); Y: (n_lock, ld) constraint
        block or None.  Returns (iterations, restarts)."""
        k = X.shape[0]
        it, rs = ctypes.c_int(), ctypes.c_int()
        n_lock = 0 if Y is None else Y.shape[0]
        _check(load().ces_lobpcg(self._h, k, _ptr(X), _ld(X), n_lock, _ptr(Y),
                                 _ld(Y) if Y is not None else 0,
                                 int(k if n_check is None else n_check), int(max_iter),
                                 float(res_tol), float(g_scale), 1 if precondition else 0,
                                 int(prec), _ptr(evals), _ptr(res), ctypes.byref(it),
                                 ctypes.byref(rs), _ptr(work), work.numel(), _stream(stream)),
               "ces_lobpcg")
        return it.value, rs.value

    def density(self, X, occ, rho_grid, rho_coef, prec, work, stream=None):
        _check(load().ces_density(self._h, X.shape[0], _ptr(X), _ld(X), _ptr(occ),
                                  _ptr(rho_grid), _ptr(rho_coef), int(prec), _ptr(work),
                                  work.numel(), _stream(stream)), "ces_density")

    def to_grid(self, X, f, work, stream=None):
        _check(load().ces_to_grid(self._h, X.shape[0], _ptr(X), _ld(X), _ptr(f), _ptr(work),
                                  work.numel(), _stream(stream)), "ces_to_grid")

    def from_grid(self, f, X, work, stream=None):
        _check(load().ces_from_grid(self._h, X.shape[0], _ptr(f), _ptr(X), _ld(X), _ptr(work),
                                    work.numel(), _stream(stream)), "ces_from_grid")

    # ------------------------------------------------------------ SCF extras
    # Grid arrays are flat torch float64 tensors of n_grid values.

    def hartree(self, tau, vh, work, stream=None):
        _check(load().ces_hartree(self._h, _ptr(tau), _ptr(vh), _ptr(work), work.numel(),
                                  _stream(stream)), "ces_hartree")

    def ks_potential(self, rho, rho_ion, vext, v, work, tau=None, stream=None):
        _check(load().ces_ks_potential(self._h, _ptr(rho), _ptr(rho_ion), _ptr(vext), _ptr(v),
                                       _ptr(tau), _ptr(work), work.numel(), _stream(stream)),
               "ces_ks_potential")

    def sad_density(self, atoms, tau00, rho, work, stream=None):
        a = np.ascontiguousarray(np.asarray(atoms, dtype=np.float64).reshape(-1, 3))
        t = np.ascontiguousarray(np.asarray(tau00, dtype=np.float64))
        assert t.shape == (int(self.basis.Nl[0]),)
        _check(load().ces_sad_density(self._h, a.shape[0], a.ctypes.data_as(ctypes.c_void_p),
                                      t.ctypes.data_as(ctypes.c_void_p), _ptr(rho), _ptr(work),
                                      work.numel(), _stream(stream)), "ces_sad_density")

    def scf_workspace(self, k, prec=CES_PREC_FP64, hist=20):
        import torch
        n = ctypes.c_size_t()
        _check(load().ces_scf_workspace_size(self._h, int(k), int(prec), int(hist),
                                             ctypes.byref(n)), "ces_scf_workspace_size")
        return torch.empty(n.value, dtype=torch.uint8, device="cuda")

    def scf(self, X, n_occ, vext, rho_ion, rho0, v0, evals, rho, work, degree=12, beta=0.2,
            hist=20, tol=1e-6, max_steps=60, first_iters=12, prec=CES_PREC_FP64, stream=None):
        """Returns (steps, per-step max |delta theta_occ|)."""
        steps = ctypes.c_int()
        dth = np.zeros(int(max_steps))
        _check(load().ces_scf(self._h, X.shape[0], _ptr(X), _ld(X), int(n_occ), _ptr(vext),
                              _ptr(rho_ion), _ptr(rho0), _ptr(v0), int(degree), float(beta),
                              int(hist), float(tol), int(max_steps), int(first_iters), int(prec),
                              _ptr(evals), _ptr(rho), ctypes.byref(steps),
                              dth.ctypes.data_as(ctypes.c_void_p), _ptr(work), work.numel(),
                              _stream(stream)), "ces_scf")
        return steps.value, dth[:steps.value].copy()

    # ---------------------------------------------------------- learned start

    def density_fit_gram(self, atoms, dirs, target, stream=None):
        """(8n+1)^2 FP64 Gram of sqrt(W) [Phi | target] (torch, column-major)."""
        import torch
        a = _host3(atoms)
        u = _host3(dirs)
        n = a.shape[0]
        sz = ctypes.c_size_t()
        _check(load().ces_density_fit_workspace_size(self._h, n, ctypes.byref(sz)),
               "ces_density_fit_workspace_size")
        work = torch.empty(sz.value, dtype=torch.uint8, device="cuda")
        nc = MLP_CHANNELS * n + 1
        gram = torch.empty((nc, nc), dtype=torch.float64, device="cuda")
        _check(load().ces_density_fit_gram(self._h, n, a.ctypes.data_as(ctypes.c_void_p),
                                           u.ctypes.data_as(ctypes.c_void_p), _ptr(target),
                                           _ptr(gram), _ptr(work), sz.value, _stream(stream)),
               "ces_density_fit_gram")
        return gram

    def density_correction(self, atoms, dirs, coef, rho, stream=None):
        import torch
        a = _host3(atoms)
        u = _host3(dirs)
        work = torch.empty(48 * a.shape[0], dtype=torch.uint8, device="cuda")
        _check(load().ces_density_correction(self._h, a.shape[0], a.ctypes.data_as(ctypes.c_void_p),
                                             u.ctypes.data_as(ctypes.c_void_p), _ptr(coef),
                                             _ptr(rho), _ptr(work), work.numel(),
                                             _stream(stream)), "ces_density_correction")

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ces_ham_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
