"""Benchmark of the Chebyshev-filtered subspace iteration hot path on one GPU.

Headline workload: the 309-atom fcc cuboctahedron of Gaussian wells with
Kleinman-Bylander projectors (l = 0, 1; 1236 projectors), R = 30 bohr,
L_max = 80, 150 radial functions per l (d = 984,150), grid 225 x 162 x 324,
1000 orbitals, Chebyshev degree 20: the largest configuration, synthetic and
seeded.  V_eff and the projectors are sampled on the device by the seeded
input generators; the projector coefficients come from the library's forward
transform.

A timed step is one outer CheFSI iteration in mixed precision: the degree-20
FP32 filter (20 H*X), then FP64 Cholesky-QR + Rayleigh-Ritz (one FP64 H*X)
and residuals, with the filter bounds taken from the previous Rayleigh-Ritz.
`value` is the algorithmic H*X flop rate of the whole step:
(degree + 1) * F / step_time, with F the separable method's algorithmic
flops per H*X (phi stage counted at nominal real-FFT cost, both projector
products at 2 d n_proj k each).

Also reported: the same workload's mixed and FP64 H*X per stage, and, on the
13-atom and 147-atom workloads, H*X rates, time to eigenpairs (13-atom: all
n_check eigenvalues within 1e-6 Ha of the stored oracle values; 147-atom:
mixed against the FP64 GPU run), the density call and the pointwise
exchange-correlation kernels; the roofline of the dominant kernel measured
with HIP events over further steps (kept out of the step time), and the CPU
oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402

PEAK_FP32 = 157.3e12   # MI355X FP32: vector (256 CUs x 2.4 GHz) = dense matrix, FLOP/s
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12      # B/s
PMC_COPY_BYTES = 1 << 30      # calibration copy of --pmc-run (read and written once)
# kernel name prefix (as rocprofv3 reports it) of each H*X stage's FP32 launch
# FP32 kernels of each H*X stage (name prefixes; the Legendre stages run the
# theta-folded kernels for L > 32)
STAGE_KERNEL = {"radial_inverse": ("k_radial_inverse_mfma<float",),
                "legendre_synth": ("k_legendre_synth<float", "k_legendre_synth_fold<float"),
                "phi_stage": ("k_phi_stage<float",),
                "legendre_analysis": ("k_legendre_analysis<float",
                                      "k_legendre_analysis_fold<float"),
                "radial_forward": ("k_radial_forward_mfma<float",),
                "kb_project": ("k_kb_gemm<float",), "kb_apply": ("k_kb_apply_wide<", "k_kb_apply<float")}


def algorithmic_flops(w, k, n_proj=0):
    """Algorithmic flops of one H*X for k orbitals (separable method):
    radial sums both ways, Legendre sums both ways with even/odd folding,
    phi synthesis + analysis at nominal real-FFT cost 2.5 N log2 N each,
    pointwise V, kinetic term, and the two projector products (2 d n_proj k
    each)."""
    L2 = w.L * w.L
    radial = 2 * (2 * w.n_r * w.N * L2) * k
    legendre = 2 * (w.n_r * w.n_theta * L2) * k
    fft = 2 * w.n_r * w.n_theta * k * 2.5 * w.n_phi * math.log2(w.n_phi)
    pointwise = w.n_grid * k
    kinetic = 2 * w.d * k
    kb = 2 * (2 * w.d * n_proj * k)
    return {"radial": radial, "legendre": legendre, "phi": fft, "pointwise": pointwise,
            "kinetic": kinetic, "kb": kb,
            "total": radial + legendre + fft + pointwise + kinetic + kb}


def stage_flops(w, k, n_proj=0):
    """Algorithmic flops of one launch of each H*X stage (same accounting as
    algorithmic_flops, split by stage; kb_gemm is both projector products)."""
    f = algorithmic_flops(w, k, n_proj)
    return {"radial_inverse": f["radial"] / 2,
            "legendre_synth": f["legendre"] / 2,
            "phi_stage": f["phi"] + f["pointwise"],
            "legendre_analysis": f["legendre"] / 2,
            "radial_forward": f["radial"] / 2 + f["kinetic"],
            "kb_project": f["kb"] / 2,
            "kb_apply": f["kb"] / 2}


def stage_bytes(w, k, n_proj, elem):
    """Algorithmic HBM bytes of one launch of each H*X stage (element size
    elem): each stage reads its input block once and writes its output once
    (the small basis tables are cache-resident); the phi stage also reads V's
    halved Fourier sums; the projector products read P (d x n_proj) once."""
    L2, S = w.L * w.L, 2 * w.L - 1
    G = w.n_r * L2 * k                      # G or A
    g = w.n_r * w.n_theta * S * k           # angular intermediate
    return {"radial_inverse": elem * (w.d * k + G),
            "legendre_synth": elem * (G + g),
            "phi_stage": elem * (2 * g + 2 * w.n_r * w.n_theta * S),
            "legendre_analysis": elem * (g + G),
            "radial_forward": elem * (G + 3 * w.d * k + (w.d * k if n_proj else 0)),
            "kb_project": elem * (w.d * n_proj + w.d * k),
            "kb_apply": elem * (w.d * n_proj + w.d * k)}


def density_rates(ces, torch, H, w, X, work_mixed, reps=10):
    """ces_density on the benchmark workload: rho on the grid for all k
    orbitals (occupations 1) and its coefficients tau, mixed and FP64.
    Algorithmic flops: the inverse radial and Legendre sums and the phi
    synthesis at real-FFT cost (half of an H*X's), plus the square, weight and
    add per grid point and orbital; algorithmic bytes: read X (FP64), write
    rho, read rho and write tau.  Also the mixed rho's error against FP64."""
    k = X.shape[0]
    f = algorithmic_flops(w, k)
    flops = f["radial"] / 2 + f["legendre"] / 2 + f["phi"] / 2 + 3 * w.n_grid * k
    nbytes = 8 * (w.d * k + 2 * w.n_grid + w.d)
    occ = torch.ones(k, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "orbitals": k, "with_coefficients": True,
           "alg_flop": flops, "alg_bytes": nbytes}
    rho = {}
    for name, prec in (("mixed", ces.CES_PREC_MIXED), ("fp64", ces.CES_PREC_FP64)):
        work = work_mixed if prec == ces.CES_PREC_MIXED else H.workspace(k, prec)
        r = torch.empty(w.n_grid, dtype=torch.float64, device="cuda")
        tau = torch.empty(w.d, dtype=torch.float64, device="cuda")
        H.density(X, occ, r, tau, prec, work)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            H.density(X, occ, r, tau, prec, work)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        rho[name] = r
        peak = PEAK_FP32 if name == "mixed" else PEAK_FP64
        out[name] = {"ms": round(sec * 1e3, 4), "tflops": round(flops / sec / 1e12, 3),
                     "frac_mfma_peak": round(flops / sec / peak, 4),
                     "alg_GBps": round(nbytes / sec / 1e9, 1),
                     "frac_hbm_peak": round(nbytes / sec / PEAK_HBM, 4)}
    out["mixed_rho_rel_err_vs_fp64"] = float(
        (rho["mixed"] - rho["fp64"]).abs().max() / rho["fp64"].abs().max())
    print(f"[bench] density (k={k}, with tau): mixed {out['mixed']['ms']} ms, "
          f"fp64 {out['fp64']['ms']} ms", file=sys.stderr, flush=True)
    return out


def pointwise_rates(ces, torch, n=1 << 26, reps=10):
    """The grid-pointwise exchange-correlation kernels on n points (about a
    147-atom grid's worth times 10): Perdew-Zunger correlation (rho in, v_c
    and eps_c out: 24 B per point) and Slater exchange (16 B per point), as
    HBM bandwidth against the peak.  Kernels run on torch's current stream,
    timed with its events."""
    rho = torch.rand(n, dtype=torch.float64, device="cuda")
    vc, ec = torch.empty_like(rho), torch.empty_like(rho)
    out = {}
    for name, call, nbytes in (("pz_correlation", lambda: ces.pz_correlation(rho, vc, ec), 24),
                               ("slater_x", lambda: ces.slater_x(rho, vc), 16)):
        call()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            call()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        gbs = nbytes * n / (ms * 1e-3) / 1e9
        out[name] = {"points": n, "ms": round(ms, 4), "GBps": round(gbs, 1),
                     "hbm_frac": round(gbs * 1e9 / PEAK_HBM, 4)}
        print(f"[bench] {name}: {ms:.3f} ms for {n} points, {gbs:.0f} GB/s",
              file=sys.stderr, flush=True)
    del rho, vc, ec
    torch.cuda.empty_cache()
    return out


def measured_traffic(kernel_prefixes, workload):
    """(HBM bytes per launch, kernel name, summary file, counter row) of the
    kernel whose name starts with one of kernel_prefixes on `workload`, from
    a committed FETCH_SIZE / WRITE_SIZE summary (profiles/*_pmc.json); None
    if there is none or it was taken on other kernel sources."""
    import glob
    from paper_1404_3773_amd import pmc_summary
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.json"))):
        with open(path) as f:
            pmc = json.load(f)
        if pmc.get("workload") != workload:
            continue
        for row in pmc.get("kernels", []):
            if row["kernel"].startswith(tuple(kernel_prefixes)) and "traffic_bytes" in row:
                if pmc_summary.source_digest(pmc["sources"]) != pmc["source_sha256"]:
                    return None
                return row["traffic_bytes"], row["kernel"], os.path.relpath(path, ROOT), row
    return None


def x0_on_device(torch, w):
    """The seeded start block of workload w as a (k, d) float64 device tensor,
    streamed to the device in row chunks (row i = column i of the block)."""
    X = torch.empty(w.k, w.d, dtype=torch.float64, device="cuda")
    for i0, rows in si.x0_row_chunks(w, 64):
        X[i0:i0 + rows.shape[0]] = torch.from_numpy(rows).cuda()
    return X


def kb_hamiltonian(ces, torch, w, B, atoms_per_chunk=16):
    """Hamiltonian of a wells + projectors workload: V_eff and the projector
    functions sampled on the grid by the seeded generators (on the device),
    projector coefficients by the library's forward transform in chunks of
    atoms.  Returns (H, n_proj, V, seconds)."""
    t0 = time.perf_counter()
    r, wr, th, wt, ph = B.grid()
    pts = torch.from_numpy(si.spherical_to_cartesian(r, th, ph).reshape(-1, 3)).cuda()
    atoms = si.atoms_for(w)
    V = si.gaussian_wells_torch(pts, atoms)
    H0 = ces.Ham(B, V)
    n_proj = 4 * len(atoms)
    P = torch.empty(n_proj, B.d, dtype=torch.float64, device="cuda")
    energies = []
    work = H0.workspace(4 * atoms_per_chunk, ces.CES_PREC_FP64)
    for a0 in range(0, len(atoms), atoms_per_chunk):
        vals, e = si.kb_projector_values_torch(pts, atoms[a0:a0 + atoms_per_chunk])
        H0.from_grid(vals, P[4 * a0:4 * a0 + vals.shape[0]], work)
        energies.append(e)
        del vals
    torch.cuda.synchronize()
    del work, H0, pts
    H = ces.Ham(B, V, P, np.concatenate(energies))
    del P
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return H, n_proj, V, time.perf_counter() - t0


def pmc_run(workload):
    """Short run for the counter passes: on one workload (the 309-atom one by
    default, or the 147-atom one) two mixed and one FP64 H*X of its orbital
    block, and a plain elementwise copy of PMC_COPY_BYTES (read and written
    once) that calibrates the byte counters."""
    import torch
    from paper_1404_3773_amd import ces
    ws = {w.name: w for w in (si.C4, si.C3)}
    if workload not in ws:
        raise SystemExit(f"--pmc-workload: one of {sorted(ws)}")
    for w in (ws[workload],):
        B = ces.Basis.for_workload(w)
        if w.potential == "wells+kb":
            H, n_proj, V, _ = kb_hamiltonian(ces, torch, w, B)
            del V
        else:
            H = ces.Ham(B, wells_on_device(torch, B, w))
        X = x0_on_device(torch, w)
        Y = torch.empty_like(X)
        print(f"[bench] pmc run: {w.name} setup done", flush=True)
        for prec, reps in ((ces.CES_PREC_MIXED, 2), (ces.CES_PREC_FP64, 1)):
            work = H.workspace(w.k, prec)
            for _ in range(reps):
                H.apply_H(X, Y, prec, work)
            torch.cuda.synchronize()
            del work
            torch.cuda.empty_cache()
            print(f"[bench] pmc run: {w.name} {reps} H*X prec={prec}", flush=True)
        del X, Y, H
        torch.cuda.empty_cache()
    src = torch.ones(PMC_COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"[bench] pmc run done: 3 copies of {PMC_COPY_BYTES} bytes", flush=True)


def wells_on_device(torch, B, w):
    """The workload's Gaussian-well V_eff on the basis grid, evaluated on the
    device by the seeded generator (float64, flat [r][theta][phi])."""
    r, wr, th, wt, ph = B.grid()
    pts = torch.from_numpy(si.spherical_to_cartesian(r, th, ph).reshape(-1, 3)).cuda()
    return si.gaussian_wells_torch(pts, si.atoms_for(w))


def stage_rates(prof, sf, peak, prec_suffix):
    """Per-stage average launch time and algorithmic rate from ces profiling."""
    out = {}
    for st, (ms, c) in prof.items():
        if c and st.endswith(prec_suffix) and sf.get(st[:-5], 0) > 0:
            rate = sf[st[:-5]] / (ms / c * 1e-3)
            out[st[:-5]] = {"ms": round(ms / c, 4), "launches": c,
                            "tflops": round(rate / 1e12, 2), "frac_peak": round(rate / peak, 4)}
    return out


def large_workload_rates(ces, torch, reps=5):
    """H*X on the 147-atom workload (L_max = 60, N = 120, 180 x 122 x 244 grid,
    k = 400) in mixed and FP64: algorithmic TFLOP/s per H*X and per stage, and
    each stage's fraction of the FP32 / FP64 peak."""
    w = si.C3
    B = ces.Basis.for_workload(w)
    H = ces.Ham(B, wells_on_device(torch, B, w))
    F = algorithmic_flops(w, w.k)["total"]
    sf = stage_flops(w, w.k)
    out = {"workload": w.name, "d": w.d, "orbitals": w.k, "alg_flop_per_HX": F}
    for name, prec, peak in (("mixed", ces.CES_PREC_MIXED, PEAK_FP32),
                             ("fp64", ces.CES_PREC_FP64, PEAK_FP64)):
        work = H.workspace(w.k, prec)
        X = torch.from_numpy(np.ascontiguousarray(si.random_block(B.d, w.k, 3).T)).cuda()
        Y = torch.empty_like(X)
        H.apply_H(X, Y, prec, work)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            H.apply_H(X, Y, prec, work)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        ces.profile_enable(True, 4096)      # stage durations over a second pass
        for _ in range(reps):
            H.apply_H(X, Y, prec, work)
        torch.cuda.synchronize()
        prof = ces.profile_read()
        ces.profile_enable(False)
        suffix = "_fp32" if name == "mixed" else "_fp64"
        stages = {}
        for st, (ms, c) in prof.items():
            if c and st.endswith(suffix) and sf[st[:-5]] > 0:
                rate = sf[st[:-5]] / (ms / c * 1e-3)
                stages[st[:-5]] = {"ms": round(ms / c, 4), "tflops": round(rate / 1e12, 2),
                                   "frac_peak": round(rate / peak, 4)}
        out[name] = {"ms_per_HX": round(sec * 1e3, 4), "tflops": round(F / sec / 1e12, 3),
                     "stages": stages}
        del work, X, Y
        torch.cuda.empty_cache()
    print(f"[bench] 147-atom H*X: mixed {out['mixed']['ms_per_HX']} ms, "
          f"fp64 {out['fp64']['ms_per_HX']} ms", file=sys.stderr, flush=True)
    return out


def large_time_to_eigenpairs(ces, torch):
    """Time to eigenpairs on the 147-atom workload (k = 400, n_check = 360,
    degree 20) from the seeded random block, mixed and FP64, with the same
    convergence test as the 13-atom run.  The CPU oracle would need hours at
    this size, so the reference is the FP64 GPU run (its H*X matches the
    oracle at this full size to 6e-15 relative); reported: seconds,
    iterations and the mixed run's largest eigenvalue difference from it."""
    w = si.C3
    B = ces.Basis.for_workload(w)
    H = ces.Ham(B, wells_on_device(torch, B, w))
    X0 = x0_on_device(torch, w)
    k = X0.shape[0]
    v0 = torch.from_numpy(si.lanczos_start(B.d)).cuda()
    ev = torch.empty(k, dtype=torch.float64, device="cuda")
    rs = torch.empty(k, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "orbitals": k, "n_check": w.n_check, "degree": w.degree,
           "reference": "FP64 GPU run (CPU oracle infeasible at this size); the absolute "
                        "eigenvalues at this size are parity-unpinned: the FP64 H*X matches "
                        "the oracle at this full size, the eigenvalues are not run there"}
    theta = {}
    for name, prec in (("fp64", ces.CES_PREC_FP64), ("mixed", ces.CES_PREC_MIXED)):
        work = H.workspace(k, prec)
        X = X0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        b = H.lanczos_bound(v0, work)
        it = H.chefsi(X, w.degree, b, w.n_check, ev, rs, work, prec, max_iter=w.max_iter)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        theta[name] = ev.cpu().numpy()[:w.n_check].copy()
        out[name] = {"seconds": round(sec, 3), "iterations": it,
                     "converged": it < w.max_iter}
        print(f"[bench] 147-atom time-to-eigenpairs {name}: {sec:.2f} s, {it} it",
              file=sys.stderr, flush=True)
        del work, X
        torch.cuda.empty_cache()
    out["max_eig_diff_mixed_vs_fp64_Ha"] = float(np.max(np.abs(theta["mixed"] - theta["fp64"])))
    return out


def c4_time_to_eigenpairs(ces, torch, max_iter=200):
    """Time to eigenpairs on the 309-atom workload (k = 1000, n_check = 900,
    degree 20, 1236 projectors) from the seeded start block, FP64 and mixed:
    the Lanczos bound, a Rayleigh-Ritz of the start block, then filter +
    Rayleigh-Ritz steps until the n_check lowest pairs meet res <= 1e-4
    max(1, |theta|) and |delta theta| < 1e-7 (the test of ces_chefsi, run
    step by step here so that every few steps report progress; about 1.5 and
    1 minute).  The reference is the FP64 run (the CPU oracle cannot run this
    size)."""
    w = si.C4
    B = ces.Basis.for_workload(w)
    H, n_proj, V, setup_s = kb_hamiltonian(ces, torch, w, B)
    del V
    X0 = x0_on_device(torch, w)
    k, nc = X0.shape[0], w.n_check
    v0 = torch.from_numpy(si.lanczos_start(B.d)).cuda()
    ev = torch.empty(k, dtype=torch.float64, device="cuda")
    rs = torch.empty(k, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "orbitals": k, "n_check": nc, "degree": w.degree,
           "projectors": n_proj, "setup_seconds": round(setup_s, 1)}
    theta_end = {}
    for name, prec in (("fp64", ces.CES_PREC_FP64), ("mixed", ces.CES_PREC_MIXED)):
        work = H.workspace(k, prec)
        X = X0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        b = H.lanczos_bound(v0, work)
        theta = H.rayleigh_ritz(X, ev, rs, work)
        it, done = 0, False
        while not done and it < max_iter:
            it += 1
            a0 = theta[0] if theta[0] < theta[-1] else theta[-1] - 1e-6 * max(1.0, abs(theta[-1]))
            H.cheb_filter(X, w.degree, theta[-1], b, a0, prec, work)
            old = theta
            theta = H.rayleigh_ritz(X, ev, rs, work)
            res = rs.cpu().numpy()
            done = bool(np.all(res[:nc] <= 1e-4 * np.maximum(1.0, np.abs(theta[:nc])))
                        and np.all(np.abs(theta[:nc] - old[:nc]) < 1e-7))
            if it % 5 == 0 or done:
                print(f"[bench] 309-atom eigenpairs {name}: step {it}, "
                      f"{time.perf_counter() - t:.1f} s, max res {float(res[:nc].max()):.2e}",
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        theta_end[name] = np.array(theta[:nc])
        out[name] = {"seconds": round(sec, 2), "iterations": it, "converged": done}
        del work, X
        torch.cuda.empty_cache()
    out["max_eig_diff_mixed_vs_fp64_Ha"] = float(np.max(np.abs(theta_end["mixed"] -
                                                               theta_end["fp64"])))
    out["mixed_speedup"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    return out


def golden_eigenvalues(w):
    path = os.path.join(ROOT, "tests", "golden", f"{w.name}_eigenvalues.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, comments="#")[:, 1]


def cpu_baseline(w, V_grid, budget_s=20.0):
    """The FP64 oracle's H*X on the host cores, on a bounded sample of the
    headline workload: single columns of its start block through the oracle's
    transforms, V_eff and kinetic term (the projector term left out, and out
    of the flop count) until ~budget_s of work.  V_grid: the workload's V_eff
    on the grid (host array from the seeded generator)."""
    from oracle import basis as ob
    from oracle import hamiltonian as oh
    blas, threads = "unknown", os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = ", ".join(sorted({f"{p.get('internal_api')} {p.get('version')}" for p in info
                                 if p.get("user_api") == "blas"})) or "unknown"
        threads = max((p.get("num_threads", 1) for p in info), default=threads)
    except Exception:
        pass
    t0 = time.perf_counter()
    bs = ob.basis_for(w)
    setup_s = time.perf_counter() - t0
    V = V_grid.reshape(w.n_r, w.n_theta, w.n_phi)
    F1 = algorithmic_flops(w, 1)["total"]
    n = 0
    t0 = time.perf_counter()
    for _, rows in si.x0_row_chunks(w, 1):
        oh.apply_H_real(bs, V, rows.T)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    dt = time.perf_counter() - t0
    try:
        ncpu = len(os.sched_getaffinity(0))
    except Exception:
        ncpu = os.cpu_count()
    return {"value": round(F1 * n / dt / 1e9, 4), "unit": "GFLOP/s", "cores": int(threads),
            "kind": "oracle", "nproc": ncpu, "blas": blas,
            "sample": f"{n} single-column FP64 oracle H*X on the {w.name} basis and grid "
                      f"(columns 0..{n - 1} of the start block; transforms, V_eff and kinetic "
                      f"term; projector term excluded from work and count), {dt:.1f} s after "
                      f"{setup_s:.1f} s of oracle table setup"}


def headline_c4(ces, torch, args):
    """The 309-atom workload: timed mixed CheFSI steps, then per-stage HIP-event
    timings over further steps, and single H*X rates per precision."""
    w = si.C4
    FP64, MIXED = ces.CES_PREC_FP64, ces.CES_PREC_MIXED
    print(f"[bench] workload {w.name}: d={w.d} grid={w.n_r}x{w.n_theta}x{w.n_phi} k={w.k} "
          f"degree={w.degree}", file=sys.stderr, flush=True)
    B = ces.Basis.for_workload(w)
    H, n_proj, V, setup_s = kb_hamiltonian(ces, torch, w, B)
    X = x0_on_device(torch, w)
    print(f"[bench] setup: {setup_s:.1f} s ({n_proj} projectors)", file=sys.stderr, flush=True)
    work = H.workspace(w.k, MIXED)
    v0 = torch.from_numpy(si.lanczos_start(B.d)).cuda()
    b = H.lanczos_bound(v0, work)
    ev = torch.empty(w.k, dtype=torch.float64, device="cuda")
    rs = torch.empty(w.k, dtype=torch.float64, device="cuda")
    F = algorithmic_flops(w, w.k, n_proj)["total"]
    theta = H.rayleigh_ritz(X, ev, rs, work)

    def step():
        nonlocal theta
        H.cheb_filter(X, w.degree, theta[-1], b, theta[0], MIXED, work)
        theta = H.rayleigh_ritz(X, ev, rs, work)   # synchronises

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps, {dt / args.steps * 1e3:.1f} ms/step",
          file=sys.stderr, flush=True)
    # per-kernel durations: HIP events around every launch on the library's
    # stream, over further steps (kept out of the step timing)
    ces.profile_enable(True, 65536)
    for _ in range(args.prof_steps):
        step()
    torch.cuda.synchronize()
    prof = ces.profile_read()
    ces.profile_enable(False)
    res_max = float(rs[:w.n_check].max())
    # single H*X per precision (mixed: FP32 transforms and projector products)
    hx = {}
    Y = torch.empty_like(X)
    for name, prec, peak in (("mixed", MIXED, PEAK_FP32), ("fp64", FP64, PEAK_FP64)):
        wk = work if prec == MIXED else H.workspace(w.k, prec)
        H.apply_H(X, Y, prec, wk)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            H.apply_H(X, Y, prec, wk)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / 3
        ces.profile_enable(True, 1024)
        H.apply_H(X, Y, prec, wk)
        torch.cuda.synchronize()
        p1 = ces.profile_read()
        ces.profile_enable(False)
        hx[name] = {"ms_per_HX": round(sec * 1e3, 2), "tflops": round(F / sec / 1e12, 3),
                    "frac_peak": round(F / sec / peak, 4),
                    "stages": stage_rates(p1, stage_flops(w, w.k, n_proj), peak,
                                          "_fp32" if name == "mixed" else "_fp64")}
        if prec != MIXED:
            del wk
        torch.cuda.empty_cache()
    print(f"[bench] {w.name} H*X: mixed {hx['mixed']['ms_per_HX']} ms, "
          f"fp64 {hx['fp64']['ms_per_HX']} ms", file=sys.stderr, flush=True)
    out = {"w": w, "n_proj": n_proj, "F": F, "dt": dt, "prof": prof, "hx": hx,
           "setup_s": setup_s, "res_max_after_steps": res_max,
           "theta_range": [float(theta[0]), float(theta[-1])], "bound": b}
    V_host = V.cpu().numpy()
    del work, X, Y, H, V
    torch.cuda.empty_cache()
    return out, V_host


def ke_cutoff_c4(ces, torch, uniform_hx, reps=3):
    """The 309-atom workload in the kinetic-energy-cutoff basis (the
    non-uniform basis of the footnote in Section 2.2.1) at E_cut =
    Lambda_{0,N-1} / 2, the kinetic energy of the uniform basis's last l = 0
    function: each l keeps the functions below that energy.  Mixed and FP64
    H*X of the 1000-orbital block (seeded random coefficients) with the same
    projectors and V_eff, against the uniform basis's times."""
    w = si.C4
    z = ces.Basis.for_workload(w).tables()[0]
    e_cut = 0.5 * (z[0, w.N - 1] / w.R) ** 2
    B = ces.Basis.for_workload(w, e_cut=e_cut)
    H, n_proj, V, setup_s = kb_hamiltonian(ces, torch, w, B)
    del V
    g = torch.Generator(device="cuda")
    g.manual_seed(20140314)
    X = torch.randn(w.k, B.d, dtype=torch.float64, device="cuda", generator=g)
    Y = torch.empty_like(X)
    out = {"e_cut_Ha": round(e_cut, 4), "d": B.d, "d_uniform": w.d,
           "radial_per_l_first_last": [int(B.Nl[0]), int(B.Nl[-1])],
           "setup_seconds": round(setup_s, 1)}
    for name, prec in (("mixed", ces.CES_PREC_MIXED), ("fp64", ces.CES_PREC_FP64)):
        work = H.workspace(w.k, prec)
        H.apply_H(X, Y, prec, work)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            H.apply_H(X, Y, prec, work)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / reps * 1e3
        out[name] = {"ms_per_HX": round(ms, 2),
                     "speedup_vs_uniform": round(uniform_hx[name]["ms_per_HX"] / ms, 3)}
        del work
        torch.cuda.empty_cache()
    print(f"[bench] {w.name} cutoff basis d={B.d}: mixed {out['mixed']['ms_per_HX']} ms, "
          f"fp64 {out['fp64']['ms_per_HX']} ms", file=sys.stderr, flush=True)
    del X, Y, H
    torch.cuda.empty_cache()
    return out


def ico13_extras(ces, torch, args):
    """The 13-atom workload: timed mixed CheFSI steps, filter rates, density,
    and time to eigenpairs against the stored oracle eigenvalues."""
    w = si.C2
    k = w.k
    FP64, MIXED = ces.CES_PREC_FP64, ces.CES_PREC_MIXED
    B = ces.Basis.for_workload(w)
    r, wr, th, wt, ph = B.grid()
    H = ces.Ham(B, torch.from_numpy(si.potential_on_grid(w, r, th, ph).reshape(-1)).cuda())
    work = H.workspace(k, MIXED)
    X0 = torch.from_numpy(np.ascontiguousarray(si.x0_block(w).T)).cuda()
    v0 = torch.from_numpy(si.lanczos_start(B.d)).cuda()
    b = H.lanczos_bound(v0, work)
    ev = torch.empty(k, dtype=torch.float64, device="cuda")
    rs = torch.empty(k, dtype=torch.float64, device="cuda")
    F = algorithmic_flops(w, k)["total"]
    X = X0.clone()
    theta = H.rayleigh_ritz(X, ev, rs, work)

    def step():
        nonlocal theta
        H.cheb_filter(X, w.degree, theta[-1], b, theta[0], MIXED, work)
        theta = H.rayleigh_ritz(X, ev, rs, work)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    n = 20
    t0 = time.perf_counter()
    for _ in range(n):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ces.profile_enable(True, 65536)
    for _ in range(n):
        step()
    torch.cuda.synchronize()
    prof = ces.profile_read()
    ces.profile_enable(False)

    def filter_rate(prec, reps=10):
        Yf = X.clone()
        H.cheb_filter(Yf, w.degree, theta[-1], b, theta[0], prec, work)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            H.cheb_filter(Yf, w.degree, theta[-1], b, theta[0], prec, work)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / reps
        return w.degree * F / sec / 1e9, sec * 1e3

    gf_mixed, ms_f_mixed = filter_rate(MIXED)
    gf_fp64, ms_f_fp64 = filter_rate(FP64)
    out = {"workload": w.name, "d": w.d, "orbitals": k, "degree": w.degree,
           "step_gflops": round((w.degree + 1) * F / (dt / n) / 1e9, 3),
           "ms_per_step": round(dt / n * 1e3, 4),
           "filter_gflops": {"mixed": round(gf_mixed, 3), "fp64": round(gf_fp64, 3),
                             "mixed_ms": round(ms_f_mixed, 4), "fp64_ms": round(ms_f_fp64, 4)},
           "stages_fp32": stage_rates(prof, stage_flops(w, k), PEAK_FP32, "_fp32")}
    out["density"] = density_rates(ces, torch, H, w, X0, work)
    if not args.no_tte:
        tte = {}
        ref = golden_eigenvalues(w)
        for name, prec in (("mixed", MIXED), ("fp64", FP64)):
            Xs = X0.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            bb = H.lanczos_bound(v0, work)
            it = H.chefsi(Xs, w.degree, bb, w.n_check, ev, rs, work, prec, max_iter=w.max_iter)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            e = ev.cpu().numpy()[:w.n_check]
            err = float(np.max(np.abs(e - ref))) if ref is not None else None
            tte[name] = {"seconds": round(sec, 4), "iterations": it,
                         "max_eig_err_vs_oracle_Ha": err,
                         "within_1e-6Ha": (err is not None and err < 1e-6)}
            print(f"[bench] 13-atom time-to-eigenpairs {name}: {sec:.3f} s, {it} it, err={err}",
                  file=sys.stderr, flush=True)
        out["time_to_eigenpairs"] = tte
        # LOBPCG with the TPA preconditioner (Section 3.1) from the same start
        # block, to residuals 1e-5 relative: the same eigenvalue accuracy
        lob = {}
        for name, prec in (("mixed", MIXED), ("fp64", FP64)):
            lw = H.lobpcg_workspace(k, 0, prec)
            Xs = X0.clone()
            H.lobpcg(Xs, ev, rs, lw, n_check=w.n_check, res_tol=1e-5, prec=prec, max_iter=2)
            Xs = X0.clone()      # after a two-iteration warm-up of the solver's libraries
            torch.cuda.synchronize()
            t = time.perf_counter()
            it, rst = H.lobpcg(Xs, ev, rs, lw, n_check=w.n_check, res_tol=1e-5, prec=prec,
                               max_iter=500)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            e = ev.cpu().numpy()[:w.n_check]
            err = float(np.max(np.abs(e - ref))) if ref is not None else None
            lob[name] = {"seconds": round(sec, 4), "iterations": it, "restarts": rst,
                         "max_eig_err_vs_oracle_Ha": err,
                         "within_1e-6Ha": (err is not None and err < 1e-6),
                         "seconds_over_chefsi": round(sec / tte[name]["seconds"], 3)}
            print(f"[bench] 13-atom LOBPCG {name}: {sec:.3f} s, {it} it, err={err}",
                  file=sys.stderr, flush=True)
            del lw
        out["lobpcg_time_to_eigenpairs"] = lob
    del work, X, X0, H
    torch.cuda.empty_cache()
    return out


def scf_eigensolver_ratio(ces, torch, tol=1e-8):
    """Per-SCF-step time with the Chebyshev filter (one filter and one
    Rayleigh-Ritz per step) against LOBPCG in every step (Sections 3.1, 3.2),
    on the SCF workload's first held-out cluster from the ion-density start,
    FP64, both converged to max |delta theta_occ| < tol; LOBPCG solves each
    step to residuals tol / 10."""
    w = si.C5
    FP64 = ces.CES_PREC_FP64
    B = ces.Basis.for_workload(w)
    r, wr, th, wt, ph = B.grid()
    pts = si.spherical_to_cartesian(r, th, ph)
    atoms = si.scf_cluster(si.HELDOUT_SEED0)
    n_occ, n_guard = si.scf_occupation(len(atoms))
    k = n_occ + n_guard

    def cuda(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()

    H = ces.Ham(B, torch.zeros(B.n_grid, dtype=torch.float64, device="cuda"))
    vext, rion = cuda(si.gaussian_wells(pts, atoms)), cuda(si.ion_density(pts, atoms))
    v0 = cuda(si.lanczos_start(B.d))
    out = {"workload": w.name, "atoms": len(atoms), "orbitals": k, "scf_tol_Ha": tol}
    evs = {}
    for name, mode in (("chefsi", 0), ("lobpcg", 2)):
        H.set_scf_eigensolver(mode, res_tol=tol / 10, max_iter=500)
        work = H.scf_workspace(k, FP64)
        X = torch.from_numpy(np.ascontiguousarray(si.random_block(B.d, k, 502).T)).cuda()
        ev = torch.empty(k, dtype=torch.float64, device="cuda")
        rho = torch.empty(B.n_grid, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        steps, dth = H.scf(X, n_occ, vext, rion, rion, v0, ev, rho, work, degree=w.degree,
                           tol=tol, max_steps=100, prec=FP64)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        evs[name] = ev.cpu().numpy()[:n_occ]
        out[name] = {"seconds": round(sec, 3), "scf_steps": steps,
                     "ms_per_scf_step": round(sec / max(steps, 1) * 1e3, 3),
                     "converged": bool(len(dth) and dth[-1] < tol)}
        del work, X
    H.set_scf_eigensolver(0)
    out["lobpcg_over_chefsi_per_scf_step"] = round(
        out["lobpcg"]["ms_per_scf_step"] / out["chefsi"]["ms_per_scf_step"], 2)
    out["max_occupied_eig_diff_Ha"] = float(np.max(np.abs(evs["chefsi"] - evs["lobpcg"])))
    print(f"[bench] SCF {w.name}: CheFSI {out['chefsi']['ms_per_scf_step']} ms/step "
          f"({out['chefsi']['scf_steps']} steps), LOBPCG {out['lobpcg']['ms_per_scf_step']} "
          f"ms/step ({out['lobpcg']['scf_steps']} steps)", file=sys.stderr, flush=True)
    del H
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prof-steps", type=int, default=2,
                    help="further steps timed per kernel with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tte", action="store_true",
                    help="skip the 147- and 309-atom time-to-eigenpairs runs")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no 13-atom / 147-atom extras)")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for rocprofv3 counter passes (no JSON line)")
    ap.add_argument("--c4-tte", action="store_true",
                    help="only the 309-atom time to eigenpairs, mixed and FP64 (minutes)")
    ap.add_argument("--pmc-workload", default=si.C4.name,
                    help="workload of --pmc-run (fcc309kb_L81_N150 or mackay147_L61_N120)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    if args.pmc_run:
        pmc_run(args.pmc_workload)
        return

    import torch
    from paper_1404_3773_amd import ces

    if args.c4_tte:
        print(json.dumps({"fcc309_time_to_eigenpairs": c4_time_to_eigenpairs(ces, torch)}),
              flush=True)
        return
    hd, V_host = headline_c4(ces, torch, args)
    w, F, prof, n_proj = hd["w"], hd["F"], hd["prof"], hd["n_proj"]
    ms_step = hd["dt"] / args.steps * 1e3
    value = (w.degree + 1) * F / (hd["dt"] / args.steps) / 1e9

    # ---- roofline of the dominant kernel: the FP32 launch class with the
    # largest total time over the profiled steps
    fp32 = [st for st in prof if st.endswith("_fp32") and prof[st][1]]
    dom = max(fp32, key=lambda st: prof[st][0])
    tot_ms, launches = prof[dom]
    avg_ms = tot_ms / launches
    stage = dom[:-5]
    alg = stage_flops(w, w.k, n_proj)[stage]
    alg_b = stage_bytes(w, w.k, n_proj, 4)[stage]
    achieved = alg / (avg_ms * 1e-3)
    tr = measured_traffic(STAGE_KERNEL[stage], w.name)
    # every H*X stage runs its contraction on FP32 MFMA (the phi stage as an
    # exact Toeplitz + Hankel product, credited at real-FFT flops only)
    roof = {"bound": "mfma", "achieved": round(achieved / 1e12, 3),
            "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32, 4),
            "traffic": None if tr is None else round(tr[0]),
            "kernel": tr[1] if tr else STAGE_KERNEL[stage][0], "stage": dom,
            "avg_launch_ms": round(avg_ms, 4), "launches": launches,
            "alg_flop_per_launch": alg, "alg_bytes_per_launch": alg_b,
            "kernel_timing": f"HIP events around each launch over {args.prof_steps} further "
                             "steps of the same workload (kept out of the step timing)"}
    if tr is not None:
        roof["traffic_source"] = tr[2]
        roof["hbm_GBps_measured"] = round(tr[0] / (avg_ms * 1e-3) / 1e9, 1)
        row = tr[3]
        if "mfma_busy_frac" in row:
            roof["mfma_busy_frac_counters"] = round(row["mfma_busy_frac"], 4)
        if "mfma_flop_f32" in row:
            # MFMA work the kernel executes (counters) over its launch time
            roof["mfma_executed_tflops"] = round(row["mfma_flop_f32"] / (avg_ms * 1e-3) / 1e12, 2)
    gemm_frac = {st: v["frac_peak"] for st, v in
                 stage_rates(prof, stage_flops(w, w.k, n_proj), PEAK_FP32, "_fp32").items()}
    # counter-based MFMA utilisation of each FP32 stage kernel (committed
    # rocprofv3 summary of the same workload), beside the algorithmic fractions
    busy = {}
    for st, prefixes in STAGE_KERNEL.items():
        t = measured_traffic(prefixes, w.name)
        if t is not None and "mfma_busy_frac" in t[3]:
            busy[st] = round(t[3]["mfma_busy_frac"], 4)

    line = {
        "metric": "Chebyshev-filter H*X GFLOP/s & time-to-eigenpairs@1e-6Ha: mixed vs FP64",
        "value": round(value, 3), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "atoms": 309, "projectors": n_proj, "R_bohr": w.R,
                   "L_max": w.L - 1, "radial_per_l": w.N, "d": w.d,
                   "grid": [w.n_r, w.n_theta, w.n_phi], "orbitals": w.k, "degree": w.degree,
                   "step": "mixed degree-20 filter + FP64 Cholesky-QR/Rayleigh-Ritz"},
        "setup_seconds": round(hd["setup_s"], 1),
        "HX": hd["hx"],
        "mixed_vs_fp64_HX_speedup": round(hd["hx"]["fp64"]["ms_per_HX"] /
                                          hd["hx"]["mixed"]["ms_per_HX"], 3),
        "stage_frac_fp32_peak": gemm_frac,
        "stage_mfma_busy_counters": busy or None,
        "roofline": roof,
        "after_steps": {"max_residual_first_n_check": hd["res_max_after_steps"],
                        "ritz_range_Ha": hd["theta_range"], "upper_bound_Ha": hd["bound"]},
    }
    if not args.no_extras:
        line["fcc309_ke_cutoff_HX"] = ke_cutoff_c4(ces, torch, hd["hx"])
        line["ico13"] = ico13_extras(ces, torch, args)
        line["xc_pointwise"] = pointwise_rates(ces, torch)
        line["scf_eigensolver_per_step"] = scf_eigensolver_ratio(ces, torch)
        line["mackay147_HX"] = large_workload_rates(ces, torch)
        torch.cuda.empty_cache()
        if not args.no_tte:
            line["mackay147_time_to_eigenpairs"] = large_time_to_eigenpairs(ces, torch)
            torch.cuda.empty_cache()
            line["fcc309_time_to_eigenpairs"] = c4_time_to_eigenpairs(ces, torch)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, V_host)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
