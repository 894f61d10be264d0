"""ces_apply_H_noalloc (the H*X entry point that allocates nothing and uses the
library's fixed per-GPU scratch array) against ces_apply_H with a caller
workspace: same kernels, so the same result, on two calls in a row with the
second block smaller, in both precisions, with and without projectors; and a
block too large for the fixed scratch is rejected before any launch."""
import numpy as np
import pytest

import synth_inputs as si

torch = pytest.importorskip("torch")
from paper_1404_3773_amd import ces  # noqa: E402

pytestmark = pytest.mark.gpu

FP64, MIXED = ces.CES_PREC_FP64, ces.CES_PREC_MIXED
TOL = {FP64: 1e-11, MIXED: 5e-5}     # the H*X parity bars of the oracle tests


def _say(msg):
    print(msg, flush=True)


def _ham(w, with_kb):
    B = ces.Basis.for_workload(w)
    r, wr, th, wt, ph = B.grid()
    V = torch.from_numpy(si.potential_on_grid(w, r, th, ph).reshape(-1)).cuda()
    P = h = None
    if with_kb:
        # projector coefficients: forward transform of the sampled projectors
        pts = si.spherical_to_cartesian(r, th, ph)
        pg, h = si.kb_projector_values(pts, si.atoms_for(w)[:2])
        f = torch.from_numpy(np.ascontiguousarray(pg.T)).cuda()
        H0 = ces.Ham(B, V)
        P = torch.empty(pg.shape[1], B.d, dtype=torch.float64, device="cuda")
        H0.from_grid(f, P, H0.workspace(pg.shape[1], FP64))
        torch.cuda.synchronize()
    return B, ces.Ham(B, V, proj=P, energies=h)


def _compare(B, H, k, seed, prec):
    X = torch.from_numpy(np.ascontiguousarray(si.random_block(B.d, k, seed).T)).cuda()
    ref = torch.empty_like(X)
    H.apply_H(X, ref, prec, H.workspace(k, prec))
    got = torch.full_like(X, float("nan"))
    H.apply_H_noalloc(X, got, prec)
    torch.cuda.synchronize()
    err = ((got - ref).abs().amax(dim=1) / ref.abs().amax(dim=1)).max().item()
    _say(f"  k={k} prec={prec}: max rel diff {err:.2e}")
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", [FP64, MIXED])
@pytest.mark.parametrize("case", ["ico13_k32_then_k5", "small_kb_k20_then_k3"])
def test_noalloc_apply_H_matches_workspace_entry(case, prec):
    _say(f"case noalloc {case} prec={prec}")
    if case.startswith("ico13"):
        B, H = _ham(si.C2, False)
        ks = (32, 5)
    else:
        B, H = _ham(si.small(6, 8, R=9.0, k=5), True)
        ks = (20, 3)
    _compare(B, H, ks[0], 31, prec)
    _compare(B, H, ks[1], 32, prec)      # second call, smaller block


def test_noalloc_rejects_a_block_beyond_its_scratch():
    B, H = _ham(si.C2, False)
    k = 400
    X = torch.zeros(k, B.d, dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(ces.CesError) as e:
        H.apply_H_noalloc(X, Y, FP64)
    assert e.value.status == 4 and "scratch" in str(e.value)
