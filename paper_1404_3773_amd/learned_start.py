"""Training and use of the learned start density of the SCF.

Every numerical step runs in libces (SCF, SAD, correction functions and
their Gram matrix, the network's forward / backward / Adam, the batched
loss); this module sequences the calls and moves arrays.

  generate  SCF from the superposition-of-atomic-densities (SAD) start for
            seeded clusters; keeps per cluster the atoms, the SCF step count
            and the terms p, t of the quadratic density loss against the
            converged density (the matrix M depends on geometry only and is
            recomputed when training).
  train     fits the per-atom network to those clusters with Adam.
  evaluate  runs the SCF from SAD and from the learned start on held-out
            clusters, both to |delta theta| < 1e-8: step counts (also at
            1e-6), converged-eigenvalue differences and the start density's
            error relative to SAD's.

  python -m paper_1404_3773_amd.learned_start generate --first 0 --count 1000 --out a.npz
  python -m paper_1404_3773_amd.learned_start train --data a.npz b.npz --out w.npz
  python -m paper_1404_3773_amd.learned_start evaluate --weights w.npz --first 10000 \\
      --count 200 --out eval.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth_inputs as si  # noqa: E402
from paper_1404_3773_amd import ces  # noqa: E402

ATOM_X0_SEED = 501
X0_SEED = 502
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                               f"learned_start_{si.C5.name}.npz")


def _say(msg):
    print(msg, flush=True)


class Context:
    """Basis, Hamiltonian handle and the single-atom density of the SCF
    workload; the atom's l = 0 density coefficients come from a GPU SCF."""

    def __init__(self, w=si.C5, prec=ces.CES_PREC_FP64, tol=1e-6, max_steps=100):
        import torch
        self.torch = torch
        self.w, self.prec, self.tol, self.max_steps = w, prec, tol, max_steps
        self.B = ces.Basis.for_workload(w)
        r, _, th, _, ph = self.B.grid()
        self.pts = si.spherical_to_cartesian(r, th, ph)
        self.H = ces.Ham(self.B, torch.zeros(self.B.n_grid, dtype=torch.float64, device="cuda"))
        self.work = self.H.workspace(1)
        self.v0 = self._dev(si.lanczos_start(self.B.d))
        self._scf_work = {}
        a1 = np.zeros((1, 3))
        _, self.atom_steps, _, rho1 = self.scf(a1, None, ATOM_X0_SEED, n_occ=1, n_guard=4)
        coef = torch.empty((1, self.B.d), dtype=torch.float64, device="cuda")
        self.H.from_grid(rho1, coef, self.work)
        self.tau00 = coef.cpu().numpy()[0, :int(self.B.Nl[0])].copy()

    def _dev(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()

    def fields(self, atoms):
        return (self._dev(si.gaussian_wells(self.pts, atoms)),
                self._dev(si.ion_density(self.pts, atoms)))

    def sad(self, atoms):
        rho = self.torch.empty(self.B.n_grid, dtype=self.torch.float64, device="cuda")
        self.H.sad_density(atoms, self.tau00, rho, self.work)
        return rho

    def scf(self, atoms, rho0, x0_seed=X0_SEED, n_occ=None, n_guard=None, fields=None):
        """SCF from rho0 (the ion density when None): (eigenvalues, steps, dtheta, rho)."""
        torch = self.torch
        if n_occ is None:
            n_occ, n_guard = si.scf_occupation(len(atoms))
        k = n_occ + n_guard
        vext, rion = self.fields(atoms) if fields is None else fields
        if k not in self._scf_work:
            self._scf_work[k] = self.H.scf_workspace(k, self.prec)
        X = torch.from_numpy(np.ascontiguousarray(si.random_block(self.B.d, k, x0_seed).T)).cuda()
        ev = torch.empty(k, dtype=torch.float64, device="cuda")
        rho = torch.empty(self.B.n_grid, dtype=torch.float64, device="cuda")
        steps, dth = self.H.scf(X, n_occ, vext, rion, rion if rho0 is None else rho0, self.v0, ev,
                                rho, self._scf_work[k], degree=self.w.degree, tol=self.tol,
                                max_steps=self.max_steps, prec=self.prec)
        return ev.cpu().numpy(), steps, dth, rho

    def loss_terms(self, atoms, dirs, target):
        """(M (8n x 8n), p (8n), t) of || sum c Phi - target ||_W^2."""
        G = self.H.density_fit_gram(atoms, dirs, target).cpu().numpy()
        nq = G.shape[0] - 1
        return G[:nq, :nq], G[:nq, nq], float(G[nq, nq])


# ---------------------------------------------------------------- generate

def generate(first, count, out, log_every=25):
    ctx = Context()
    _say(f"single atom: {ctx.atom_steps} SCF steps")
    rec = {k: [] for k in ("seed", "n", "atoms", "p", "t", "steps", "eig", "last_dtheta")}
    t0 = time.time()
    for s in range(first, first + count):
        atoms = si.scf_cluster(s)
        n_occ, _ = si.scf_occupation(len(atoms))
        _, dirs = ces.atom_descriptors(atoms)
        fields = ctx.fields(atoms)
        rho_sad = ctx.sad(atoms)
        ev, steps, dth, rho = ctx.scf(atoms, rho_sad, fields=fields)
        _, p, t = ctx.loss_terms(atoms, dirs, rho - rho_sad)
        rec["seed"].append(s)
        rec["n"].append(len(atoms))
        rec["atoms"].append(atoms.reshape(-1))
        rec["p"].append(p)
        rec["t"].append(t)
        rec["steps"].append(steps)
        rec["eig"].append(ev[:n_occ])
        rec["last_dtheta"].append(dth[-1])
        if (s - first + 1) % log_every == 0:
            _say(f"generated {s - first + 1}/{count} clusters, {time.time() - t0:.0f}s, "
                 f"mean SAD steps {np.mean(rec['steps']):.2f}")
    np.savez(out, seed=np.array(rec["seed"]), n=np.array(rec["n"]),
             atoms=np.concatenate(rec["atoms"]), p=np.concatenate(rec["p"]),
             t=np.array(rec["t"]), steps=np.array(rec["steps"]),
             eig=np.concatenate(rec["eig"]), last_dtheta=np.array(rec["last_dtheta"]))
    _say(f"wrote {out}")


# ------------------------------------------------------------------- train

class Batch:
    """Device arrays of a set of clusters for the batched loss."""

    def __init__(self, ctx, seeds_atoms, p_list, t_list, torch):
        feats, M, moff, rows = [], [], [0], [0]
        for atoms in seeds_atoms:
            d, dirs = ces.atom_descriptors(atoms)
            feats.append(d)
            Mc, _, _ = ctx.loss_terms(atoms, dirs, None)
            M.append(Mc.astype(np.float32).reshape(-1))
            moff.append(moff[-1] + Mc.size)
            rows.append(rows[-1] + len(atoms))
        self.rows = int(rows[-1])
        self.max_atoms = int(max(len(a) for a in seeds_atoms))
        self.T = float(np.sum(t_list))
        self.feats_host = np.concatenate(feats)
        self.X = torch.from_numpy(self.feats_host).cuda()
        self.M = torch.from_numpy(np.concatenate(M)).cuda()
        self.moff = torch.from_numpy(np.array(moff[:-1], dtype=np.int64)).cuda()
        self.row_off = torch.from_numpy(np.array(rows, dtype=np.int64)).cuda()
        self.p = torch.from_numpy(np.concatenate(p_list).astype(np.float32)).cuda()
        self.t = torch.from_numpy(np.asarray(t_list, dtype=np.float32)).cuda()
        self.out = torch.empty((self.rows, ces.MLP_CHANNELS), dtype=torch.float32, device="cuda")
        self.gout = torch.empty_like(self.out)
        self.loss = torch.empty(len(seeds_atoms), dtype=torch.float32, device="cuda")


def _split(data):
    """Per-cluster atoms, p and t from a generate() file."""
    n = data["n"]
    a_off = np.concatenate([[0], np.cumsum(3 * n)])
    p_off = np.concatenate([[0], np.cumsum(ces.MLP_CHANNELS * n)])
    atoms = [data["atoms"][a_off[i]:a_off[i + 1]].reshape(-1, 3) for i in range(len(n))]
    ps = [data["p"][p_off[i]:p_off[i + 1]] for i in range(len(n))]
    return atoms, ps, list(data["t"])


def train(files, out, epochs=400, batch=100, lr=1e-3, seed=0, val_file=None):
    import torch
    ctx = Context()
    atoms, ps, ts = [], [], []
    for f in files:
        a, p, t = _split(np.load(f))
        atoms += a
        ps += p
        ts += t
    order = np.random.default_rng(seed).permutation(len(atoms))
    batches = []
    t0 = time.time()
    for b0 in range(0, len(order), batch):
        idx = order[b0:b0 + batch]
        batches.append(Batch(ctx, [atoms[i] for i in idx], [ps[i] for i in idx],
                             [ts[i] for i in idx], torch))
    val = None
    if val_file:
        va, vp, vt = _split(np.load(val_file))
        val = Batch(ctx, va, vp, vt, torch)
    _say(f"{len(atoms)} clusters in {len(batches)} batches prepared in {time.time() - t0:.0f}s")
    allf = np.concatenate([b.feats_host for b in batches])
    mean = allf.mean(0)
    std = allf.std(0) + 1e-3
    net = ces.MLP(seed=seed + 1)
    net.set(mean=mean, std=std)
    # start at zero correction: last layer weights and bias 0
    p0, _, _ = net.get()
    n_last = net.sizes[-2] * net.sizes[-1] + net.sizes[-1]
    p0[-n_last:] = 0.0
    net.set(params=p0)
    rows_max = max(b.rows for b in batches + ([val] if val else []))
    work = net.workspace(rows_max)
    step = 0
    hist = []
    rng = np.random.default_rng(seed + 2)
    t0 = time.time()
    for ep in range(1, epochs + 1):
        lr_ep = lr * (0.1 ** (ep / epochs))
        tot_l, tot_t = 0.0, 0.0
        for bi in rng.permutation(len(batches)):
            b = batches[bi]
            net.forward(b.X, b.out, work)
            ces.cluster_quad_loss(b.row_off, b.moff, b.M, b.p, b.t, b.out, b.gout, b.loss,
                                  b.max_atoms, scale=1.0 / b.T)
            net.backward(b.gout, work)
            step += 1
            net.adam_step(step, lr_ep)
            tot_l += float(b.loss.sum())
            tot_t += b.T
        rec = {"epoch": ep, "train_rel": tot_l / tot_t}
        if val is not None and (ep % 10 == 0 or ep == epochs):
            net.forward(val.X, val.out, work)
            ces.cluster_quad_loss(val.row_off, val.moff, val.M, val.p, val.t, val.out, val.gout,
                                  val.loss, val.max_atoms, scale=1.0)
            rec["val_rel"] = float(val.loss.sum()) / val.T
        hist.append(rec)
        if ep % 10 == 0 or ep == 1:
            _say(f"epoch {ep} {time.time() - t0:.0f}s train rel {rec['train_rel']:.4f}"
                 + (f" val rel {rec['val_rel']:.4f}" if "val_rel" in rec else ""))
    params, mean, std = net.get()
    np.savez(out, params=params, mean=mean, std=std, sizes=np.array(net.sizes),
             history=json.dumps(hist), n_train=len(atoms))
    _say(f"wrote {out}")
    return hist


def load_network(path=DEFAULT_WEIGHTS):
    w = np.load(path)
    sizes = [int(x) for x in w["sizes"]]
    net = ces.MLP(n_in=sizes[0], width=sizes[1], depth=len(sizes) - 2, n_out=sizes[-1])
    net.set(w["params"], w["mean"], w["std"])
    return net


def learned_density(ctx, net, atoms, rho_sad=None):
    """rho_SAD + the network's correction for this cluster (device tensor)."""
    torch = ctx.torch
    desc, dirs = ces.atom_descriptors(atoms)
    out = torch.empty((len(atoms), ces.MLP_CHANNELS), dtype=torch.float32, device="cuda")
    work = net.workspace(len(atoms))
    net.forward(torch.from_numpy(desc).cuda(), out, work)
    rho = (ctx.sad(atoms) if rho_sad is None else rho_sad).clone()
    ctx.H.density_correction(atoms, dirs, out, rho)
    return rho, out, dirs


# ---------------------------------------------------------------- evaluate

def steps_to(dtheta, tol):
    """SCF steps until the largest occupied eigenvalue change first fell below
    tol (the run's own step count if it never did before it stopped)."""
    for i, v in enumerate(dtheta):
        if v < tol:
            return i + 1
    return len(dtheta)


def evaluate(weights, first, count, out, data_out=None, tol=1e-8, count_tol=1e-6):
    """Both SCFs (SAD start, learned start) run to |delta theta| < tol; the
    step counts are reported at tol and at count_tol (the first step whose
    change fell below it), and the converged eigenvalues of the two runs are
    compared at tol."""
    ctx = Context(tol=tol)
    net = load_network(weights)
    rows = []
    rec = {k: [] for k in ("seed", "n", "atoms", "p", "t", "steps", "eig", "last_dtheta")}
    t0 = time.time()
    for s in range(first, first + count):
        atoms = si.scf_cluster(s)
        n_occ, _ = si.scf_occupation(len(atoms))
        fields = ctx.fields(atoms)
        rho_sad = ctx.sad(atoms)
        ev_s, st_s, dth_s, rho = ctx.scf(atoms, rho_sad, fields=fields)
        rho_l, coef, dirs = learned_density(ctx, net, atoms, rho_sad)
        ev_l, st_l, dth_l, _ = ctx.scf(atoms, rho_l, fields=fields)
        M, p, t = ctx.loss_terms(atoms, dirs, rho - rho_sad)
        c = coef.cpu().numpy().astype(np.float64).reshape(-1)
        rel_err = (c @ M @ c - 2 * p @ c + t) / t
        rows.append({"seed": s, "n": len(atoms), "steps_sad": st_s, "steps_learned": st_l,
                     "steps_sad_at_count_tol": steps_to(dth_s, count_tol),
                     "steps_learned_at_count_tol": steps_to(dth_l, count_tol),
                     "converged": bool(dth_s[-1] < tol and dth_l[-1] < tol),
                     "max_eig_diff": float(np.max(np.abs(ev_s[:n_occ] - ev_l[:n_occ]))),
                     "start_rel_sq_err": float(rel_err)})
        for k, v in (("seed", s), ("n", len(atoms)), ("atoms", atoms.reshape(-1)), ("p", p),
                     ("t", t), ("steps", st_s), ("eig", ev_s[:n_occ]), ("last_dtheta", dth_s[-1])):
            rec[k].append(v)
        if (s - first + 1) % 20 == 0:
            _say(f"evaluated {s - first + 1}/{count}, {time.time() - t0:.0f}s: mean steps SAD "
                 f"{np.mean([r['steps_sad'] for r in rows]):.2f}, learned "
                 f"{np.mean([r['steps_learned'] for r in rows]):.2f}")
    ss = np.array([r["steps_sad"] for r in rows])
    sl = np.array([r["steps_learned"] for r in rows])
    cs = np.array([r["steps_sad_at_count_tol"] for r in rows])
    cl = np.array([r["steps_learned_at_count_tol"] for r in rows])
    diffs = np.array([r["max_eig_diff"] for r in rows])
    summary = {
        "clusters": count, "tol": ctx.tol, "count_tol": count_tol,
        "all_converged": bool(all(r["converged"] for r in rows)),
        "mean_steps_sad": float(ss.mean()), "mean_steps_learned": float(sl.mean()),
        "median_steps_sad": float(np.median(ss)), "median_steps_learned": float(np.median(sl)),
        "fraction_fewer": float(np.mean(sl < ss)), "fraction_more": float(np.mean(sl > ss)),
        "mean_steps_sad_at_count_tol": float(cs.mean()),
        "mean_steps_learned_at_count_tol": float(cl.mean()),
        "hist_sad": np.bincount(ss).tolist(), "hist_learned": np.bincount(sl).tolist(),
        "max_eig_diff": float(diffs.max()),
        "clusters_eig_diff_above_1e-6": int(np.sum(diffs > 1e-6)),
        "median_start_rel_sq_err": float(np.median([r["start_rel_sq_err"] for r in rows])),
        "per_cluster": rows,
    }
    with open(out, "w") as f:
        json.dump(summary, f, indent=1)
    if data_out:
        np.savez(data_out, seed=np.array(rec["seed"]), n=np.array(rec["n"]),
                 atoms=np.concatenate(rec["atoms"]), p=np.concatenate(rec["p"]),
                 t=np.array(rec["t"]), steps=np.array(rec["steps"]),
                 eig=np.concatenate(rec["eig"]), last_dtheta=np.array(rec["last_dtheta"]))
    _say(json.dumps({k: v for k, v in summary.items() if k != "per_cluster"}))
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--first", type=int, default=si.TRAIN_SEED0)
    g.add_argument("--count", type=int, default=1000)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--val")
    t.add_argument("--epochs", type=int, default=400)
    t.add_argument("--batch", type=int, default=100)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--first", type=int, default=si.HELDOUT_SEED0)
    e.add_argument("--count", type=int, default=200)
    e.add_argument("--out", required=True)
    e.add_argument("--data-out")
    e.add_argument("--tol", type=float, default=1e-8)
    e.add_argument("--count-tol", type=float, default=1e-6)
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        generate(a.first, a.count, a.out)
    elif a.cmd == "train":
        train(a.data, a.out, epochs=a.epochs, batch=a.batch, lr=a.lr, val_file=a.val)
    else:
        evaluate(a.weights, a.first, a.count, a.out, a.data_out, a.tol, a.count_tol)


if __name__ == "__main__":
    main()
