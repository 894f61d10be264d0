"""Summarise rocprofv3 FETCH_SIZE / WRITE_SIZE passes into HBM bytes per launch.

Each pass is a separate `rocprofv3 --pmc <counter> --output-format csv` run of
`bench.py --pmc-run`, which launches the H*X kernels and a plain elementwise
copy of a known number of bytes (read and written once).  The copy's counter
readings calibrate each counter: scale = copy bytes / (counter KiB * 1024).
Per kernel, traffic = fetch KiB * 1024 * fetch scale + write KiB * 1024 *
write scale, averaged over its dispatches.

  python -m paper_1404_3773_amd.pmc_summary --fetch DIR --write DIR \\
      --copy-bytes N --kernel 'k_phi_stage<float, 96>' --workload NAME \\
      [--extra DIR ...] --json OUT.json

--extra passes (e.g. SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE,
SQ_INSTS_VALU_MFMA_MOPS_F32 / _F64) are averaged per kernel into the same
rows, with two derived figures where their counters are present:
  mfma_busy_frac = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / n_xcc * n_simd)
    (GRBM_GUI_ACTIVE sums the active cycles of the n_xcc dies; the busy
    cycles sum over all n_simd SIMDs; both from the pass's agent table)
  mfma_flop_f32 / _f64 = SQ_INSTS_VALU_MFMA_MOPS_F32 / _F64 * 512
    (the counter counts MFMA work in units of 512 flops)

  python -m paper_1404_3773_amd.pmc_summary stats --db RUN_results.db [--top 40]
prints the kernel table (calls, average and total milliseconds, share) of a
rocprofv3 --kernel-trace --stats database, and

  python -m paper_1404_3773_amd.pmc_summary table SUMMARY.json [...]
the MFMA kernels of summaries written by the first form: launches, MFMA busy,
executed MFMA flop and traffic per launch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(name):
    name = name.replace("void ", "").replace("ces::(anonymous namespace)::", "")
    name = name.replace("ces::", "")
    return re.sub(r"\(.*", "", name).strip()


def per_kernel(pass_dir, counter):
    """{kernel: mean counter value per dispatch} from one pass directory."""
    vals = collections.defaultdict(list)
    for path in glob.glob(os.path.join(pass_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] != counter:
                    continue
                vals[short_name(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def kernel_source(text, name):
    """The source of the __global__ function `name` in `text`: from the
    template line (if any) before its declaration to the closing brace at
    the start of a line."""
    m = re.search(r"__global__[^;{]*?\b" + re.escape(name) + r"\s*\(", text)
    if not m:
        raise SystemExit(f"kernel {name} not found")
    start = m.start()
    t = text.rfind("template", 0, start)
    if t != -1 and text[t:start].count("\n") <= 1:
        start = t
    end = text.index("\n}\n", m.end()) + 3
    return text[start:end]


def source_digest(files):
    """SHA-256 over the listed sources in csrc/: a whole file, or `file#kernel`
    for one kernel's own source."""
    h = hashlib.sha256()
    for f in files:
        path, _, kern = f.partition("#")
        with open(os.path.join(HERE, "csrc", path), encoding="utf-8") as fh:
            text = fh.read()
        h.update((kernel_source(text, kern) if kern else text).encode())
    return h.hexdigest()


def counters_in(pass_dir):
    """Names of the counters a pass directory holds."""
    names = set()
    for path in glob.glob(os.path.join(pass_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                names.add(row["Counter_Name"])
    return sorted(names)


def gpu_agent(pass_dir):
    """(Simd_Count, Num_Xcc) of the GPU agent recorded by a pass."""
    for path in glob.glob(os.path.join(pass_dir, "**", "*agent_info.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Agent_Type") == "GPU":
                    return int(row["Simd_Count"]), int(row["Num_Xcc"])
    return None


def derived(row, agent):
    busy, active = row.get("SQ_VALU_MFMA_BUSY_CYCLES"), row.get("GRBM_GUI_ACTIVE")
    if busy is not None and active and agent:
        n_simd, n_xcc = agent
        row["mfma_busy_frac"] = busy / (active / n_xcc * n_simd)
    for prec in ("F32", "F64"):
        mops = row.get(f"SQ_INSTS_VALU_MFMA_MOPS_{prec}")
        if mops is not None:
            row[f"mfma_flop_{prec.lower()}"] = mops * 512.0


def kernel_stats(db, top):
    """Rows (kernel, calls, avg_ms, total_ms, share %) of a rocprofv3 stats
    database's top_kernels view (which holds microseconds)."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select * from top_kernels").fetchall()
    con.close()
    out = []
    for name, calls, total_us, avg_us, pct in rows[:top]:
        out.append((short_name(name), int(calls), avg_us / 1e3, total_us / 1e3, pct))
    return out


def stats_main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", required=True)
    ap.add_argument("--top", type=int, default=40)
    a = ap.parse_args(argv)
    print(f"{'share%':>7s} {'calls':>6s} {'avg_ms':>11s} {'total_ms':>12s}  kernel")
    for name, calls, avg, tot, pct in kernel_stats(a.db, a.top):
        print(f"{pct:7.2f} {calls:6d} {avg:11.3f} {tot:12.1f}  {name}")


def table_main(paths):
    print(f"# {'workload':18s}  {'kernel':44s}  {'launches':>8s}  {'mfma_busy':>9s}  "
          f"{'mfma_Tflop':>10s}  {'traffic_GB':>10s}")
    for path in paths:
        with open(path) as f:
            d = json.load(f)
        for r in d["kernels"]:
            fl = r.get("mfma_flop_f32", 0) + r.get("mfma_flop_f64", 0)
            if "mfma_busy_frac" in r and fl > 0:
                print(f"  {d['workload']:18s}  {r['kernel']:44s}  {r['dispatches']:8d}  "
                      f"{r['mfma_busy_frac']:9.3f}  {fl / 1e12:10.3f}  "
                      f"{r['traffic_bytes'] / 1e9:10.2f}")


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "stats":
        return stats_main(argv[1:])
    if argv and argv[0] == "table":
        return table_main(argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--copy-match", default="elementwise")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--sources", nargs="+",
                    default=["kernels_angular.hip", "kernels_radial.hip", "kernels_kb.hip",
                             "mfma.h"],
                    help="sources the summary is valid for: files in csrc/, or file#kernel "
                         "(by default every H*X stage kernel's source: the summary carries "
                         "the counters of all of them)")
    ap.add_argument("--json", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="")
    ap.add_argument("--extra", nargs="*", default=[],
                    help="further pass directories (e.g. MFMA counters), averaged per kernel")
    a = ap.parse_args(argv)
    fetch = per_kernel(a.fetch, "FETCH_SIZE")
    write = per_kernel(a.write, "WRITE_SIZE")
    extra = {}
    agent = None
    for d in a.extra:
        agent = agent or gpu_agent(d)
        for c in counters_in(d):
            extra[c] = per_kernel(d, c)
    copy_f = [v for k, (v, n) in fetch.items() if a.copy_match in k]
    copy_w = [v for k, (v, n) in write.items() if a.copy_match in k]
    if not copy_f or not copy_w:
        raise SystemExit("copy kernel not found in the passes")
    fs = a.copy_bytes / (max(copy_f) * 1024.0)
    ws = a.copy_bytes / (max(copy_w) * 1024.0)
    rows = []
    for k in sorted(set(fetch) & set(write)):
        if not k.startswith("k_"):
            continue
        fk, nf = fetch[k]
        wk, nw = write[k]
        row = {"kernel": k, "dispatches": min(nf, nw), "fetch_kib": fk, "write_kib": wk,
               "traffic_bytes": fk * 1024 * fs + wk * 1024 * ws}
        for c, vals in extra.items():
            if k in vals:
                row[c] = vals[k][0]
        derived(row, agent)
        rows.append(row)
    target = [r for r in rows if r["kernel"] == a.kernel]
    out = {"kernel": a.kernel, "workload": a.workload, "copy_bytes": a.copy_bytes,
           "copy_fetch_kib": max(copy_f), "copy_write_kib": max(copy_w),
           "fetch_scale": fs, "write_scale": ws,
           "traffic_bytes": target[0]["traffic_bytes"] if target else None,
           "sources": a.sources, "source_sha256": source_digest(a.sources),
           "command": a.command, "kernels": rows}
    with open(a.json, "w") as f:
        json.dump(out, f, indent=1)
    print(f"copy calibration: fetch x{fs:.4f}, write x{ws:.4f}")
    for r in rows:
        more = "".join(f"  {c} {r[c]:.4g}" for c in list(extra) + ["mfma_busy_frac"] if c in r)
        print(f"{r['kernel']:48s} {r['dispatches']:5d}  fetch {r['fetch_kib']:12.1f} KiB  "
              f"write {r['write_kib']:12.1f} KiB  traffic {r['traffic_bytes'] / 1e6:10.3f} MB"
              + more)


if __name__ == "__main__":
    main()
