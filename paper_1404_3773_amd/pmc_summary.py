"""Summarise rocprofv3 FETCH_SIZE / WRITE_SIZE passes into HBM bytes per launch.

Each pass is a separate `rocprofv3 --pmc <counter> --output-format csv` run of
`bench.py --pmc-run`, which launches the H*X kernels and a plain elementwise
copy of a known number of bytes (read and written once).  The copy's counter
readings calibrate each counter: scale = copy bytes / (counter KiB * 1024).
Per kernel, traffic = fetch KiB * 1024 * fetch scale + write KiB * 1024 *
write scale, averaged over its dispatches.

  python -m paper_1404_3773_amd.pmc_summary --fetch DIR --write DIR \\
      --copy-bytes N --kernel 'k_phi_stage<float>' --json OUT.json
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


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--copy-match", default="elementwise")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--sources", nargs="+", default=["kernels_angular.hip", "mfma.h"])
    ap.add_argument("--json", required=True)
    ap.add_argument("--command", default="")
    a = ap.parse_args(argv)
    fetch = per_kernel(a.fetch, "FETCH_SIZE")
    write = per_kernel(a.write, "WRITE_SIZE")
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
        rows.append({"kernel": k, "dispatches": min(nf, nw), "fetch_kib": fk, "write_kib": wk,
                     "traffic_bytes": fk * 1024 * fs + wk * 1024 * ws})
    target = [r for r in rows if r["kernel"] == a.kernel]
    out = {"kernel": a.kernel, "copy_bytes": a.copy_bytes,
           "copy_fetch_kib": max(copy_f), "copy_write_kib": max(copy_w),
           "fetch_scale": fs, "write_scale": ws,
           "traffic_bytes": target[0]["traffic_bytes"] if target else None,
           "sources": a.sources, "source_sha256": source_digest(a.sources),
           "command": a.command, "kernels": rows}
    with open(a.json, "w") as f:
        json.dump(out, f, indent=1)
    print(f"copy calibration: fetch x{fs:.4f}, write x{ws:.4f}")
    for r in rows:
        print(f"{r['kernel']:40s} {r['dispatches']:5d}  fetch {r['fetch_kib']:12.1f} KiB  "
              f"write {r['write_kib']:12.1f} KiB  traffic {r['traffic_bytes'] / 1e6:10.3f} MB")


if __name__ == "__main__":
    main()
