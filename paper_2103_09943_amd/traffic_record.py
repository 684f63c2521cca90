"""Turn two rocprofv3 counter runs of traffic_probe (FETCH_SIZE, then WRITE_SIZE) into per-launch HBM traffic.

    cd /tmp && export TMPDIR=/tmp
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d F -o run -- python3 -m paper_2103_09943_amd.traffic_probe
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d W -o run -- python3 -m paper_2103_09943_amd.traffic_probe
    python3 -m paper_2103_09943_amd.traffic_record F W profiles/traffic_8x2048.json

The probe's first kernel is a device copy of COPY_BYTES (read and written once), which calibrates the two
counters (KiB per dispatch as reported) against bytes.  Every iteration kernel's counters are averaged over its
dispatches, scaled, and stored with a hash of the kernel sources, so that readers can tell whether the record
still describes the code.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

from .traffic_probe import COPY_BYTES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCE_FILES = [
    "paper_2103_09943_amd/csrc/llp_sweep.hip",
    "paper_2103_09943_amd/csrc/llp_fast.hip",
    "paper_2103_09943_amd/csrc/llp_fast_util.h",
    "paper_2103_09943_amd/csrc/llp_device.h",
]
KERNELS = ("k_llp", "k_data", "k_apply_fast", "k_dir_fast")


def source_hash(files=SOURCE_FILES):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def read_counter(outdir, counter):
    """{kernel name: [value per dispatch]} from a rocprofv3 csv counter run."""
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {outdir}")
    vals = defaultdict(list)
    for fn in files:
        with open(fn) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                vals[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return vals


def main():
    if len(sys.argv) != 4:
        raise SystemExit(__doc__)
    fdir, wdir, out = sys.argv[1:]
    fetch, write = read_counter(fdir, "FETCH_SIZE"), read_counter(wdir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k or "copy" in k.lower()]
    if not copy:
        raise SystemExit("calibration copy not found")
    cf = max(fetch[copy[0]])  # the 256 MiB copy is the largest copy dispatch
    cw = max(write[copy[0]])
    fscale = COPY_BYTES / (cf * 1024.0)
    wscale = COPY_BYTES / (cw * 1024.0)
    rec = {"source_hash": source_hash(), "source_files": SOURCE_FILES,
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_kib_raw": cf, "write_kib_raw": cw,
                           "fetch_scale": fscale, "write_scale": wscale},
           "workload": "8 bands, 2048x2048, c=4, n=17, r=2; 10 CG iterations (all bands active)",
           "kernels": {}}
    rows = []
    for name in sorted(fetch):
        short = name.replace("(anonymous namespace)::", "").split("(")[0].removeprefix("void ").strip()
        if not any(k in short for k in KERNELS) or name not in write:
            continue
        # the iteration launches (mode 1 / mode 2) dominate; use the median dispatch
        fv = sorted(fetch[name])[len(fetch[name]) // 2]
        wv = sorted(write[name])[len(write[name]) // 2]
        rb, wb = fv * 1024.0 * fscale, wv * 1024.0 * wscale
        rec["kernels"][short] = {"dispatches": len(fetch[name]), "fetch_kib_raw": fv, "write_kib_raw": wv,
                                 "read_bytes": rb, "write_bytes": wb, "traffic_bytes": rb + wb}
        rows.append((short, len(fetch[name]), fv, wv, rb / 2**20, wb / 2**20))
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"calibration: FETCH_SIZE {cf:.0f} KiB -> x{fscale:.3f}, WRITE_SIZE {cw:.0f} KiB -> x{wscale:.3f}")
    print("| kernel | dispatches | FETCH_SIZE raw KiB (median) | WRITE_SIZE raw KiB | read MiB | write MiB |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| `{r[0]}` | {r[1]} | {r[2]:.0f} | {r[3]:.0f} | {r[4]:.0f} | {r[5]:.0f} |")


if __name__ == "__main__":
    main()
