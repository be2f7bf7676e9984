"""Per-launch hardware counters of the kernels, reduced from rocprofv3 runs.

`python -m paper_2108_12742_amd.counters --workload W --fetch D1 --write D2 [--sq D3]
[--calib-mib 256] [--out profiles/counters.json]` reads the counter-collection CSV
files that rocprofv3 wrote under the directories D1 (`--pmc FETCH_SIZE`), D2
(`--pmc WRITE_SIZE`) and D3 (a pass with `SQ_INSTS_VALU_FLOPS_FP64`), and records
per kernel symbol:
  * bytes_per_launch: HBM bytes read and written per dispatch.  FETCH_SIZE and
    WRITE_SIZE are in KiB per dispatch; each is scaled by what the same counter
    reads for the first device-to-device copy of the run (bench.py
    --copy-calibration-mib: a copy of known size, which reads and writes that
    many bytes);
  * fp64_flops_per_launch: executed FP64 flops per dispatch (the counter counts per
    wave instruction, an FMA as 2: times 64 lanes).
The record carries the hash of the HIP sources and build flags it was taken with;
bench.py uses it only while that hash matches.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_sources_hash() -> str:
    """sha256 (first 16 hex) of the HIP sources and of the build script that holds the
    compiler flags: a change to either invalidates recorded counters."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.hpp")))
    files.append(os.path.join(HERE, "build.py"))
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_symbol(name: str) -> str:
    """a profiler's kernel name without return type and argument list:
    "void enoao::sweep_y<5, 2, false, 8, true>(enoao::KParams)" -> "enoao::sweep_y<5, 2, false, 8, true>" """
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def read_counter(directory: str, counter: str):
    """[(dispatch id, kernel name, value)] of one counter from the CSV files under
    directory, in dispatch order."""
    rows = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                rows.append((int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0), kernel_symbol(r["Kernel_Name"]),
                             float(r["Counter_Value"])))
    rows.sort()
    return rows


def per_kernel_mean(rows, skip_first_copy=True):
    """mean value per kernel name; the first copy dispatch (the calibration) separately"""
    acc = defaultdict(list)
    calib = None
    for _, name, v in rows:
        if name.startswith(COPY_KERNEL) and calib is None:
            calib = v
            if skip_first_copy:
                continue
        acc[name].append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}, calib


def reduce(workload: str, fetch_dir: str, write_dir: str, sq_dir: str | None, calib_mib: int, cells: int | None):
    fetch, fcal = per_kernel_mean(read_counter(fetch_dir, "FETCH_SIZE"))
    write, wcal = per_kernel_mean(read_counter(write_dir, "WRITE_SIZE"))
    if fcal is None or wcal is None:
        raise SystemExit("no calibration copy found: run bench.py with --copy-calibration-mib")
    copied_kib = calib_mib * 1024.0
    fs, ws = copied_kib / fcal, copied_kib / wcal
    rec = {"fetch_scale": fs, "write_scale": ws, "calibration_mib": calib_mib, "bytes_per_launch": {},
           "fetch_kib_raw": {}, "write_kib_raw": {}}
    if cells:
        rec["cells"] = cells
    for name in sorted(set(fetch) & set(write)):
        if name.startswith(COPY_KERNEL):
            continue
        rec["bytes_per_launch"][name] = (fetch[name] * fs + write[name] * ws) * 1024.0
        rec["fetch_kib_raw"][name] = fetch[name]
        rec["write_kib_raw"][name] = write[name]
    if sq_dir:
        fl, _ = per_kernel_mean(read_counter(sq_dir, "SQ_INSTS_VALU_FLOPS_FP64"), skip_first_copy=False)
        rec["fp64_flops_per_launch"] = {k: 64.0 * v for k, v in fl.items() if not k.startswith(COPY_KERNEL)}
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--sq", default=None)
    ap.add_argument("--calib-mib", type=int, default=256)
    ap.add_argument("--cells", type=int, default=None)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "counters.json"))
    a = ap.parse_args()
    rec = reduce(a.workload, a.fetch, a.write, a.sq, a.calib_mib, a.cells)
    try:
        with open(a.out) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        data = {}
    h = kernel_sources_hash()
    if data.get("source_hash") != h:
        data = {"source_hash": h, "workloads": {}}
    data["workloads"][a.workload] = rec
    with open(a.out, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")
    for k, v in sorted(rec["bytes_per_launch"].items()):
        print(f"{v / 1e6:10.1f} MB  {k}")


if __name__ == "__main__":
    main()
