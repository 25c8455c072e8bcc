"""HBM traffic of one kernel from two rocprofv3 counter runs.

rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (one counter per run) give
KiB per dispatch.  Both runs also hold launches of the library's plain copy
probe (fdbb_probe_copy of 1 GiB), whose true traffic is known: 1 GiB read
and 1 GiB written.  Each counter is scaled by what it reads for the copy, so
the result is HBM bytes per launch of the kernel.  The record carries a hash
of the kernel's sources; a record whose hash no longer matches the sources
describes another kernel and is not used.

    python -m paper_1809_09851_amd.traffic --kernel k_fused \\
        --fetch pmc_fetch/fetch_counter_collection.csv \\
        --write pmc_write/write_counter_collection.csv \\
        --n 16777216 --out profiles/fused3d_f64_2p24_traffic.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
FUSED_SOURCES = ("euler_point.hpp", "euler_tiles.hpp", "kernels_fused.hip")
COPY_BYTES = 1 << 30
COPY_KERNEL = "k_copy"


def kernel_hash(sources=FUSED_SOURCES) -> str:
    """First 16 hex digits of the SHA-256 of the kernel's source files."""
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_values(path: str, kernel: str):
    """Counter_Value of every dispatch whose kernel name contains `kernel`."""
    with open(path) as f:
        return [float(r["Counter_Value"]) for r in csv.DictReader(f) if kernel in r["Kernel_Name"]]


def build_record(kernel: str, fetch_csv: str, write_csv: str, n: int) -> dict:
    fk, wk = counter_values(fetch_csv, kernel), counter_values(write_csv, kernel)
    fc, wc = counter_values(fetch_csv, COPY_KERNEL), counter_values(write_csv, COPY_KERNEL)
    if not (fk and wk and fc and wc):
        raise ValueError("a counter file lacks the kernel's or the copy probe's dispatches")
    fetch_scale = COPY_BYTES / (statistics.mean(fc) * 1024)
    write_scale = COPY_BYTES / (statistics.mean(wc) * 1024)
    fetch_bytes = statistics.mean(fk) * 1024 * fetch_scale
    write_bytes = statistics.mean(wk) * 1024 * write_scale
    return {"kernel": kernel, "n": n, "kernel_hash": kernel_hash(),
            "fetch_kib_raw": statistics.mean(fk), "write_kib_raw": statistics.mean(wk),
            "copy_fetch_kib_raw": statistics.mean(fc), "copy_write_kib_raw": statistics.mean(wc),
            "fetch_scale": fetch_scale, "write_scale": write_scale,
            "fetch_bytes": fetch_bytes, "write_bytes": write_bytes,
            "bytes_per_launch": fetch_bytes + write_bytes}


def load_bytes_per_launch(path: str, n: int):
    """bytes_per_launch of a stored record, or None when it is missing, for
    another size, or for kernel sources that have changed since."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash() or rec.get("n") != n:
        return None
    return rec.get("bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    rec = build_record(args.kernel, args.fetch, args.write, args.n)
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
