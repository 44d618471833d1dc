"""HBM traffic per launch, from rocprofv3 counter runs.

Two counter runs of the benchmark (one with FETCH_SIZE, one with
WRITE_SIZE: the KiB the L2 read from and wrote to memory per dispatch, as
the hardware counts them) give the raw readings per kernel.  Two more runs
of a plain device copy of known size give the ratio between those readings
and real bytes (reading / bytes moved), which is divided out.  The result
goes to a small JSON file beside the profile summaries, together with a
hash of the kernel sources it was measured on; bench.py reports the
traffic of a kernel class only while those sources are unchanged.

  python -m paper_2406_19920_amd.pmc --fetch D1 --write D2 --copy-fetch D3 \\
      --copy-write D4 --copy-bytes N --out profiles/traffic_256cube.json

D1..D4 are rocprofv3 output directories (-d) holding *counter_collection.csv.
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
import sys

PKG = os.path.dirname(os.path.abspath(__file__))

# profile class -> (kernel-name pattern, source files it is built from)
CLASSES = {
    "xgemm_f64": (r"\b(xgemm_f64_kernel|xfold_f64_kernel)<", ("k_xform.hip", "k_fold.hip")),
    "zgemm_f64": (r"\b(zgemm_f64_kernel|zfold_f64_kernel)<", ("k_xform.hip", "k_fold.hip")),
    "tridiag_f64": (r"\btridiag_kernel<double", ("k_tridiag.hip",)),
    "tridiag_f32": (r"\btridiag_kernel<float", ("k_tridiag.hip",)),
    "divergence": (r"\bdivergence_kernel\b", ("k_stencil.hip",)),
    "correct": (r"\bcorrect_kernel\b", ("k_stencil.hip",)),
    "residual": (r"\bresidual_f32_kernel\b", ("k_split.hip",)),
    "xgemm_split": (r"\bsplit_x\w*kernel<\d+, \d+, (double|float), 0(, false)?(, \d+)?>", ("k_split.hip",)),
    "zgemm_split": (r"\bsplit_z\w*kernel<", ("k_split.hip",)),
    "update": (r"\bsplit_x\w*kernel<\d+, \d+, float, [1-4](, true)?(, \d+)?>", ("k_split.hip",)),
    "explicit": (r"\bexplicit_kernel\b", ("k_fstep.hip",)),
    "ibm": (r"\bibm_kernel\b", ("k_fstep.hip",)),
}


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in sorted(set(files) | {"ibs_internal.h"}):
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def read_counter(directory: str, counter: str) -> dict:
    """kernel name -> list of per-dispatch readings of `counter`."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {directory}")
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for f in files:
        for row in csv.DictReader(open(f)):
            if row.get("Counter_Name") != counter:
                continue
            key = (f, row.get("Dispatch_Id", row.get("Correlation_Id", "")))
            per[row["Kernel_Name"]][key] += float(row["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def mean(xs):
    return sum(xs) / len(xs) if xs else 0.0


def copy_ratio(directory: str, counter: str, nbytes: int) -> float:
    """Reading / real bytes for the largest kernel of a plain-copy run."""
    k = read_counter(directory, counter)
    name = max(k, key=lambda n: mean(k[n]))
    return mean(k[name]) * 1024.0 / nbytes


def class_means(directory: str, counter: str) -> dict:
    k = read_counter(directory, counter)
    out = {}
    for cls, (pat, _) in CLASSES.items():
        vals = [v for name, vs in k.items() if re.search(pat, name) for v in vs]
        if vals:
            out[cls] = (mean(vals), len(vals))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="", help="the profiled command, recorded in the output")
    a = ap.parse_args(argv)
    rf = copy_ratio(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
    rw = copy_ratio(a.copy_write, "WRITE_SIZE", a.copy_bytes)
    fetch = class_means(a.fetch, "FETCH_SIZE")
    write = class_means(a.write, "WRITE_SIZE")
    res = {"copy_ratio": {"fetch": rf, "write": rw, "copy_bytes": a.copy_bytes},
           "command": a.command, "kernels": {}}
    for cls in sorted(set(fetch) & set(write)):
        f_kib, nf = fetch[cls]
        w_kib, nw = write[cls]
        res["kernels"][cls] = {
            "fetch_bytes_per_launch": f_kib * 1024.0 / rf,
            "write_bytes_per_launch": w_kib * 1024.0 / rw,
            "bytes_per_launch": f_kib * 1024.0 / rf + w_kib * 1024.0 / rw,
            "raw_fetch_kib": f_kib, "raw_write_kib": w_kib, "dispatches": [nf, nw],
            "source_hash": source_hash(CLASSES[cls][1]),
        }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    json.dump(res, sys.stdout, indent=1, sort_keys=True)
    print()


def traffic_for(cls: str, path: str):
    """Bytes per launch of class `cls` from a stored measurement, or None
    when there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    d = json.load(open(path)).get("kernels", {}).get(cls)
    if not d or d.get("source_hash") != source_hash(CLASSES[cls][1]):
        return None
    return d["bytes_per_launch"]


if __name__ == "__main__":
    main()
