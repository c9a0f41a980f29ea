"""HBM traffic of one kernel from rocprofv3 counter runs.

Two runs of the same command, one with ``--pmc FETCH_SIZE`` and one with
``--pmc WRITE_SIZE`` (each counter reads KiB per dispatch), are reduced to
bytes per launch of the named kernel.  Both counters are scaled by what they
read for a plain device copy of known size in the same process (``bench.py
--pmc-apply`` ends with copies of 1 GiB), so the figures are HBM bytes.

The record is stored with the SHA-256 of the kernel source and the workload
key; ``bench.py`` reports it only while both still match, i.e. never for a
kernel changed after its counters were taken.

    python -m paper_2502_08382_amd.traffic FETCH_CSV WRITE_CSV KEY [--kernel NAME]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
STORE = os.path.join(HERE, "traffic.json")
COPY_BYTES = 1 << 30


# the source of the operator kernels (assembly and apply) and the headers it
# includes; the solver kernels live in another file and do not enter the hash
KERNEL_SOURCES = ("device_types.hpp", "kernels.hip", "kernels.hpp")


def kernel_source_hash():
    """SHA-256 (hex, first 16) of the operator kernel sources."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _dispatches(path, counter):
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            out.append((row["Kernel_Name"], float(row["Counter_Value"]),
                        (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3))
    return out


def _copy_kib(rows):
    """Counter of the 1 GiB copies: the dispatches of a copy kernel whose
    value is within 10 % of the largest such value."""
    cands = [v for name, v, _ in rows if "copy" in name.lower()]
    if not cands:
        raise ValueError("no copy dispatch in the counter file")
    top = max(cands)
    sel = [v for v in cands if v >= 0.9 * top]
    return sum(sel) / len(sel)


def summarize(fetch_csv, write_csv, kernel="apply_band_kernel"):
    fr, wr = _dispatches(fetch_csv, "FETCH_SIZE"), _dispatches(write_csv, "WRITE_SIZE")
    f_fetch = COPY_BYTES / (_copy_kib(fr) * 1024.0)
    f_write = COPY_BYTES / (_copy_kib(wr) * 1024.0)
    fk = [v for name, v, _ in fr if kernel in name]
    wk = [v for name, v, _ in wr if kernel in name]
    if not fk or not wk:
        raise ValueError(f"no dispatch of {kernel}")
    fetch = sum(fk) / len(fk) * 1024.0 * f_fetch
    write = sum(wk) / len(wk) * 1024.0 * f_write
    return {"kernel": kernel, "dispatches": len(fk), "fetch_kib": [min(fk), max(fk)],
            "write_kib": [min(wk), max(wk)], "fetch_factor": round(f_fetch, 4), "write_factor": round(f_write, 4),
            "fetch_bytes": fetch, "write_bytes": write, "traffic_bytes": fetch + write,
            "source_sha256_16": kernel_source_hash()}


def lookup(key):
    """Stored traffic record for a workload key if the kernels are unchanged."""
    try:
        with open(STORE) as f:
            rec = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256_16") != kernel_source_hash():
        return None
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("key", help="workload key printed by bench.py --pmc-apply")
    ap.add_argument("--kernel", default="apply_band_kernel")
    args = ap.parse_args()
    rec = summarize(args.fetch_csv, args.write_csv, args.kernel)
    data = {}
    if os.path.exists(STORE):
        with open(STORE) as f:
            data = json.load(f)
    data[args.key] = rec
    with open(STORE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
