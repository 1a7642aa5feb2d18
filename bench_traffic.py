"""Helpers that turn rocprofv3 counter databases into the HBM-traffic record
bench.py reports (roofline.traffic).

Two profiled runs of the same command are needed, one with --pmc FETCH_SIZE
and one with --pmc WRITE_SIZE (rocprofv3 collects a counter set per run).
Both counters are in KiB per dispatch.  They are scaled by what they read for
a plain copy of known size in the same run (bench.py --calib-copy-mib N copies
N MiB once before timing): FETCH_SIZE has read half the copied bytes on this
GPU, WRITE_SIZE all of them.

Usage (from the repository root, after the two profiled runs):
  python bench_traffic.py FETCH_DB WRITE_DB KERNEL CALIB_MIB OUT_JSON "COMMAND" [SOURCE]

SOURCE is the kernel's source file (default: the tiled Gram kernels); its
SHA-256 goes into the record so that bench.py drops the figure once the source
changes.
"""
from __future__ import annotations

import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def dispatches(db_path: str):
    """(dispatch_id, kernel_name, value_kib, duration_ns) of every counter row."""
    db = sqlite3.connect(db_path)
    try:
        return list(db.execute("select dispatch_id, kernel_name, value, duration from counters_collection "
                               "order by dispatch_id"))
    finally:
        db.close()


def calibration_factor(rows, calib_bytes: int, is_write: bool) -> float:
    """Known bytes / counted bytes for the calibration copy: the first copy dispatch
    whose counted size is within a factor 4 of the copied size."""
    for _, name, kib, _ in rows:
        if "copyBuffer" in name or "direct_copy" in name:
            counted = kib * 1024.0
            if calib_bytes / 4 <= counted <= calib_bytes * 4:
                return calib_bytes / counted
    raise ValueError("no calibration copy of %d bytes found" % calib_bytes)


def kernel_rows(rows, kernel: str):
    """Rows of the named kernel with the largest grid work: the longest dispatches
    (the first processed mode of every step)."""
    sel = [r for r in rows if kernel in r[1].replace("(anonymous namespace)", "")]
    if not sel:
        raise ValueError("kernel %r not found" % kernel)
    longest = max(r[3] for r in sel)
    return [r for r in sel if r[3] >= 0.5 * longest]


def source_digest(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def summarize(fetch_db, write_db, kernel, calib_mib, out_json, command, source_file):
    calib = calib_mib * (1 << 20)
    fr, wr = dispatches(fetch_db), dispatches(write_db)
    ff, wf = calibration_factor(fr, calib, False), calibration_factor(wr, calib, True)
    fk, wk = kernel_rows(fr, kernel), kernel_rows(wr, kernel)
    fetch = sum(r[2] for r in fk) / len(fk) * 1024.0 * ff
    write = sum(r[2] for r in wk) / len(wk) * 1024.0 * wf
    rec = {"kernel": kernel, "source": os.path.relpath(source_file, HERE),
           "source_sha256": source_digest(source_file),
           "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
           "traffic_bytes_per_launch": round(fetch + write),
           "fetch_scale": round(ff, 4), "write_scale": round(wf, 4), "launches_averaged": len(fk),
           "calibration_copy_mib": calib_mib, "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


if __name__ == "__main__":
    if len(sys.argv) not in (7, 8):
        print(__doc__, file=sys.stderr)
        sys.exit(2)
    fdb, wdb, kern, mib, out, cmd = sys.argv[1:7]
    src = sys.argv[7] if len(sys.argv) == 8 else os.path.join(HERE, "paper_2107_01384_amd", "csrc",
                                                                "atc_gram_kc.hip")
    print(json.dumps(summarize(fdb, wdb, kern, int(mib), out, cmd, src)))
