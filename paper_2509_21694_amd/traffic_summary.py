"""Turn two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE) of
`bench.py --copy-calibration MIB` into HBM bytes per launch of the
specialised edge kernels.

Each counter is scaled by what it reads for the device-to-device copy of
known size in the same run (the copy reads and writes MIB mebibytes), so the
result is in bytes of the copy's own accounting.  Prints a markdown summary
with one machine-readable `TRAFFIC_JSON:` line per kernel; `bench.py` reads
those lines and reports the figure while the kernel's source file still has
the recorded SHA-256.

usage: python -m paper_2509_21694_amd.traffic_summary FETCH_CSV WRITE_CSV MIB "command text"
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the edge kernels' translation unit and the headers it includes
SOURCES = ["paper_2509_21694_amd/csrc/k_fast.hip", "paper_2509_21694_amd/csrc/edge_common.h",
           "paper_2509_21694_amd/csrc/kernels.h", "paper_2509_21694_amd/csrc/common.h"]


def sources_sha256(root):
    h = hashlib.sha256()
    for rel in SOURCES:
        h.update(open(os.path.join(root, rel), "rb").read())
    return h.hexdigest()
# phase name in the engine's timer -> kernel symbol pattern (BF16 form)
PHASES = {
    "edge_fwd_t1": r"k_l1_fwd<1,",
    "edge_bwd_t1": r"k_l1_bwd<1,",
    "edge_fwd_t2": r"k_l2_msg<",
    "edge_sum_t2": r"k_l2_msum<",
    "edge_bwd_t2": r"k_l2_adj<",
}
COPY = r"copyBuffer"


def per_kernel(path, counter):
    """Counter values of every dispatch, by kernel name."""
    vals = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return vals


def mean_of(d, pat):
    """Mean over the large dispatches (at least half the largest) of the
    kernel matching pat: the run also evaluates smaller systems."""
    hits = [v for k, v in d.items() if re.search(pat, k.replace(" ", ""))]
    if not hits:
        return None
    v = max(hits, key=len)
    big = [x for x in v if x >= 0.5 * max(v)]
    return sum(big) / len(big)


def largest_of(d, pat):
    """The largest single dispatch among kernels matching pat (the calibration copy)."""
    hits = [x for k, v in d.items() if re.search(pat, k.replace(" ", "")) for x in v]
    return max(hits) if hits else None


def main():
    fetch_csv, write_csv, mib, cmd = sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4]
    fe, wr = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    known_kib = mib * 1024.0
    cf, cw = largest_of(fe, COPY), largest_of(wr, COPY)
    sf, sw = known_kib / cf, known_kib / cw
    sha = sources_sha256(ROOT)
    print("# HBM traffic per launch of the edge kernels, bulk1m (BF16 form)\n")
    print("Commands (run from the repository root on one MI355X, `cd /tmp` first for rocprofv3):\n")
    print("```\n" + cmd + "\n```\n")
    print(f"Copy calibration: {mib} MiB copied; FETCH_SIZE read {cf:.0f} KiB (factor {sf:.4f}), "
          f"WRITE_SIZE {cw:.0f} KiB (factor {sw:.4f}).\n")
    print("| Phase | FETCH KiB | WRITE KiB | scaled bytes per launch |")
    print("|---|---|---|---|")
    lines = []
    for ph, pat in PHASES.items():
        f, w = mean_of(fe, pat), mean_of(wr, pat)
        if f is None or w is None:
            continue
        b = f * sf * 1024 + w * sw * 1024
        print(f"| {ph} | {f:.0f} | {w:.0f} | {b:.4g} |")
        lines.append(json.dumps({"phase": ph, "bytes_per_launch": b, "fetch_kib": f, "write_kib": w,
                                 "sources_sha256": sha}))
    print()
    for ln in lines:
        print("TRAFFIC_JSON: " + ln)


if __name__ == "__main__":
    main()
