"""Turn rocprofv3 counter runs (`--pmc ... --output-format csv`) of
`bench.py` into a per-kernel markdown table of utilisation figures.

Each CSV holds one row per (dispatch, counter).  Per kernel the dispatches
of at least half the largest GRBM_GUI_ACTIVE are averaged (the run also
evaluates smaller systems).  GRBM_GUI_ACTIVE is summed over the 8 XCDs in
the CSV, so one dispatch lasts GRBM_GUI_ACTIVE / 8 GPU cycles; utilisations
are per SIMD (1024) or per CU (256) over that time:
  MFMA busy   = SQ_VALU_MFMA_BUSY_CYCLES / (cycles * 1024)
  VALU active = SQ_ACTIVE_INST_VALU / (cycles * 256)   (quad-cycles, summed over the waves of a CU: above 100 % when several waves' VALU instructions are in flight together)
  co-issue    = SQ_VALU_MFMA_COEXEC_CYCLES / (cycles * 1024)
  LDS bank conflict = SQ_LDS_BANK_CONFLICT / (cycles * 256)
  waves/SIMD  = 4 SQ_WAVE_CYCLES / (cycles * 1024)      (quad-cycles)
  wait        = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES

usage: python -m paper_2509_21694_amd.counter_summary "command text" CSV [CSV ...]
       python -m paper_2509_21694_amd.counter_summary --trace "title" "command text" KERNEL_TRACE_CSV
(the second form: per-kernel dispatch times from a --kernel-trace run)
"""
from __future__ import annotations

import collections
import csv
import re
import sys

KERNELS = collections.OrderedDict([
    ("k_l2_adj", r"k_l2_adj<"), ("k_l2_msg", r"k_l2_msg<"), ("k_l2_msum", r"k_l2_msum<"),
    ("k_l1_fwd", r"k_l1_fwd<"), ("k_l1_bwd", r"k_l1_bwd<"), ("k_node1_fwd", r"k_node1_fwd<"),
    ("k_node1_bwd", r"k_node1_bwd<"), ("k_nodeK", r"k_nodeK<"), ("k_nbr_w (count)", r"k_nbr_w<false>"),
    ("k_nbr_w (fill)", r"k_nbr_w<true>"), ("k_nbr_rev", r"k_nbr_rev"), ("k_forces", r"k_forces"),
    ("k_l2_msg32", r"k_l2_msg32<"), ("k_l2_adj32", r"k_l2_adj32<"), ("k_l2_msum32", r"k_l2_msum32<"),
    ("k_gemm_lds", r"k_gemm_lds<"),
])
SIMD, CU, XCD = 1024, 256, 8


def collect(paths):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    for path in paths:
        disp, kname = collections.defaultdict(dict), {}
        with open(path) as f:
            for row in csv.DictReader(f):
                name = row["Kernel_Name"].replace(" ", "")
                for k, pat in KERNELS.items():
                    if re.search(pat, name):
                        disp[row["Dispatch_Id"]][row["Counter_Name"]] = float(row["Counter_Value"])
                        kname[row["Dispatch_Id"]] = k
                        meta[k] = (row.get("Scratch_Size"), row.get("LDS_Block_Size"))
                        break
        top = collections.defaultdict(float)
        for d, cv in disp.items():
            top[kname[d]] = max(top[kname[d]], cv.get("GRBM_GUI_ACTIVE", 0.0))
        for d, cv in disp.items():
            if cv.get("GRBM_GUI_ACTIVE", 0.0) >= 0.5 * top[kname[d]]:
                for c, x in cv.items():
                    vals[kname[d]][c].append(x)
    return vals, meta


def main():
    cmd, paths = sys.argv[1], sys.argv[2:]
    vals, meta = collect(paths)
    print("# Per-kernel counters, bulk1m (1,000,000 atoms, K = 2, l_max = 2, C = 128)\n")
    print("Commands (run from the repository root on one MI355X, `cd /tmp` first for rocprofv3):\n")
    print("```\n" + cmd + "\n```\n")
    defs = __doc__.split("over that time:")[1].split("usage:")[0].strip().splitlines()
    print("Utilisation per SIMD (1024) or per CU (256) over the dispatch's GRBM_GUI_ACTIVE / 8 cycles:\n")
    print("\n".join("- " + d.strip() for d in defs) + "\n")
    cols = ["kernel", "time ms", "MFMA busy", "VALU active", "co-issue", "waves/SIMD", "wait/wave", "LDS conflict",
            "VALU instr/wave", "MFMA instr/wave", "trans/VALU", "scratch B/lane", "LDS B/workgroup"]
    print("| " + " | ".join(cols) + " |")
    print("|" + "---|" * len(cols))
    for k in KERNELS:
        if k not in vals:
            continue
        v = {c: sum(x) / len(x) for c, x in vals[k].items()}
        cyc = v.get("GRBM_GUI_ACTIVE", 0.0) / XCD
        if cyc <= 0:
            continue

        def frac(c, n):
            return f"{100.0 * v[c] / (cyc * n):.1f}%" if c in v else "-"
        waves = v.get("SQ_WAVES")
        row = [k, f"{cyc / 2.4e6:.3f}" if cyc else "-", frac("SQ_VALU_MFMA_BUSY_CYCLES", SIMD),
               frac("SQ_ACTIVE_INST_VALU", CU), frac("SQ_VALU_MFMA_COEXEC_CYCLES", SIMD),
               f"{4.0 * v['SQ_WAVE_CYCLES'] / (cyc * SIMD):.2f}" if "SQ_WAVE_CYCLES" in v else "-",
               f"{v['SQ_WAIT_INST_ANY'] / v['SQ_WAVE_CYCLES']:.2f}" if "SQ_WAIT_INST_ANY" in v and "SQ_WAVE_CYCLES" in v else "-",
               frac("SQ_LDS_BANK_CONFLICT", CU),
               f"{v['SQ_INSTS_VALU'] / waves:.4g}" if waves and "SQ_INSTS_VALU" in v else "-",
               f"{v['SQ_INSTS_MFMA'] / waves:.4g}" if waves and "SQ_INSTS_MFMA" in v else "-",
               f"{v['SQ_INSTS_VALU_TRANS_F32'] / v['SQ_INSTS_VALU']:.3f}" if "SQ_INSTS_VALU_TRANS_F32" in v and "SQ_INSTS_VALU" in v else "-"]
        m = meta.get(k, ("-",) * 2)
        row += [str(x) for x in m]
        print("| " + " | ".join(row) + " |")
    print("\n(time: GRBM_GUI_ACTIVE / 8 at 2.4 GHz; counters of one pass per group, averaged over the large dispatches)")


def trace_main():
    title, cmd, path = sys.argv[2], sys.argv[3], sys.argv[4]
    t = collections.defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            t[row["Kernel_Name"]].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-3)
    total = sum(sum(v) for v in t.values())
    print(f"# Kernel time per dispatch, {title}\n")
    print("Command (run from the repository root on one MI355X):\n")
    print("```\n" + cmd + "\n```\n")
    print(f"Total kernel time {total * 1e-3:.2f} ms over all dispatches.\n")
    print("| Kernel | Calls | Total ms | Avg us | Min us | Max us | % |")
    print("|---|---|---|---|---|---|---|")
    for name, v in sorted(t.items(), key=lambda kv: -sum(kv[1])):
        nm = name if len(name) <= 90 else name[:87] + "..."
        print(f"| `{nm}` | {len(v)} | {sum(v) * 1e-3:.3f} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
              f"{100.0 * sum(v) / total:.2f} |")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--trace":
        trace_main()
    else:
        main()
