#!/usr/bin/env python3
"""Throughput of one energy + forces + virial evaluation on one MI355X.

Workload (default): 1,000,000-atom periodic box (100^3 jittered simple-cubic
lattice at 0.085 atoms/A^3, 3 species 0.5/0.3/0.2), cutoff 5 A, 2
message-passing layers, l_max = 2, 128 channels, radial MLP 8->64->64->paths.
One step = one complete evaluation through the C ABI (cell list, neighbour
list, both layers forward, readout, the hand-written adjoint with edge
intermediates recomputed, forces, virial); inputs are resident in HBM and
two slightly different position sets (+-0.01 A) alternate between steps.

Prints ONE JSON line.  `value` is the BF16-form rate (atom-steps/s); the
FP32-form rate, the BF16 speedup and the force error of both forms against
the FP64 oracle (at atoms whose oracle forces are exact, from a local
cluster) are extra fields.  `roofline` is for the kernel with the largest
share of the step (HIP-event durations from the timed steps);
`cpu_baseline` times the FP64 oracle on a bounded cluster of the same box.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "atom-steps/s (E+F) at 1M atoms, BF16 vs FP32 form on 1 GPU; force RMS vs FP64"

# MI355X published peaks
PEAK = {"hbm": 8.0e12, "mfma_bf16": 2.5e15, "mfma_fp32": 157.3e12, "alu_fp32": 157.3e12}


def workload(name):
    if name == "bulk1m":
        return W.bulk1m_system(), W.HP_BULK, W.WEIGHT_SEEDS["bulk1m"], 2
    if name == "mpdp":
        return W.mpdp_system(), W.HP_MPDP, W.WEIGHT_SEEDS["mpdp"], 2
    if name == "small":
        return W.small_system(), W.HP_SMALL, W.WEIGHT_SEEDS["small"], 2
    raise SystemExit(f"unknown workload {name}")


def edge_kernel_counts(hp, kind):
    """Algorithmic work per directed edge of one fused edge kernel (live
    paths only, no recompute): (mfma_flop, valu_flop, hbm_bytes).
    kind: 'fwd_first', 'fwd_last', 'bwd_first', 'bwd_last'."""
    C, L, H, nb = hp.channels, hp.l_max, hp.radial_hidden, hp.n_basis
    P = L + 1
    nlm = (L + 1) ** 2
    mlp = nb * H + H * H + H * P * C
    if kind == "fwd_first":     # R_e, then A_i[c, lm] += R_l h_z(j) Y_lm / sqrt(2l+1)
        valu = C * (P + nlm)
        hbm = 16 + 4                       # edge vector + sender index
    elif kind == "fwd_last":    # s_l = <ht_j,l , Y_l>, A_i[c] += sum_l R_l s_l
        valu = C * (nlm + P)
        hbm = 16 + 4 + nlm * C * 4         # gathered ht_j (FP32)
    elif kind == "bwd_first":   # dR_l = sum_m dA_i,lm Y_lm h ; dY_lm = sum_c R_l h dA_i,lm
        valu = C * 2 * (nlm + P)
        hbm = 16 + 4 + 16
    else:                       # bwd_last: dR, dY and the sender-side pull through the reverse edge
        valu = C * 3 * (nlm + P)
        hbm = 16 + 4 + 16 + nlm * C * 4 + C * 4
    return 2.0 * mlp, 2.0 * valu, float(hbm)


def roofline_entry(phases, hp, n_edges, prec, n_atoms):
    """Roofline of the edge kernel with the largest share of the step."""
    cand = {k: v for k, v in phases.items() if k.startswith("edge_")}
    name = max(cand, key=lambda k: cand[k][0] / max(1, cand[k][1]))
    ms_total, calls = cand[name]
    t = ms_total / calls * 1e-3
    layer = int(name.split("_t")[-1])
    kind = ("fwd_" if "fwd" in name else "bwd_") + ("first" if layer == 1 else "last")
    fm, fv, b = edge_kernel_counts(hp, kind)
    # node-level bytes are shared by all edges of a row: add them per launch
    nlm = (hp.l_max + 1) ** 2
    node_bytes = n_atoms * (nlm * hp.channels * 4 + 8)
    peak_m = PEAK["mfma_bf16"] if prec == "bf16" else PEAK["mfma_fp32"]
    times = {"mfma": fm * n_edges / peak_m, "alu": fv * n_edges / PEAK["alu_fp32"],
             "hbm": (b * n_edges + node_bytes) / PEAK["hbm"]}
    bound = max(times, key=times.get)
    work = {"mfma": fm * n_edges, "alu": fv * n_edges, "hbm": b * n_edges + node_bytes}[bound]
    peak = {"mfma": peak_m, "alu": PEAK["alu_fp32"], "hbm": PEAK["hbm"]}[bound]
    unit = "GB/s" if bound == "hbm" else "TFLOP/s"
    scale = 1e-9 if bound == "hbm" else 1e-12
    achieved = work / t
    return {"kernel": name, "bound": bound, "achieved": round(achieved * scale, 3),
            "peak": round(peak * scale, 3), "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": None, "avg_ms": round(t * 1e3, 4),
            "work_per_launch": work, "roof_ms": {k: round(v * 1e3, 4) for k, v in times.items()}}


def cpu_baseline(s, hp, blob, K, radius):
    """FP64 oracle on one non-periodic cluster cut from the same box.

    Energies are summed over the atoms within radius - K r_c of the center
    (their environments are complete); the forces of atoms within
    radius - 2 K r_c are then exact full-system forces."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    center = s.n_atoms // 2 + 17
    lp, ls, n_in, gi, c = oracle.local_cluster(s.positions, s.species, s.cell, center, radius,
                                               radius - K * hp.r_cut)
    t0 = time.time()
    res = oracle.evaluate(lp, ls, np.eye(3), [False] * 3, blob, hp, K=K, n_owned=n_in)
    dt = time.time() - t0
    dist = np.linalg.norm(lp - lp[c], axis=1)
    exact = np.flatnonzero(dist <= radius - 2 * K * hp.r_cut)
    return {"value": round(lp.shape[0] / dt, 3), "unit": "atom-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{lp.shape[0]}-atom non-periodic cluster (radius {radius:g} A) cut from the "
                      f"same box, FP64 energy+forces of all its atoms, {dt:.1f} s"}, \
        (gi[exact], res.forces[exact])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bulk1m")
    ap.add_argument("--precisions", default="bf16,fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cluster-radius", type=float, default=24.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the halo-partition design for several GPUs is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_21694_amd as M

    s, hp, wseed, K = workload(args.workload)
    blob = W.make_weights(hp, wseed)
    model = M.Model(hp, blob)
    dev = torch.device("cuda", 0)
    pos_sets = [torch.tensor(s.positions, dtype=torch.float64, device=dev),
                torch.tensor(W.rejitter(s.positions, 11), dtype=torch.float64, device=dev)]
    species = torch.tensor(s.species, dtype=torch.int32, device=dev)
    N = s.n_atoms

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    base = {}
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle on a cluster) ...")
        base, exact = cpu_baseline(s, hp, blob, K, args.cluster_radius)
        log(f"cpu baseline: {base['value']} atom-steps/s on {base['cores']} threads")
    results = {}
    precs = [p for p in args.precisions.split(",") if p]
    for prec in precs:
        o = model.evaluate(pos_sets[0], species, s.cell, s.pbc, K=K, precision=prec)
        n_edges = o["n_edges"]
        cap = int(n_edges * 1.02) + 4096
        F0 = o["forces"].cpu().numpy()
        E0 = float(o["energy"].cpu()[0])
        outs = [model.evaluate(p, species, s.cell, s.pbc, K=K, precision=prec, max_edges=cap)
                for p in pos_sets]
        for k in range(args.warmup):
            model.evaluate(pos_sets[k % 2], species, s.cell, s.pbc, K=K, precision=prec, max_edges=cap,
                           out=outs[k % 2], check=False)
        M.lib.mpip_timing_enable(model._h, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            model.evaluate(pos_sets[k % 2], species, s.cell, s.pbc, K=K, precision=prec, max_edges=cap,
                           out=outs[k % 2], check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm = M.read_timing(model)
        M.lib.mpip_timing_enable(model._h, 0)
        st = M.workspace_status(model)
        if st != 0:
            raise SystemExit(f"evaluation reported status {st}: {M.lib.mpip_last_error().decode()}")
        ms = (t1 - t0) / args.steps * 1e3
        log(f"{prec}: {ms:.3f} ms/step, {n_edges} edges")
        r = {"ms_per_step": round(ms, 4), "value": round(N / (ms * 1e-3), 1), "n_edges": n_edges,
             "energy": E0, "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in tm.items()},
             "roofline": roofline_entry(tm, hp, n_edges, prec, N)}
        if base:
            gi, Fx = exact
            d = F0[gi] - Fx
            r["force_err_vs_fp64"] = {"rms": float(np.sqrt(np.mean(d ** 2))), "max": float(np.abs(d).max()),
                                      "ref_rms": float(np.sqrt(np.mean(Fx ** 2))), "atoms": int(gi.size)}
        results[prec] = r

    head = precs[0]
    line = {"metric": METRIC, "value": results[head]["value"], "unit": "atom-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": results[head]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": head,
            "data": "synthetic",
            "config": {"workload": f"{args.workload}: {N}-atom jittered simple-cubic periodic box, density 0.085/A^3, "
                                   f"3 species, r_cut 5 A, K={K} layers, l_max={hp.l_max}, C={hp.channels}, "
                                   f"radial MLP 8-64-64-paths",
                       "n_atoms": N, "n_edges": results[head]["n_edges"], "K": K, "l_max": hp.l_max,
                       "channels": hp.channels, "precision": head},
            "roofline": results[head]["roofline"],
            "cpu_baseline": base or None,
            "forms": results}
    if "bf16" in results and "fp32" in results:
        line["bf16_speedup_over_fp32"] = round(results["fp32"]["ms_per_step"] / results["bf16"]["ms_per_step"], 3)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
