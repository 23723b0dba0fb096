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
Extra fields: `md` (on-device MD steps with neighbour-list reuse),
`depth_pruning` (a 13,824-atom box, one 6-layer weight set run to K = 6
and to K = 2) and `partitioned` (a whole 8,000,000-atom box evaluated as 8
slab partitions one after the other, geometric and graph halos, with the
halo growth against depth).
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


def phase_counts(hp, prec):
    """Algorithmic work of the specialised first/last-layer edge kernels, per
    directed edge and per atom, for the formulation they implement (live
    paths only, nothing recomputed is counted): {phase: (mfma_flop/edge,
    valu_flop/edge, bytes/edge, bytes/atom)}.  Bytes are each array read or
    written once per launch (unique bytes, not per-edge gathers)."""
    C, L, H, nb, S = hp.channels, hp.l_max, hp.radial_hidden, hp.n_basis, hp.n_species
    nlm, P = (L + 1) ** 2, L + 1
    fb = 2 if prec == "bf16" else 4            # storage of Q/P and h~ in the form
    mlp12, mlp3 = nb * H + H * H, H * P * C
    ev, src, grw = 16, 4, 32                   # e_vec, e_src, g read+write
    d = {
        # Q_i += a2 (x) YC over the row: layers 1-2 of the MLP and the outer product
        "edge_fwd_t1": (2 * (mlp12 + H * nlm), 0.0, ev, 8 + nlm * 64 * S * fb),
        # MLP adjoint through layers 2, 1; dE/da2 = P^T Ysel; dE/dYC = P a2
        "edge_bwd_t1": (2 * (mlp12 + 2 * H * nlm), 0.0, ev + grw, 8 + nlm * 64 * S * fb),
        # full MLP; s_l = <h~_j,l , YC_l> (nlm FMA/channel) and A += R s (P FMA/channel)
        "edge_fwd_t2": (2 * (mlp12 + mlp3), 2.0 * C * (nlm + P), ev + src, 8 + nlm * C * fb + C * 4),
        # MLP adjoint (W3, W2, W1); s (nlm FMA), dYC (nlm FMA), dR and R dA (2P mul) per channel
        "edge_bwd_t2": (2 * (mlp12 + mlp3), C * (4.0 * nlm + 2 * P), ev + src + grw, 8 + nlm * C * fb + C * 4),
        # h~bar_i = sum_e YC^T (R dA_j): nlm MAC per channel on MFMA; R dA_j: P mul per channel
        "edge_pull_t2": (2.0 * nlm * C, 1.0 * P * C, ev + src, 8 + C * 4 + nlm * C * 4),
    }
    if prec == "bf16":
        # one fused adjoint over the reverse edges: the MLP adjoint, and
        # s_l = <h~_i,l , YC_l>, dYC and the pull (nlm MAC per channel each) on
        # MFMA; dR and R dA_j (P mul per channel each) on the VALU; e_rev read
        # per edge; h~_i read and h~bar_i written (BF16) once per atom
        d["edge_bwd_t2"] = (2 * (mlp12 + mlp3) + 6.0 * nlm * C, 2.0 * P * C, ev + 2 * src + grw,
                            8 + nlm * C * fb + C * 4 + nlm * C * fb)
        del d["edge_pull_t2"]
        # forward as sender-side messages: full MLP, X_l = <h~_j,l , YC_l> on
        # MFMA (nlm MAC per channel), m = sum_l R_l X_l on the VALU (P FMA per
        # channel); the message (C BF16) written once per edge; h~_j read once per atom
        d["edge_fwd_t2"] = (2 * (mlp12 + mlp3) + 2.0 * nlm * C, 2.0 * P * C, ev + src + 2 * C,
                            8 + nlm * C * fb)
        # A_i = sum over the row of the messages: C BF16 read per edge, C FP32 written per atom
        d["edge_sum_t2"] = (0.0, 1.0 * C, 2 * C, 8 + 4 * C)
    return d


def kernel_roofline(name, t, hp, prec, n_edges, n_atoms):
    counts = phase_counts(hp, prec)
    if name not in counts:
        return None
    fm, fv, be, ba = counts[name]
    peak_m = PEAK["mfma_bf16"] if prec == "bf16" else PEAK["mfma_fp32"]
    work = {"mfma": fm * n_edges, "alu": fv * n_edges, "hbm": be * n_edges + ba * n_atoms}
    peak = {"mfma": peak_m, "alu": PEAK["alu_fp32"], "hbm": PEAK["hbm"]}
    times = {k: work[k] / peak[k] for k in work}
    bound = max(times, key=times.get)
    unit = "GB/s" if bound == "hbm" else "TFLOP/s"
    scale = 1e-9 if bound == "hbm" else 1e-12
    return {"kernel": name, "bound": bound, "achieved": round(work[bound] / t * scale, 3),
            "peak": round(peak[bound] * scale, 3), "unit": unit, "frac": round(work[bound] / t / peak[bound], 4),
            "avg_ms": round(t * 1e3, 4), "work_per_launch": work[bound],
            "roof_ms": {k: round(v * 1e3, 4) for k, v in times.items()}}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "edge_traffic_bulk1m.md")


def measured_traffic(kernel_phase):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, or None when there is none for it or its sources have changed."""
    from paper_2509_21694_amd.traffic_summary import sources_sha256
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if not ln.startswith("TRAFFIC_JSON: "):
            continue
        d = json.loads(ln[len("TRAFFIC_JSON: "):])
        if d.get("phase") != kernel_phase:
            continue
        return d["bytes_per_launch"] if d.get("sources_sha256") == sources_sha256(ROOT) else None
    return None


def roofline_entry(phases, hp, n_edges, prec, n_atoms):
    """Roofline of the edge kernel with the largest share of the step, plus
    the same figures for every specialised edge kernel."""
    per = {}
    for k, (ms_total, calls) in phases.items():
        r = kernel_roofline(k, ms_total / calls * 1e-3, hp, prec, n_edges, n_atoms)
        if r is not None:
            per[k] = r
    if not per:
        return None
    name = max(per, key=lambda k: phases[k][0])
    top = dict(per[name])
    top["traffic"] = measured_traffic(name) if prec == "bf16" else None
    top["kernels"] = {k: {"bound": v["bound"], "frac": v["frac"], "avg_ms": v["avg_ms"]} for k, v in per.items()}
    return top


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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy MIB mebibytes device to device once before the steps (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--md-steps", type=int, default=10,
                    help="also time this many on-device MD steps (first precision; 0: skip)")
    ap.add_argument("--depth-steps", type=int, default=5,
                    help="also time the 13,824-atom box at K=6 and K=2 of one 6-layer weight set (0: skip)")
    ap.add_argument("--partitioned-steps", type=int, default=2,
                    help="also time this many evaluations of the 8M-atom box as 8 slab partitions (0: skip)")
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

    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read and written")
        del src, dst

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
    md = None
    if args.md_steps > 0:
        # velocity Verlet around the evaluation (mpip_md_run), neighbour list of
        # radius r_c + 0.5 A reused until an atom has moved 0.25 A
        x = pos_sets[0].clone()
        v = torch.tensor(W.velocities(N, 0.005, 12), dtype=torch.float64, device=dev)
        ms_t = torch.tensor(W.MASSES_LPO, dtype=torch.float64, device=dev)
        cap = int(results[head]["n_edges"] * 1.02) + 4096
        F = model.evaluate(x, species, s.cell, s.pbc, K=K, precision=head, max_edges=cap)["forces"]
        _, _, F = model.md_run(x, v, species, ms_t, s.cell, s.pbc, dt=1.0, n_steps=2, forces=F, skin=0.5, K=K,
                               precision=head, max_edges=cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ep, ek, F = model.md_run(x, v, species, ms_t, s.cell, s.pbc, dt=1.0, n_steps=args.md_steps, forces=F,
                                 skin=0.5, K=K, precision=head, max_edges=cap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        et = (ep + ek).cpu().numpy()
        md_ms = (t1 - t0) / args.md_steps * 1e3
        log(f"md ({head}): {md_ms:.3f} ms/step")
        md = {"metric": "MD atom-steps/s (velocity Verlet on the device, dt 1 fs, neighbour list reused "
                        "within a 0.5 A skin)", "value": round(N / (md_ms * 1e-3), 1),
              "us_per_atom_step": round(md_ms * 1e3 / N, 6), "ms_per_step": round(md_ms, 4),
              "steps": args.md_steps, "dtype": head,
              "energy_drift_per_atom": float(np.abs(et - et[0]).max() / N)}
    depth = None
    if args.depth_steps > 0:
        # message-passing depth pruning: the same 6-layer weight set evaluated
        # to K = 6 and truncated to K = 2 (13,824-atom box, l_max = 2, C = 64)
        sd, hpd = W.mpdp_system(), W.HP_MPDP
        modeld = M.Model(hpd, W.make_weights(hpd, W.WEIGHT_SEEDS["mpdp"]))
        pd = torch.tensor(sd.positions, dtype=torch.float64, device=dev)
        spd = torch.tensor(sd.species, dtype=torch.int32, device=dev)
        depth = {"metric": "ms per E+F evaluation of a 13,824-atom box, one 6-layer weight set run to K layers",
                 "n_atoms": sd.n_atoms, "steps": args.depth_steps}
        for prec in precs:
            row = {}
            for Kd in (6, 2):
                o = modeld.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec)
                cap = int(o["n_edges"] * 1.02) + 4096
                modeld.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec, max_edges=cap, out=o, check=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.depth_steps):
                    modeld.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec, max_edges=cap, out=o,
                                    check=False)
                torch.cuda.synchronize()
                row[f"K{Kd}_ms"] = round((time.perf_counter() - t0) / args.depth_steps * 1e3, 3)
            row["K6_over_K2"] = round(row["K6_ms"] / row["K2_ms"], 2)
            depth[prec] = row
            log(f"depth pruning ({prec}): K=6 {row['K6_ms']} ms, K=2 {row['K2_ms']} ms")
        del modeld, pd, spd
    part = None
    if args.partitioned_steps > 0:
        # one-GPU partitioned mode: the whole 200^3 box in 8 slabs along x,
        # halo K r_cut, each share built, evaluated (trimmed) and integrated
        # on the device one after the other (mpip_evaluate_partitioned)
        Kp, n_parts = 2, 8
        s8 = W.slab_full_system(200, 200, 200, 401, 402)
        hp8 = W.HP_MPDP
        model8 = M.Model(hp8, W.make_weights(hp8, W.WEIGHT_SEEDS["slab8m"]))
        p8 = torch.tensor(s8.positions, dtype=torch.float64, device=dev)
        sp8 = torch.tensor(s8.species, dtype=torch.int32, device=dev)
        o8 = model8.evaluate_partitioned(p8, sp8, s8.cell, s8.pbc, n_parts=n_parts, K=Kp, precision=head)
        parts = o8["parts"]
        ml, me = int(parts[:, 0].max() * 1.02) + 1024, int(parts[:, 2].max() * 1.02) + 4096
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.partitioned_steps):
            model8.evaluate_partitioned(p8, sp8, s8.cell, s8.pbc, n_parts=n_parts, K=Kp, precision=head,
                                        max_local=ml, max_edges=me)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p_ms = (t1 - t0) / args.partitioned_steps * 1e3
        log(f"partitioned ({head}): {p_ms:.3f} ms per 8M-atom evaluation")
        part = {"metric": "atom-steps/s of a whole 8,000,000-atom box evaluated as 8 slab partitions one after "
                          "the other on one GPU (K=2, l_max=2, C=64, halo 2 r_cut, trimmed shares)",
                "value": round(s8.n_atoms / (p_ms * 1e-3), 1), "ms_per_step": round(p_ms, 3),
                "steps": args.partitioned_steps, "dtype": head, "n_parts": n_parts,
                "halo_growth_H": round(float(parts[:, 0].sum()) / s8.n_atoms - 1.0, 4),
                "share_rows_max": int(parts[:, 0].max()), "share_edges_max": int(parts[:, 2].max())}
        # the same with the K-hop graph halo (whole-structure list once, hops per part)
        og = model8.evaluate_partitioned(p8, sp8, s8.cell, s8.pbc, n_parts=n_parts, K=Kp, precision=head,
                                         graph_halo=True, max_local=ml, max_edges=me)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.partitioned_steps):
            og = model8.evaluate_partitioned(p8, sp8, s8.cell, s8.pbc, n_parts=n_parts, K=Kp, precision=head,
                                             graph_halo=True, max_local=ml, max_edges=me)
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - t0) / args.partitioned_steps * 1e3
        log(f"partitioned, graph halo ({head}): {g_ms:.3f} ms per 8M-atom evaluation")
        part["graph_halo"] = {"value": round(s8.n_atoms / (g_ms * 1e-3), 1), "ms_per_step": round(g_ms, 3),
                              "halo_growth_H": round(float(og["parts"][:, 0].sum()) / s8.n_atoms - 1.0, 4)}
        # halo growth of one share against depth: geometric K r_cut vs K hops
        hg = {}
        for Kh in (2, 6):
            gp, _, _, no = M.slab_share(p8, sp8, s8.cell, n_parts, 0, Kh * hp8.r_cut)
            nl_geo = int(gp.shape[0])
            del gp
            nl_bfs = int(M.bfs_share(p8, sp8, s8.cell, n_parts, 0, Kh, hp8.r_cut)[0].shape[0])
            hg[f"K{Kh}"] = {"geometric": round((nl_geo - no) / no, 4), "graph": round((nl_bfs - no) / no, 4)}
        part["halo_growth_vs_K"] = hg
        del model8, p8, sp8, o8, og
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
            "forms": results,
            "md": md,
            "depth_pruning": depth,
            "partitioned": part}
    if "bf16" in results and "fp32" in results:
        line["bf16_speedup_over_fp32"] = round(results["fp32"]["ms_per_step"] / results["bf16"]["ms_per_step"], 3)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
