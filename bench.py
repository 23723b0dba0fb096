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
FP32-form rate, the BF16 speedup and the errors of both forms against stored
FP64 oracle values (`errors_vs_fp64`: energies and forces of the 1M-atom box
where local clusters give them exactly; energy, forces and stress of every
atom of a 32,768-atom box with the same potential) are extra fields.
`roofline` is for the kernel with the largest share of the step (HIP-event
durations from the timed steps); `step_roofline` sums the roofline times of
every phase of the step over the measured step time; `cpu_baseline` times the
FP64 oracle on a periodic box of the same lattice and potential, on all host
cores and on one.  Extra fields: `md` (on-device MD steps with
neighbour-list reuse), `depth_pruning` (a 13,824-atom box, one 6-layer
weight set run to K = 6 and to K = 2, with per-layer times), `partitioned`
(a whole 8,000,000-atom box evaluated as 8 slab partitions one after the
other, geometric and graph halos, the halo growth against depth, and one
share evaluated at K = 2 and K = 6) and `batch512` (512 independent small
cells evaluated together, both forms).
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

# MI355X published peaks.  The published FP32 vector peak (157.3 TFLOP/s)
# counts packed FMA; every kernel here is compiled with packed FP32 off, so
# the VALU ceiling used is the unpacked rate: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flop x 2.4 GHz = 78.6 TFLOP/s.
PEAK = {"hbm": 8.0e12, "mfma_bf16": 2.5e15, "mfma_fp32": 157.3e12, "alu_fp32": 78.6e12}


def workload(name):
    if name == "bulk1m":
        return W.bulk1m_system(), W.HP_BULK, W.WEIGHT_SEEDS["bulk1m"], 2
    if name == "mpdp":
        return W.mpdp_system(), W.HP_MPDP, W.WEIGHT_SEEDS["mpdp"], 2
    if name == "small":
        return W.small_system(), W.HP_SMALL, W.WEIGHT_SEEDS["small"], 2
    raise SystemExit(f"unknown workload {name}")


def phase_counts(hp, prec):
    """Algorithmic work of the step's phases, per directed edge and per atom,
    for the formulation they implement (live paths only, nothing recomputed
    is counted): {phase: (mfma_flop/edge, valu_flop/edge, bytes/edge,
    bytes/atom[, mfma_flop/atom])}.  Bytes are each array read or written
    once per launch (unique bytes, not per-edge gathers)."""
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
        # last layer, sender side (both forms): messages with the full MLP,
        # X_l = <h~_j,l , YC_l> on MFMA (nlm MAC per channel), m = sum_l R_l X_l
        # on the VALU (P FMA per channel); h~_j read once per atom, e_vec, e_rev
        # read per edge.  The per-edge messages this form writes (and the sum
        # reads back) are not algorithmic bytes of the layer: they count in the
        # measured traffic only
        "edge_fwd_t2": (2 * (mlp12 + mlp3) + 2.0 * nlm * C, 2.0 * P * C, ev + src, 8 + nlm * C * fb),
        # A_i = sum over the row of the messages: C adds per edge; A_i (C FP32) written per atom
        "edge_sum_t2": (0.0, 1.0 * C, 0, 8 + 4 * C),
        # one fused adjoint over the reverse edges: the MLP adjoint, and
        # s_l = <h~_i,l , YC_l>, dYC and the pull (nlm MAC per channel each) on
        # MFMA; dR and R dA_j (P mul per channel each) on the VALU; e_rev read
        # per edge; h~_i read and h~bar_i written once per atom
        "edge_bwd_t2": (2 * (mlp12 + mlp3) + 6.0 * nlm * C, 2.0 * P * C, ev + 2 * src + grw,
                        8 + nlm * C * fb + C * 4 + nlm * C * fb),
    }
    if prec == "bf16":
        # fused node kernels between the two layers, forward and adjoint
        # (one phase): z = Q (VW) and h~ = h W_up forward, h-bar = h~-bar W_up^T
        # and P = z-bar (VW)^T backward; Q read twice, P written, h_0 (FP32) and
        # h~ (BF16) written, h~-bar (BF16) read
        KQ = 64 * S
        zq = 2.0 * KQ * (C * (1 + L) + (nlm - 1) * C)
        up = 2.0 * nlm * C * C
        d["node_fused"] = (0.0, 0.0, 0, 3 * nlm * KQ * 2 + 4 * C + 2 * nlm * C * 2, 2 * (zq + up))
        # last-layer node update and its adjoint, with the message sum A_i =
        # sum over the row of the messages (C adds per edge; the messages are
        # intermediate, not algorithmic bytes): h_0 read, dE/dA written, E_i
        # written; z_0 = W_down^T A and dE/dA = W_down z-bar on MFMA
        d["node_last"] = (0.0, 1.0 * C, 0, 2 * 4 * C + 8, 2 * 2.0 * C * C)
    # neighbour list: positions and species read, the sorted copies, permutation
    # and row pointers written per atom; sender, shift, vector and reverse index
    # written per edge
    d["neighbors"] = (0.0, 0.0, 4 + 4 + 16 + 4, 28 + 28 + 8 + 4)
    # forces / virial: g, e_vec, e_rev read per edge; forces (FP64) and atom energy written per atom
    d["outputs"] = (0.0, 0.0, 16 + 16 + 4, 24 + 8 + 4 + 8)
    return d


def kernel_roofline(name, t, hp, prec, n_edges, n_atoms):
    counts = phase_counts(hp, prec)
    if name not in counts:
        return None
    fm, fv, be, ba, fma = (tuple(counts[name]) + (0.0,))[:5]
    peak_m = PEAK["mfma_bf16"] if prec == "bf16" else PEAK["mfma_fp32"]
    work = {"mfma": fm * n_edges + fma * n_atoms, "alu": fv * n_edges, "hbm": be * n_edges + ba * n_atoms}
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


def step_roofline(phases, steps, hp, n_edges, prec, n_atoms):
    """Whole-step figure: sum over the step's phases of each one's roofline
    time (largest of MFMA, VALU and HBM time of its algorithmic work) over
    the measured step time.  Phases without an algorithmic count are listed
    with their time and a roof of zero."""
    counts = phase_counts(hp, prec)
    peak_m = PEAK["mfma_bf16"] if prec == "bf16" else PEAK["mfma_fp32"]
    per, roof_sum, t_sum = {}, 0.0, 0.0
    for k, (ms_total, calls) in phases.items():
        ms = ms_total / steps
        t_sum += ms
        if k in counts:
            fm, fv, be, ba, fma = (tuple(counts[k]) + (0.0,))[:5]
            roof = max((fm * n_edges + fma * n_atoms) / peak_m, fv * n_edges / PEAK["alu_fp32"],
                       (be * n_edges + ba * n_atoms) / PEAK["hbm"]) * 1e3
        else:
            roof = 0.0
        roof_sum += roof
        per[k] = {"ms": round(ms, 4), "roof_ms": round(roof, 4), "frac": round(roof / ms, 4) if ms > 0 else None}
    return {"sum_roof_ms": round(roof_sum, 4), "step_ms": round(t_sum, 4),
            "frac": round(roof_sum / t_sum, 4) if t_sum > 0 else None, "phases": per}


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


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _force_errors(F, Fref):
    d = F - Fref
    ref_rms = float(np.sqrt(np.mean(Fref ** 2)))
    rms = float(np.sqrt(np.mean(d ** 2)))
    return {"rms": rms, "max": float(np.abs(d).max()), "ref_rms": ref_rms,
            "rel_rms": rms / ref_rms if ref_rms > 0 else None}


def errors_vs_fp64(name, model, prec, F, atom_e, K, dev):
    """Errors of one form against stored FP64 oracle values (written by
    tests/golden/make_golden.py from the oracle alone).  bulk1m: the atoms of
    eight local clusters whose oracle energies (about 7,900) and forces
    (about 180) equal the full-box values; bulk32k: a 32,768-atom periodic
    box with the same potential, every atom, energy, forces and stress."""
    import torch
    out = {}
    if name == "bulk1m":
        path = os.path.join(GOLDEN, "bulk1m_clusters.npz")
        if os.path.exists(path):
            g = np.load(path)
            dE = np.abs(atom_e[g["energy_index"]] - g["atom_energy"])
            fe = _force_errors(F[g["force_index"]], g["forces"])
            fe["atoms"] = int(g["force_index"].size)
            out["bulk1m_clusters"] = {"atom_energy_abs_mean_eV": float(dE.mean()),
                                      "atom_energy_abs_max_eV": float(dE.max()),
                                      "atoms_energy": int(dE.size), "forces_eV_per_A": fe}
    path = os.path.join(GOLDEN, "bulk32k_K2.npz")
    if os.path.exists(path) and model.hp == W.HP_BULK and K == 2:
        g = np.load(path)
        sb = W.bulk_system(32, 311, 312)
        pos = torch.tensor(sb.positions, dtype=torch.float64, device=dev)
        sp = torch.tensor(sb.species, dtype=torch.int32, device=dev)
        o = model.evaluate(pos, sp, sb.cell, sb.pbc, K=K, precision=prec)
        vol = float(abs(np.linalg.det(sb.cell)))
        Wg = o["virial"].cpu().numpy().reshape(3, 3)
        dW = np.abs(Wg - g["virial"]).max() / vol
        out["bulk32k"] = {"n_atoms": sb.n_atoms,
                          "energy_abs_per_atom_eV": abs(float(o["energy"].cpu()[0]) - float(g["energy"])) / sb.n_atoms,
                          "forces_eV_per_A": _force_errors(o["forces"].cpu().numpy(), g["forces"]),
                          "stress_abs_max_eV_per_A3": float(dW),
                          "stress_ref_max_eV_per_A3": float(np.abs(g["virial"]).max() / vol)}
    return out


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(hp, blob, K, n_side):
    """The FP64 oracle on a periodic n_side^3 box of the same lattice,
    density, species mix and potential (every atom fully coordinated, as in
    the 1M-atom box): neighbour list, forward and analytic backward, timed
    with BLAS on all host cores and again on one core."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    sb = W.bulk_system(n_side, 321, 322)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])

    def run():
        t0 = time.time()
        oracle.evaluate(sb.positions, sb.species, sb.cell, sb.pbc, blob, hp, K=K)
        return time.time() - t0

    dt_all = run()
    with threadpool_limits(limits=1):
        dt_one = run()
    return {"value": round(sb.n_atoms / dt_all, 3), "unit": "atom-steps/s", "cores": int(threads),
            "kind": "oracle", "value_1core": round(sb.n_atoms / dt_one, 3), "cpu_model": _cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"{sb.n_atoms}-atom periodic box ({n_side}^3 jittered lattice, the same density, species "
                      f"mix and potential as the workload), FP64 energy+forces+virial of every atom: "
                      f"{dt_all:.1f} s on {threads} BLAS threads, {dt_one:.1f} s on 1"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="bulk1m")
    ap.add_argument("--precisions", default="bf16,fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-box", type=int, default=12, help="side of the periodic box the oracle is timed on")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error statement against stored oracle values (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy MIB mebibytes device to device once before the steps (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    ap.add_argument("--md-steps", type=int, default=10,
                    help="also time this many on-device MD steps (first precision; 0: skip)")
    ap.add_argument("--depth-steps", type=int, default=5,
                    help="also time the 13,824-atom box at K=6 and K=2 of one 6-layer weight set (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10,
                    help="also time this many evaluations of 512 independent small cells (0: skip)")
    ap.add_argument("--partitioned-steps", type=int, default=2,
                    help="also time this many evaluations of the 8M-atom box as 8 slab partitions (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
        log("cpu baseline (FP64 oracle on a periodic box) ...")
        base = cpu_baseline(hp, blob, K, args.cpu_box)
        log(f"cpu baseline: {base['value']} atom-steps/s on {base['cores']} threads, "
            f"{base['value_1core']} on 1")
    results = {}
    precs = [p for p in args.precisions.split(",") if p]
    for prec in precs:
        o = model.evaluate(pos_sets[0], species, s.cell, s.pbc, K=K, precision=prec, atom_energy=True)
        n_edges = o["n_edges"]
        cap = int(n_edges * 1.02) + 4096
        F0 = o["forces"].cpu().numpy()
        E0 = float(o["energy"].cpu()[0])
        errors = None if args.no_errors else errors_vs_fp64(args.workload, model, prec, F0,
                                                             o["atom_energy"].cpu().numpy(), K, dev)
        del o
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
             "roofline": roofline_entry(tm, hp, n_edges, prec, N),
             "step_roofline": step_roofline(tm, args.steps, hp, n_edges, prec, N),
             "errors_vs_fp64": errors}
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
        # to K = 6 and truncated to K = 2 (13,824-atom box, l_max = 2, C = 64).
        # K = 2 runs the specialised first- and last-layer kernels only, K = 6
        # adds four middle layers on the generic kernels, so K6/K2 mixes depth
        # with the kernel-class gap; the per-layer times and a run with the
        # generic kernels for every layer (K2_generic) separate the two
        sd, hpd = W.mpdp_system(), W.HP_MPDP
        blobd = W.make_weights(hpd, W.WEIGHT_SEEDS["mpdp"])
        modeld = M.Model(hpd, blobd)
        os.environ["MPIP_FORCE_GENERIC"] = "1"
        modelg = M.Model(hpd, blobd)
        del os.environ["MPIP_FORCE_GENERIC"]
        pd = torch.tensor(sd.positions, dtype=torch.float64, device=dev)
        spd = torch.tensor(sd.species, dtype=torch.int32, device=dev)
        depth = {"metric": "ms per E+F evaluation of a 13,824-atom box, one 6-layer weight set run to K layers",
                 "n_atoms": sd.n_atoms, "steps": args.depth_steps,
                 "note": "K=2 uses the specialised first/last-layer kernels, K=6 adds 4 generic middle layers: "
                         "K6_over_K2 includes that kernel-class gap; K6_over_K2_generic compares K=6 with K=2 "
                         "run on the generic kernels; layers_ms splits each run by layer (edge kernels)"}

        def timed(mdl, Kd, prec):
            o = mdl.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec)
            cap = int(o["n_edges"] * 1.02) + 4096
            mdl.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec, max_edges=cap, out=o, check=False)
            M.lib.mpip_timing_enable(mdl._h, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.depth_steps):
                mdl.evaluate(pd, spd, sd.cell, sd.pbc, K=Kd, precision=prec, max_edges=cap, out=o, check=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.depth_steps * 1e3
            tm = M.read_timing(mdl)
            M.lib.mpip_timing_enable(mdl._h, 0)
            layers = {}
            for k, (tot, _) in tm.items():
                if k.startswith("edge_"):
                    t = int(k.rsplit("_t", 1)[1])
                    layers[f"t{t}"] = round(layers.get(f"t{t}", 0.0) + tot / args.depth_steps, 3)
            return round(ms, 3), layers

        for prec in precs:
            row = {}
            row["K6_ms"], l6 = timed(modeld, 6, prec)
            row["K2_ms"], l2 = timed(modeld, 2, prec)
            row["K2_generic_ms"], l2g = timed(modelg, 2, prec)
            row["K6_over_K2"] = round(row["K6_ms"] / row["K2_ms"], 2)
            row["K6_over_K2_generic"] = round(row["K6_ms"] / row["K2_generic_ms"], 2)
            row["layers_ms"] = {"K6": l6, "K2": l2, "K2_generic": l2g}
            depth[prec] = row
            log(f"depth pruning ({prec}): K=6 {row['K6_ms']} ms, K=2 {row['K2_ms']} ms, "
                f"K=2 generic {row['K2_generic_ms']} ms")
        del modeld, modelg, pd, spd
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
        # one GPU's share of the 8M box (slab 0 of 8: 1M roots) with a halo of
        # K r_cut, evaluated (trimmed) at K = 2 and K = 6 of the 6-layer weights
        shares = {}
        for Kh in (2, 6):
            gp, gs, _, no = M.slab_share(p8, sp8, s8.cell, n_parts, 0, Kh * hp8.r_cut)
            pbc_s = (False, True, True)
            o = model8.evaluate(gp, gs, s8.cell, pbc_s, K=Kh, precision=head, n_owned=no)
            cap = int(o["n_edges"] * 1.02) + 4096
            reps = 3 if Kh == 2 else 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                model8.evaluate(gp, gs, s8.cell, pbc_s, K=Kh, precision=head, n_owned=no, max_edges=cap, out=o)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            shares[f"K{Kh}"] = {"ms": round(ms, 3), "rows": int(gp.shape[0]), "roots": no,
                                "root_atom_steps_per_s": round(no / (ms * 1e-3), 1), "steps": reps}
            log(f"share of the 8M box, K={Kh} ({head}): {ms:.1f} ms, {gp.shape[0]} rows")
            del gp, gs, o
        part["share_K2_vs_K6"] = shares
        del model8, p8, sp8, o8, og
    batch = None
    if args.batch_steps > 0:
        # 512 independent periodic cells of 8-512 atoms (l_max = 2, C = 64,
        # K = 2) in one pass of every kernel over the block-diagonal list
        structs = W.batch_structures()
        hpb = W.HP_BATCH
        modelb = M.Model(hpb, W.make_weights(hpb, W.WEIGHT_SEEDS["batch512"]))
        bt = M.Batch(structs, dev)
        batch = {"metric": "atom-steps/s of 512 independent periodic cells (8-512 atoms, l_max=2, C=64, K=2) "
                           "evaluated together", "n_structures": bt.B, "n_atoms": bt.n_atoms,
                 "steps": args.batch_steps}
        for prec in precs:
            o = M.evaluate_batch(modelb, bt, K=2, precision=prec)
            cap = int(o["n_edges"] * 1.02) + 4096
            M.evaluate_batch(modelb, bt, K=2, precision=prec, max_edges=cap, check=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.batch_steps):
                M.evaluate_batch(modelb, bt, K=2, precision=prec, max_edges=cap, check=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.batch_steps * 1e3
            batch[prec] = {"ms_per_step": round(ms, 4), "value": round(bt.n_atoms / (ms * 1e-3), 1),
                           "n_edges": o["n_edges"]}
            log(f"batch512 ({prec}): {ms:.3f} ms per step")
        if "bf16" in batch and "fp32" in batch:
            batch["bf16_speedup_over_fp32"] = round(batch["fp32"]["ms_per_step"] / batch["bf16"]["ms_per_step"], 3)
        del modelb, bt
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
            "partitioned": part,
            "batch512": batch}
    if "bf16" in results and "fp32" in results:
        line["bf16_speedup_over_fp32"] = round(results["fp32"]["ms_per_step"] / results["bf16"]["ms_per_step"], 3)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
