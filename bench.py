#!/usr/bin/env python3
"""Throughput of the SBR trace-integrate path on one MI355X.

Workload: square trihedral corner reflector (a = 1 m, 1,536 triangles),
10 GHz, elevation 35.26 deg, azimuth 0..90 deg in 0.5 deg steps (181 angles),
ray spacing lambda/10 (48,377,932 rays in all), at most 5 bounces, VECTOR PO
(all four H/V pairs from one trace).  One step = the whole path for the
sweep: mesh preparation and BVH build, ray generation, multi-bounce
transport, PO sum and RCS for all 181 angles.

Prints one JSON line.  ``value`` is closest-hit queries (rays x bounces) per
second over the timed steps; angles/s is reported beside it.  ``roofline``
prices the dominant trace kernel by the reference traversal work of the
oracle's SAH tree against the non-packed VALU issue rate;
``cpu_baseline`` times the CPU oracle (brute force, as it stands) on a
bounded sample of the same sweep.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays*bounces/s + RCS angles/s at <=0.05 dB vs oracle; surrogate vs plain SBR"

# Reference traversal work per closest-hit query, per bounce, on the
# trihedral sweep: box and triangle tests and hits per query of the oracle's
# binned-SAH BVH (4 triangles per leaf, 16 bins), every 10th angle
# (`python -m oracle.visit_counts`).
REF_VISITS = {1: (14.09, 2.41, 0.677), 2: (23.25, 3.34, 0.928), 3: (19.89, 1.96, 0.541),
              4: (11.97, 0.02, 0.0), 5: (0.0, 0.0, 0.0)}
# VALU lane operations per unit of work (float32 spec arithmetic, no fused
# multiply-add in the triangle test): slab test of one box 15 (6 FMA, 6
# min/max, min3/max3, compare); triangle test 66 (two cross products 18, four
# dot products 20, s = o - v0 3, correctly rounded reciprocal ~10, three
# products 3, barycentric/t tests and the closest-hit update 12); per query
# 12 (reciprocal direction, scaled origin); per hit 80 (hit point, fp64 path
# and offset correction, reflection of d and both field vectors, new origin,
# fp64 phase path, record).
C_BOX, C_TRI, C_QUERY, C_HIT = 15, 66, 12, 80
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s of
# non-packed VALU issue (the 157.3 TFLOP/s fp32 figure counts packed FMA as 4).
PEAK_LANE_OPS = 256 * 64 * 2.4e9

PMC_FILE = os.path.join(ROOT, "profiles", "trace_trihedral_pmc.json")


def work_per_query(b):
    box, tri, hit = REF_VISITS.get(b, (0.0, 0.0, 0.0))
    return box * C_BOX + tri * C_TRI + C_QUERY + hit * C_HIT


def source_hash():
    h = hashlib.sha256()
    for f in ("trace.hip", "sbr_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2604_09243_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel, launches_per_step):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, scaled by the plain-copy calibration; None if absent or if the
    trace source changed since the counters were taken."""
    try:
        with open(PMC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash() or kernel not in d.get("kernels", {}):
        return None
    k = d["kernels"][kernel]
    return (k["fetch_kib"] * d["fetch_scale"] + k["write_kib"] * d["write_scale"]) * 1024.0


def cpu_baseline(w, A_gpu, seconds):
    """The oracle, brute force as it stands, on whole angles of the same sweep
    (taken in a fixed order) until about `seconds` of CPU time; also checks
    those angles against the GPU result."""
    from oracle import oracle as O
    m = O.Mesh(w.V, w.T)
    order = [90, 0, 180, 45, 135, 23, 157, 68, 112, 11, 169]
    q = 0
    n = 0
    t0 = time.perf_counter()
    worst_db, worst_rel = 0.0, 0.0
    amax = float(np.abs(A_gpu).max())
    for i in order:
        r = O.rcs_angle(m, w.theta_deg[i], w.phi_deg[i], w.freqs_hz, w.samples_per_lambda, bmax=w.max_bounces)
        q += r["queries"]
        n += 1
        Ao, Ag = r["A"], A_gpu[i]
        den = np.maximum(np.abs(Ao), 1e-3 * amax)
        worst_rel = max(worst_rel, float((np.abs(Ag - Ao) / den).max()))
        so, sg = O.sigma_dbsm(Ao), O.sigma_dbsm(Ag)
        sel = so > -200
        if sel.any():
            worst_db = max(worst_db, float(np.abs(so - sg)[sel].max()))
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return dict(value=q / dt, unit="rays*bounces/s", cores=O.num_threads(), kind="oracle",
                sample="%d of the 181 angles (full ray grids), brute-force closest hit, %.1f s" % (n, dt),
                angles_per_s=n / dt), dict(angles_checked=n, max_abs_db=worst_db, max_rel_complex=worst_rel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=("trihedral", "batch"), default="trihedral",
                    help="trihedral: the 181-angle sweep (default); batch: the 64-scene uneven batch, one graph "
                         "replay per step (a secondary measurement)")
    ap.add_argument("--autotune", action="store_true", help="batch: autotune the launch parameters first")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: every incidence angle is independent, so a sweep shards by "
              "angle with no communication beyond gathering the per-angle results (DESIGN.md, sharding); "
              "no multi-GPU figure is measured here.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return

    import sbr_inputs as si
    from paper_2604_09243_amd import Context

    if args.workload == "batch":
        return bench_batch(args)
    w = si.trihedral_case()
    ctx = Context(0)

    def step():
        bvh = ctx.build_bvh(w.V, w.T)
        A, S, st = ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                 samples_per_lambda=w.samples_per_lambda)
        bvh.free()
        return A, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        A, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    queries = sum(s["queries"] for s in stats)
    angles = sum(s["angles"] for s in stats)
    ms_step = 1e3 * dt / args.steps
    # roofline of the trace kernel (one streaming launch per step): reference
    # work of every query it made, priced per bounce, over its GPU time
    nb = w.max_bounces
    q_b = np.zeros(nb + 1)
    for s in stats:
        q_b += np.array(s["queries_bounce"][:nb + 1])
    work = sum(q_b[b] * work_per_query(b) for b in range(1, nb + 1))
    t_kernel = sum(s["ms_trace"] for s in stats) * 1e-3
    launches = args.steps
    achieved = work / t_kernel
    traffic = pmc_traffic("k_stream", 1)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlaneop/s",
                "frac": achieved / PEAK_LANE_OPS, "traffic": traffic, "kernel": "k_stream<0> (all bounces, angle grid)",
                "avg_launch_ms": 1e3 * t_kernel / launches, "work_per_launch_lane_ops": work / launches}
    out = {
        "metric": METRIC,
        "value": queries / dt,
        "unit": "rays*bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (intersection, field) + f64 (path, phase, PO weights)",
        "data": "synthetic (seeded procedural mesh)",
        "config": {"workload": w.name + "_181az_lambda10_b5", "angles": w.n_angles, "rays_per_step": stats[-1]["rays"],
                   "queries_per_step": stats[-1]["queries"], "triangles": int(len(w.T)), "mode": "VECTOR",
                   "polarisations": "HH,HV,VH,VV"},
        "angles_per_s": angles / dt,
        "trace_ms_per_step": sum(s["ms_trace"] for s in stats) / args.steps,
        "po_ms_per_step": sum(s["ms_po"] for s in stats) / args.steps,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        cb, parity = cpu_baseline(w, A.cpu().numpy(), args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity_sample"] = parity
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 seeded scenes (10k-500k triangles), 16-256 directions and 1-32
    frequencies each (9,084 items, 1.7e10 rays), one graph replay per step;
    scene set and batch planning are set-up, outside the timed steps."""
    import torch
    import sbr_inputs as si
    from paper_2604_09243_amd import Context
    t0 = time.perf_counter()
    w = si.batch_case()
    ctx = Context(0)
    bvhs = [ctx.build_bvh(s.V, s.T) for s in w.scenes]
    scn = ctx.pack_scenes(bvhs)
    for b in bvhs:
        b.free()
    b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tune = b.autotune().as_dict() if args.autotune else b.info()["tune"]
    for _ in range(args.warmup):
        b.run(stats=False)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, st = b.run()
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    info = b.info()
    out = {
        "metric": METRIC, "value": sum(s["queries"] for s in stats) / dt, "unit": "rays*bounces/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (intersection, field) + f64 (path, phase, weights)",
        "data": "synthetic (seeded procedural meshes)",
        "config": {"workload": w.name + "_uneven_lambda10_b6", "scenes": len(w.scenes), "items": info["n_items"],
                   "rows": info["n_rows"], "rays_per_step": info["rays"], "queries_per_step": stats[-1]["queries"],
                   "triangles": int(scn.n_tris), "min_item_rays": info["min_item_rays"],
                   "max_item_rays": info["max_item_rays"], "chunks": info["n_chunks"], "tune": tune,
                   "mode": "VECTOR"},
        "items_per_s": info["n_items"] * args.steps / dt,
        "rows_per_s": info["n_rows"] * args.steps / dt,
        "graph_ms_per_step": sum(s["ms_total"] for s in stats) / args.steps,
        "setup_s": t_setup,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
