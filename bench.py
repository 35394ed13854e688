#!/usr/bin/env python3
"""Throughput of the SBR trace-integrate path on one MI355X.

Default workload: the procedural aircraft (1,505,310 triangles; fuselage
15 m, wings 12 m span, fins, two open inlets), 10 GHz, elevation 0, azimuth
0..359 deg in 1 deg steps (360 angles), ray spacing lambda/8, at most 8
bounces, VECTOR PO (all four H/V pairs from one trace).  The tree is built
once per mesh (its time is reported apart, as the paper amortises it over
all angles); one step = the whole path for the 360-angle sweep: ray
generation, multi-bounce transport, PO sum and RCS.  ``--workload
trihedral`` is the 181-angle corner-reflector sweep, with the tree built in
every step.

Prints one JSON line.  ``value`` is closest-hit queries (rays x bounces) per
second over the timed steps, the primary rays that the mask resolves
without traversal included (``value_traced`` leaves them out); angles/s is
reported beside it.  ``roofline`` prices the dominant trace kernel by the
reference traversal work of the oracle's SAH tree against the non-packed
VALU issue rate; ``cpu_baseline`` times the CPU oracle (its tree mode, which
is pinned bit for bit to brute force) on a bounded sample of the same sweep
and ``parity_sample`` compares those angles with the GPU result.
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
REF_VISITS = {1: (14.092, 2.407, 0.6774), 2: (23.162, 3.327, 0.9282), 3: (19.845, 1.951, 0.5408), 4: (11.966, 0.023, 0.0), 5: (0.0, 0.0, 0.0)}
# The same on the 1.5 M-triangle aircraft sweep: every 45th of its 360
# azimuths, 200,000 seeded rays of each (`python -m oracle.visit_counts
# --aircraft`).
REF_VISITS_AIRCRAFT = {1: (18.616, 1.33, 0.2516), 2: (53.579, 4.893, 0.0836), 3: (60.512, 5.409, 0.2803), 4: (67.134, 6.713, 0.6555), 5: (68.942, 6.154, 0.8434), 6: (78.66, 7.243, 0.9329), 7: (67.706, 5.842, 0.6012), 8: (66.383, 6.32, 0.5812)}
# The same on the 64-scene batch: 64 items drawn in proportion to their rays,
# 20,000 seeded rays of each (`python -m oracle.visit_counts --batch`).
REF_VISITS_BATCH = {1: (20.15, 2.173, 0.2682), 2: (48.174, 6.447, 0.0506), 3: (57.054, 8.329, 0.1284), 4: (68.309, 10.402, 0.3818), 5: (71.437, 10.884, 0.4266), 6: (74.614, 11.303, 0.4904)}
# The same over the rays a primary-ray mask keeps (8 x 8-ray cells touched
# by a projected leaf box of the oracle's tree): the sweeps' default.  Later
# bounces equal the all-ray figures (only hits bounce); the oracle's masks
# keep 72 % of the trihedral's, 26 % of the aircraft's and 29 % of the
# batch's primary rays.
REF_VISITS_UNMASKED = {1: (19.159, 3.339, 0.9397), 2: (23.162, 3.327, 0.9282), 3: (19.845, 1.951, 0.5408), 4: (11.966, 0.023, 0.0), 5: (0.0, 0.0, 0.0)}
REF_VISITS_AIRCRAFT_UNMASKED = {1: (53.104, 5.144, 0.9734), 2: (53.579, 4.893, 0.0836), 3: (60.512, 5.409, 0.2803), 4: (67.134, 6.713, 0.6555), 5: (68.942, 6.154, 0.8434), 6: (78.66, 7.243, 0.9329), 7: (67.706, 5.842, 0.6012), 8: (66.383, 6.32, 0.5812)}
REF_VISITS_BATCH_UNMASKED = {1: (53.538, 7.62, 0.9405), 2: (48.174, 6.447, 0.0506), 3: (57.054, 8.329, 0.1284), 4: (68.309, 10.402, 0.3818), 5: (71.437, 10.884, 0.4266), 6: (74.614, 11.303, 0.4904)}
# VALU lane operations per unit of traversal work, the survey's constants
# (midpoints of its ranges): a slab test of one box 14 (6 FMA, min/max of the
# three slabs, the compare), a triangle test 40 (the float32
# Moller-Trumbore specification with its correctly rounded reciprocal, the
# barycentric and t tests and the closest-hit update), and 60 per query for
# the rest of a bounce (reciprocal direction, the box rule of the winner,
# the hit point, the float64 path, the reflection of d and of both field
# vectors, the new origin, the record).
C_BOX, C_TRI, C_BOUNCE = 14, 40, 60
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s of
# non-packed VALU issue (the 157.3 TFLOP/s fp32 figure counts packed FMA as 4).
PEAK_LANE_OPS = 256 * 64 * 2.4e9


def pmc_file(builder, workload="trihedral"):
    if workload == "aircraft":
        return os.path.join(ROOT, "profiles", "trace_aircraft_360az_%s_pmc.json" % builder)
    return os.path.join(ROOT, "profiles", "trace_trihedral_%s_pmc.json" % builder)


BUILDER_SOURCE = {"lbvh": "lbvh.hip", "sah": "sah.cpp", "ploc": "lbvh.hip"}
BUILDER_ID = {"lbvh": 0, "sah": 1, "ploc": 2}


def priced_work(q_b, masked, nb, ref_all, ref_unmasked, mask_on):
    """Reference lane operations of a trace: every query at its bounce's price.
    With the primary-ray mask the masked rays (misses, no traversal) are left
    out and the other first-bounce queries take the price of unmasked rays;
    later bounces only ever follow hits, which the mask never touches."""
    if not mask_on:
        return sum(q_b[b] * work_per_query(b, ref_all) for b in range(1, nb + 1))
    return ((q_b[1] - masked) * work_per_query(1, ref_unmasked) +
            sum(q_b[b] * work_per_query(b, ref_unmasked) for b in range(2, nb + 1)))


def sbr_default_tune():
    from paper_2604_09243_amd import sbr
    return sbr.default_tune()


def mask_flag(args):
    """Trace flags of the command line: the primary-ray mask off, the binary tree instead of its four-wide copy."""
    from paper_2604_09243_amd import sbr
    return (sbr.OPT_NO_MASK if args.no_mask else 0) | (sbr.OPT_BVH4 if getattr(args, "bvh4", False) else 0)


def C_sizeof_tune(sbr):
    import ctypes
    return ctypes.sizeof(sbr.Tune)


def work_per_query(b, ref=None):
    box, tri, _hit = (REF_VISITS if ref is None else ref).get(b, (0.0, 0.0, 0.0))
    return box * C_BOX + tri * C_TRI + C_BOUNCE


def source_hash(builder):
    """Hash of the sources the trace kernel's memory traffic depends on: the
    kernel and the builder that lays out its tree."""
    h = hashlib.sha256()
    for f in ("trace.hip", BUILDER_SOURCE[builder]):
        with open(os.path.join(ROOT, "paper_2604_09243_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel, builder, workload="trihedral"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this builder's tree, scaled by the plain-copy calibration;
    None if absent or if the trace or builder source changed since the
    counters were taken."""
    try:
        with open(pmc_file(builder, workload)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash(builder) or kernel not in d.get("kernels", {}):
        return None
    k = d["kernels"][kernel]
    # fetch_kib and write_kib are per-dispatch averages
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
                angles_per_s=n / dt, cpu=cpu_model()), dict(angles_checked=n, max_abs_db=worst_db,
                                                            max_rel_complex=worst_rel)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 20 for the trihedral sweep, 3 for batch, mlp and builders, "
                         "3 for the trihedral surrogate and 1 for the aircraft surrogate)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 10 for the trihedral sweep: the GPU clock settles over "
                         "the first ~8 sweeps; 1 elsewhere, 0 for the aircraft surrogate)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=("trihedral", "aircraft", "batch", "surrogate", "mlp", "builders"),
                    default="aircraft",
                    help="aircraft: the 360-angle sweep of the 1.5 M-triangle aircraft (tree built once; the "
                         "default); trihedral: the 181-angle corner-reflector sweep; batch: the 64-scene uneven batch, one graph "
                         "replay per step; surrogate: surrogate-plus-fallback fill vs plain SBR on a "
                         "3600 x 512 grid; mlp: network inference and training throughput; builders: build "
                         "time, tree quality and trace time of the three BVH builders on the trihedral and "
                         "the aircraft (secondary measurements)")
    ap.add_argument("--target", choices=("trihedral", "aircraft"), default="trihedral",
                    help="surrogate: band-limited trihedral or the procedural aircraft")
    ap.add_argument("--autotune", action="store_true",
                    help="aircraft, batch: autotune the launch parameters first (set-up, not timed)")
    ap.add_argument("--no-mask", action="store_true",
                    help="trace every primary ray (no per-angle mask of empty cells)")
    ap.add_argument("--chunk-log2", type=int, default=0,
                    help="batch and aircraft: rays per chunk = 2^N (16..30; 0 = the library default)")
    ap.add_argument("--bvh4", action="store_true",
                    help="walk a four-wide copy of the tree (same results; a traversal study, slower on the aircraft)")
    ap.add_argument("--builder", choices=("lbvh", "sah", "ploc"), default="sah",
                    help="BVH builder of each step: host binned SAH (default; fewer node and triangle tests "
                         "per ray), the GPU LBVH, or GPU PLOC clustering")
    args = ap.parse_args()
    if args.steps is None or args.warmup is None:
        big = args.workload == "surrogate" and args.target == "aircraft"
        # the aircraft surrogate pipeline and its plain sweep take ~13 s each: one warm-up pair, one timed
        steps, warmup = {"trihedral": (20, 10), "aircraft": (5, 3)}.get(args.workload, (1, 1) if big else (3, 1))
        args.steps = steps if args.steps is None else args.steps
        args.warmup = warmup if args.warmup is None else args.warmup
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: every incidence angle is independent, so a sweep shards by "
              "angle with no communication beyond gathering the per-angle results; "
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
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "builders":
        return bench_builders(args)
    if args.workload == "aircraft":
        return bench_aircraft(args)
    if args.workload == "mlp":
        return bench_mlp(args)
    w = si.trihedral_case()
    ctx = Context(0)

    builder = BUILDER_ID[args.builder]

    build_s = []

    def step():
        tb = time.perf_counter()
        bvh = ctx.build_bvh(w.V, w.T, builder=builder)  # returns with the tree on the device
        build_s.append(time.perf_counter() - tb)
        A, S, st = ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                 samples_per_lambda=w.samples_per_lambda, flags=mask_flag(args))
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
    masked = sum(s["masked"] for s in stats)
    work = priced_work(q_b, masked, nb, REF_VISITS, REF_VISITS_UNMASKED, not args.no_mask)
    t_kernel = sum(s["ms_trace"] for s in stats) * 1e-3
    launches = args.steps
    achieved = work / t_kernel
    traffic = pmc_traffic("k_stream", args.builder)
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
                   "bvh": args.builder, "tree_width": 4 if args.bvh4 else 2, "primary_mask": not args.no_mask,
                   "polarisations": "HH,HV,VH,VV"},
        "value_traced": (queries - masked) / dt,
        "masked_rays_per_step": masked / args.steps,
        "angles_per_s": angles / dt,
        "trace_ms_per_step": sum(s["ms_trace"] for s in stats) / args.steps,
        "po_ms_per_step": sum(s["ms_po"] for s in stats) / args.steps,
        "build_ms_per_step": 1e3 * float(np.mean(build_s[-args.steps:])),
        # the same queries over the trace kernel's GPU time alone, and angles over
        # the GPU time of trace + PO + finalize (value divides by the whole step)
        "trace_queries_per_s": queries / t_kernel,
        "angles_per_s_gpu": angles / (sum(s["ms_trace"] + s["ms_po"] for s in stats) * 1e-3),
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
    bvhs = [ctx.build_bvh(s.V, s.T, builder=BUILDER_ID[args.builder]) for s in w.scenes]
    scn = ctx.pack_scenes(bvhs)
    for b in bvhs:
        b.free()
    from paper_2604_09243_amd import sbr
    b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                  flags=mask_flag(args),
                  tune=sbr.make_tune(chunk_log2=args.chunk_log2) if args.chunk_log2 else None)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    if args.autotune:
        print("autotuning the batch", file=sys.stderr, flush=True)
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
                   "mode": "VECTOR", "bvh": args.builder},
        "items_per_s": info["n_items"] * args.steps / dt,
        "rows_per_s": info["n_rows"] * args.steps / dt,
        "graph_ms_per_step": sum(s["ms_total"] for s in stats) / args.steps,
        "setup_s": t_setup,
    }
    # roofline of the trace launches (one streaming launch per chunk): the
    # graph replay has one clock, so one more run, launched eagerly with the
    # same plan and events around each chunk's trace, gives their GPU time
    b.close()
    from paper_2604_09243_amd import sbr
    be = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                   flags=sbr.OPT_NO_GRAPH | mask_flag(args), tune=sbr.Tune(C_sizeof_tune(sbr), **tune))
    _, _, se = be.run()
    be.close()
    nb = w.max_bounces
    q_b = np.array(se["queries_bounce"][:nb + 1], np.float64)
    work = priced_work(q_b, se["masked"], nb, REF_VISITS_BATCH, REF_VISITS_BATCH_UNMASKED, not args.no_mask)
    t_kernel = se["ms_trace"] * 1e-3
    nc = info["n_chunks"]
    out["masked_rays_per_step"] = se["masked"]
    out["config"]["primary_mask"] = not args.no_mask
    out["trace_ms_eager"] = se["ms_trace"]
    out["po_ms_eager"] = se["ms_po"]
    out["trace_queries_per_s"] = se["queries"] / t_kernel
    out["roofline"] = {"bound": "alu", "achieved": work / t_kernel / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                       "unit": "Tlaneop/s", "frac": work / t_kernel / PEAK_LANE_OPS, "traffic": None,
                       "kernel": "k_stream<0> (one launch per chunk, all bounces of its items)", "launches": nc,
                       "avg_launch_ms": se["ms_trace"] / nc, "work_per_launch_lane_ops": work / nc}
    print(json.dumps(out), flush=True)


def _copol_db(A):
    """sigma (dBsm) of (HH, VV) of an [..., 2] or [..., 2, 2] complex array."""
    if A.ndim >= 2 and A.shape[-2:] == (2, 2):
        A = np.stack([A[..., 0, 0], A[..., 1, 1]], axis=-1)
    return 10 * np.log10(np.maximum(4 * np.pi * np.abs(A) ** 2, 1e-300))


def bench_surrogate(args):
    """Dense grid 0.1 deg x 512 frequencies (3600 x 512 points, 8-12 GHz,
    ray spacing lambda(12 GHz)/8) filled two ways on the same GPU: plain SBR
    (one trace per direction + 512-frequency PO) and the anchored surrogate
    pipeline (SBR at the 1 deg training directions for every grid frequency,
    training on 64 of them, a held-out check at the others that sends a
    hopeless grid to plain SBR, else inference, SBR probes per tile of the
    0.9 deg between anchors x 32 frequencies and SBR fallback on failing
    tiles).  Steps alternate the two; the error is audited on every grid
    point against the plain result."""
    import torch
    import sbr_inputs as si
    from paper_2604_09243_amd import Context, pipeline
    C0 = 299_792_458.0
    ctx = Context(0)
    if args.target == "trihedral":
        V, T = si.trihedral(1.0, 16)
        th0, bm = 54.74, 5
    else:
        w = si.aircraft_case()
        V, T = w.V, w.T
        th0, bm = 90.0, 8
    bvh = ctx.build_bvh(V, T)
    ds = C0 / 12e9 / 8
    query = (np.full(3600, th0), np.arange(3600) * 0.1, np.linspace(8e9, 12e9, 512))
    # training set on the grid: every 10th direction (1 deg) x every 8th frequency (64 in 8-12 GHz)
    train = (np.full(360, th0), np.arange(360.0), query[2][::8])
    kw = dict(net_kw=dict(ff_sigma=2.0, seed=1), train_kw=dict(epochs=40, batch=4096, lr=4e-3, lr_min=4e-5, seed=0),
              tile_freqs=32, tol_db=0.25, floor_db=40.0)
    for _ in range(args.warmup):
        pipeline.anchored_fill(ctx, bvh, train, query, ds, bm, **kw)
        ctx.rcs_sweep(bvh, *query, bm, ds=ds, stats=False)
    t_sur, t_plain = [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A, info = pipeline.anchored_fill(ctx, bvh, train, query, ds, bm, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Ap, _, st = ctx.rcs_sweep(bvh, *query, bm, ds=ds)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_sur.append(t1 - t0)
        t_plain.append(t2 - t1)
    sp = _copol_db(Ap.cpu().numpy())
    ss = _copol_db(A.cpu().numpy())
    n = sp.shape[0] * sp.shape[1]
    audit = {}
    for fl in (20, 30, 40):
        sel = sp >= sp.max() - fl
        e = np.abs(ss - sp)[sel]
        audit["floor_%ddB" % fl] = dict(frac_points=float(sel.mean()), p50=float(np.median(e)),
                                        p99=float(np.percentile(e, 99)), max=float(e.max()),
                                        within_0p5dB=float(np.mean(e <= 0.5)))
    fb = info["fallback"]
    ts, tp = float(np.median(t_sur)), float(np.median(t_plain))
    out = {
        "metric": METRIC, "value": n / ts, "unit": "grid points/s (surrogate + fallback)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * ts, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 MFMA (fp32 accumulation) + SBR f32/f64",
        "data": "synthetic (seeded procedural mesh)",
        "config": {"workload": "surrogate_%s_3600x512" % args.target, "train": "360 x 64", "query": "3600 x 512",
                   "tiles": "9 directions between anchors x 32 f", "probes": "1 direction x 2 f per tile",
                   "tol_db": 0.25,
                   "floor_db": 40.0, "audit_floor_db": 30.0, "epochs": 40, "batch": 4096, "lr": 4e-3},
        "plain_points_per_s": n / tp, "plain_ms": 1e3 * tp, "gain": tp / ts, "beats_plain_sbr": bool(tp > ts),
        "fallback_tile_frac": float(fb.mean()), "stage_s": {k: v for k, v in info.items() if k.startswith("s_")},
        "decision": info.get("decision"), "held_out_fail_frac": info.get("held_out_fail_frac"),
        "fill_ms": {k: v for k, v in info["fill"].items() if k.startswith("ms_")},
        "final_loss": float(info["loss"][-1]), "audit_vs_plain": audit,
        "plain_trace_ms": st["ms_trace"], "plain_po_ms": st["ms_po"], "plain_rays": st["rays"],
    }
    print(json.dumps(out), flush=True)


def bench_mlp(args):
    """The surrogate network alone: inference over the 3600 x 512 query grid
    (1,843,200 points) and training steps on the 360 x 64 training set,
    against the bf16 dense MFMA peak (2.5 PFLOP/s)."""
    import torch
    from paper_2604_09243_amd import Context, pipeline
    ctx = Context(0)
    net = ctx.mlp([0, 0, 8e9], [180, 360, 12e9], out_scale=1.0, ff_sigma=2.0, seed=3)
    info = net.info()
    pts = torch.from_numpy(pipeline.grid_points(np.full(3600, 90.0), np.arange(3600) * 0.1,
                                                np.linspace(8e9, 12e9, 512))).cuda()
    M = pts.shape[0]
    for _ in range(args.warmup):
        net.predict(pts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.predict(pts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    flops = info["flops_per_point"] * M
    tp = torch.from_numpy(pipeline.grid_points(np.full(360, 90.0), np.arange(360.0),
                                               np.linspace(8e9, 12e9, 64))).cuda()
    tg = torch.randn(tp.shape[0], 2, dtype=torch.complex128, device="cuda")
    net.train(tp, tg, epochs=2, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    epochs = 20
    net.train(tp, tg, epochs=epochs, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    dtt = time.perf_counter() - t0
    steps = epochs * ((tp.shape[0] + 4095) // 4096)
    out = {
        "metric": "surrogate inference points/s", "value": M / dt, "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulation)", "data": "synthetic",
        "config": {"workload": "mlp_ff64_4x256_grid_3600x512", "params": info["n_params"],
                   "flops_per_point": info["flops_per_point"]},
        "roofline": {"bound": "mfma", "achieved": flops / dt / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flops / dt / 2.5e15, "traffic": None},
        "train_ms_per_step": 1e3 * dtt / steps, "train_batch": 4096,
        "train_tflops": 3 * info["flops_per_point"] * 4096 * steps / dtt / 1e12,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_aircraft(w, A_gpu, seconds):
    """The oracle as it stands on a bounded sample of the aircraft sweep: its
    binned-SAH tree (built once, timed apart) in fast mode, which the CPU
    tests pin bit for bit to brute force, on whole angles taken in a fixed
    order until about `seconds` have passed (at least two); brute force on
    400 seeded rays of the first angle as a check of those angles; a
    one-thread figure of the fast mode on 50,000 seeded rays.  Also compares
    the sampled angles with the GPU result (parity sample)."""
    from oracle import oracle as O
    m = O.Mesh(w.V, w.T)
    t0 = time.perf_counter()
    m.build_bvh("sah")
    build_s = time.perf_counter() - t0
    order = [0, 90, 180, 270, 45, 135, 225, 315, 23, 157, 203, 337, 68, 112, 248, 292]
    q = n = 0
    worst_db, worst_rel = 0.0, 0.0
    amax = float(np.abs(A_gpu).max())
    t0 = time.perf_counter()
    for i in order:
        r = O.rcs_angle(m, w.theta_deg[i], w.phi_deg[i], w.freqs_hz, w.samples_per_lambda, bmax=w.max_bounces,
                        use_bvh=True)
        q += r["queries"]
        n += 1
        Ao, Ag = r["A"], A_gpu[i]
        den = np.maximum(np.abs(Ao), 1e-3 * amax)
        worst_rel = max(worst_rel, float((np.abs(Ag - Ao) / den).max()))
        so, sg = O.sigma_dbsm(Ao), O.sigma_dbsm(Ag)
        sel = so >= so.max() - 40.0
        worst_db = max(worst_db, float(np.abs(so - sg)[sel].max()))
        if n >= 2 and time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    # brute force on seeded rays of the first angle: the same results as the tree, at its own rate
    th, ph = w.theta_deg[order[0]], w.phi_deg[order[0]]
    k, tv, pv = O.frame(th, ph)
    o, d, _, _ = O.gen_rays(m.bbox, th, ph, w.ds)
    ids = np.sort(np.random.default_rng(11).choice(len(o), 400, replace=False))
    tb = time.perf_counter()
    rb = O.trace(m, o[ids], d, pv, tv, k, w.max_bounces, want_path=True)
    tb = time.perf_counter() - tb
    rf = O.trace(m, o[ids], d, pv, tv, k, w.max_bounces, want_path=True, use_bvh=True)
    brute_equal = all(np.array_equal(rb[key], rf[key]) for key in ("tri_path", "nb", "D", "x_last"))
    # one thread
    threads = O.num_threads()
    ids = np.sort(np.random.default_rng(12).choice(len(o), 50_000, replace=False))
    O.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        r1 = O.trace(m, o[ids], d, pv, tv, k, w.max_bounces, use_bvh=True)
        t1 = time.perf_counter() - t1
    finally:
        O.set_num_threads(threads)
    base = dict(value=q / dt, unit="rays*bounces/s", cores=threads, kind="oracle",
                sample="%d of the 360 angles (full ray grids) in the oracle's SAH-tree mode, %.1f s; tree build "
                       "%.1f s apart" % (n, dt, build_s),
                angles_per_s=n / dt, single_thread=r1["queries"] / t1, brute_force=rb["queries"] / tb,
                brute_force_rays=400, brute_force_equal_to_tree=bool(brute_equal), cpu=cpu_model())
    return base, dict(angles_checked=n, max_abs_db=worst_db, max_rel_complex=worst_rel,
                      db_within="40 dB of each angle's maximum", brute_force_rays_equal=bool(brute_equal))


def bench_aircraft(args):
    """The aircraft sweep (1.5 M triangles, 360 azimuths at elevation 0, 10 GHz,
    lambda/8, up to 8 bounces, HH/HV/VH/VV): the tree is built once (its
    time reported), each step is the whole 360-angle sweep (ray generation,
    every bounce, PO, RCS).  Roofline of the trace kernel priced on the
    oracle's SAH tree of the aircraft."""
    import torch
    import sbr_inputs as si
    from paper_2604_09243_amd import Context
    w = si.aircraft_case()
    ctx = Context(0)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    bvh = ctx.build_bvh(w.V, w.T, builder=BUILDER_ID[args.builder])
    torch.cuda.synchronize()
    build_ms = 1e3 * (time.perf_counter() - tb)
    tune, tune_s = None, 0.0
    if args.chunk_log2:
        from paper_2604_09243_amd import sbr
        tune = sbr.make_tune(chunk_log2=args.chunk_log2)
    if args.autotune:
        print("autotuning the sweep", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        tune = ctx.autotune(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                            samples_per_lambda=w.samples_per_lambda, flags=mask_flag(args))
        tune_s = time.perf_counter() - t0

    def step():
        A, S, st = ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                 samples_per_lambda=w.samples_per_lambda, flags=mask_flag(args), tune=tune)
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
    nb = w.max_bounces
    q_b = np.zeros(nb + 1)
    for s in stats:
        q_b += np.array(s["queries_bounce"][:nb + 1])
    masked = sum(s["masked"] for s in stats)
    work = priced_work(q_b, masked, nb, REF_VISITS_AIRCRAFT, REF_VISITS_AIRCRAFT_UNMASKED, not args.no_mask)
    t_kernel = sum(s["ms_trace"] for s in stats) * 1e-3
    launches = sum(s["chunks"] for s in stats)
    out = {
        "metric": METRIC, "value": queries / dt, "unit": "rays*bounces/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (intersection, field) + f64 (path, phase, PO weights)",
        "data": "synthetic (seeded procedural mesh)",
        "config": {"workload": w.name + "_360az_lambda8_b8", "angles": w.n_angles, "rays_per_step": stats[-1]["rays"],
                   "queries_per_step": stats[-1]["queries"], "triangles": int(len(w.T)), "mode": "VECTOR",
                   "bvh": args.builder, "tree_width": 4 if args.bvh4 else 2, "primary_mask": not args.no_mask, "polarisations": "HH,HV,VH,VV",
                   "tune": (tune if tune is not None else sbr_default_tune()).as_dict(),
                   "chunks_per_step": launches // args.steps},  # chunk_log2 0: the library's automatic size
        # the queries that traversed the tree: the mask's primary-ray misses left out
        "value_traced": (queries - masked) / dt,
        "autotune_s": tune_s,
        "masked_rays_per_step": masked / args.steps,
        "angles_per_s": w.n_angles * args.steps / dt,
        "trace_ms_per_step": 1e3 * t_kernel / args.steps,
        "po_ms_per_step": sum(s["ms_po"] for s in stats) / args.steps,
        "build_ms_once": build_ms,
        "angles_per_s_build_amortised": w.n_angles / (dt / args.steps + build_ms * 1e-3),
        "trace_queries_per_s": queries / t_kernel,
        "angles_per_s_gpu": w.n_angles * args.steps / (sum(s["ms_trace"] + s["ms_po"] for s in stats) * 1e-3),
        "roofline": {"bound": "alu", "achieved": work / t_kernel / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlaneop/s", "frac": work / t_kernel / PEAK_LANE_OPS,
                     "traffic": pmc_traffic("k_stream", args.builder, "aircraft"),
                     "kernel": "k_stream<0> (all bounces of a chunk of angles, angle grid)", "launches": launches,
                     "avg_launch_ms": 1e3 * t_kernel / launches, "work_per_launch_lane_ops": work / launches,
                     "pricing": "per query: box tests x %d + triangle tests x %d + %d, visit counts of the oracle's "
                                "SAH tree" % (C_BOX, C_TRI, C_BOUNCE)},
    }
    if not args.no_cpu_baseline:
        cb, parity = cpu_baseline_aircraft(w, A.cpu().numpy(), args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity_sample"] = parity
    print(json.dumps(out), flush=True)


def bench_builders(args):
    """Each builder on the trihedral (1,536 triangles, all 181 angles) and the
    aircraft (1.5 M triangles, 8 of its 360 angles): build time (median of
    the timed steps, build and free), the tree's surface-area estimates of
    node visits and triangle tests per line (sbr_bvh_quality_of), and the
    trace kernel's time.  value = closest-hit queries/s of the PLOC tree on
    the aircraft sample."""
    import torch
    import sbr_inputs as si
    from paper_2604_09243_amd import Context
    ctx = Context(0)
    rows = []
    value = None
    for w in (si.trihedral_case(), si.aircraft_case()):
        sel = slice(None) if w.n_angles <= 181 else slice(None, None, 45)
        th, ph = w.theta_deg[sel], w.phi_deg[sel]
        for name, builder in (("sah", 1), ("lbvh", 0), ("ploc", 2)):
            reps = args.steps if len(w.T) < 100_000 or builder != 1 else 1
            times = []
            for it in range(args.warmup + reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                bvh = ctx.build_bvh(w.V, w.T, builder=builder)
                torch.cuda.synchronize()
                if it >= args.warmup or reps == 1:
                    times.append(time.perf_counter() - t0)
                if it < args.warmup + reps - 1:
                    bvh.free()
            q = bvh.quality()
            tr = []
            for it in range(8):  # the GPU clock settles over the first sweeps; the minimum is reported
                A, _, st = ctx.rcs_sweep(bvh, th, ph, w.freqs_hz, w.max_bounces,
                                         samples_per_lambda=w.samples_per_lambda)
                tr.append(st["ms_trace"])
            bvh.free()
            row = {"mesh": w.name, "triangles": len(w.T), "angles": len(th), "builder": name,
                   "build_ms": 1e3 * float(np.median(times)), "nodes": bvh.n_nodes, "depth": bvh.depth,
                   "node_visits": q["node_visits"], "tri_tests": q["tri_tests"], "trace_ms": min(tr),
                   "queries": st["queries"]}
            rows.append(row)
            if name == "ploc" and len(w.T) > 100_000:
                value = st["queries"] / (min(tr) * 1e-3)
    out = {
        "metric": "rays*bounces/s", "value": value, "unit": "rays*bounces/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (intersection) + f64 (path)",
        "data": "synthetic (seeded procedural meshes)",
        "config": {"workload": "bvh_builders_trihedral_aircraft"}, "builders": rows,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
