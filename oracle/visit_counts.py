"""Reference traversal work for the roofline of the trace kernels.

TEST INFRASTRUCTURE.  The algorithmic work of a closest-hit query is priced
on the oracle's own binned-SAH BVH (Algorithm 1 with the SAH cost, 4
triangles per leaf, 16 bins), not on the tree the GPU builds, so a worse GPU
tree cannot inflate the achieved rate.  For each bounce b the script runs the
oracle's fast mode with B_max = b and differences the cumulative counters,
giving per-bounce queries, box tests, triangle tests and hits on a fixed
sample of the trihedral sweep (every 10th angle of the 181).

    python -m oracle.visit_counts             ->  oracle/visit_counts_trihedral.json
    python -m oracle.visit_counts --aircraft  ->  oracle/visit_counts_aircraft.json
      (every 45th of the aircraft's 360 azimuths, 200,000 seeded rays each)
    python -m oracle.visit_counts --batch     ->  oracle/visit_counts_batch.json
      (64 items of the 64-scene batch drawn in proportion to their rays,
      20,000 seeded rays each)
"""
import json
import os
import sys

import numpy as np

import sbr_inputs as si
from . import oracle as O

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "visit_counts_trihedral.json")
OUT_AIRCRAFT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "visit_counts_aircraft.json")
OUT_BATCH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "visit_counts_batch.json")


def per_bounce_counts(w, angle_idx, bmax, ray_sample=None, seed=0):
    """ray_sample: trace only this many rays of each angle, drawn with a
    seeded generator (the per-query averages of a large grid)."""
    m = O.Mesh(w.V, w.T).build_bvh("sah", 4, 16)
    subsets = {}
    if ray_sample:
        rng = np.random.default_rng(seed)
        for i in angle_idx:
            Nu, Nv, *_ = O.aperture(m.bbox, w.theta_deg[i], w.phi_deg[i], O.C0 / float(np.max(w.freqs_hz)) /
                                    w.samples_per_lambda)
            subsets[i] = np.sort(rng.choice(Nu * Nv, size=min(ray_sample, Nu * Nv), replace=False))
    cum = []
    rays = 0
    for b in range(1, bmax + 1):
        q = box = tri = hits = 0
        rays = 0
        for i in angle_idx:
            r = O.rcs_angle(m, w.theta_deg[i], w.phi_deg[i], w.freqs_hz, w.samples_per_lambda, bmax=b,
                            use_bvh=True, ray_subset=subsets.get(i))
            q += r["queries"]
            box += r["box_tests"]
            tri += r["tri_tests"]
            hits += int(r["nb"].sum())
            rays += len(r["nb"])
        cum.append((q, box, tri, hits))
    out = []
    prev = (0, 0, 0, 0)
    for b, c in enumerate(cum, start=1):
        d = [c[i] - prev[i] for i in range(4)]
        out.append(dict(bounce=b, queries=d[0], box_tests=d[1], tri_tests=d[2], hits=d[3],
                        box_per_query=d[1] / max(d[0], 1), tri_per_query=d[2] / max(d[0], 1),
                        hits_per_query=d[3] / max(d[0], 1)))
        prev = c
    return dict(workload=w.name, angles_sampled=len(angle_idx), rays=rays, tree="binned SAH, leaf<=4, 16 bins",
                ray_sample=ray_sample, per_bounce=out)


def batch_per_bounce_counts(w, draws=64, ray_sample=20_000, seed=0):
    """The 64-scene batch: `draws` items drawn (seeded, with replacement) with
    probability proportional to their ray counts, `ray_sample` seeded rays of
    each, traced on the oracle's binned-SAH tree of the item's scene; the
    per-query averages then weight bounces as the batch's own queries do."""
    items = w.items()
    freqs = w.freqs()
    rays, ds_of = [], []
    for sc, th, ph, fo, nf in items:
        s = w.scenes[sc]
        P = np.asarray(s.V, np.float64)[np.asarray(s.T).ravel()]
        bbox = np.concatenate([P.min(0), P.max(0)])
        ds = O.C0 / float(np.max(freqs[fo:fo + nf])) / w.samples_per_lambda
        Nu, Nv, *_ = O.aperture(bbox, th, ph, ds)
        rays.append(Nu * Nv)
        ds_of.append(ds)
    rays = np.asarray(rays, np.float64)
    rng = np.random.default_rng(seed)
    picks = rng.choice(len(items), size=draws, replace=True, p=rays / rays.sum())
    subsets = [np.sort(rng.choice(int(rays[i]), size=min(ray_sample, int(rays[i])), replace=False)) for i in picks]
    meshes = {}
    cum = []
    for b in range(1, w.max_bounces + 1):
        q = box = tri = hits = 0
        for i, ids in zip(picks, subsets):
            sc, th, ph, fo, nf = items[i]
            if sc not in meshes:
                meshes[sc] = O.Mesh(w.scenes[sc].V, w.scenes[sc].T).build_bvh("sah", 4, 16)
            r = O.rcs_angle(meshes[sc], th, ph, freqs[fo:fo + nf], w.samples_per_lambda, ds=ds_of[i], bmax=b,
                            use_bvh=True, ray_subset=ids)
            q += r["queries"]
            box += r["box_tests"]
            tri += r["tri_tests"]
            hits += int(r["nb"].sum())
        cum.append((q, box, tri, hits))
    out = []
    prev = (0, 0, 0, 0)
    for b, c in enumerate(cum, start=1):
        d = [c[k] - prev[k] for k in range(4)]
        out.append(dict(bounce=b, queries=d[0], box_tests=d[1], tri_tests=d[2], hits=d[3],
                        box_per_query=d[1] / max(d[0], 1), tri_per_query=d[2] / max(d[0], 1),
                        hits_per_query=d[3] / max(d[0], 1)))
        prev = c
    return dict(workload=w.name, draws=draws, ray_sample=ray_sample, scenes_used=len(meshes),
                tree="binned SAH, leaf<=4, 16 bins", per_bounce=out)


def main():
    if "--batch" in sys.argv:
        res = batch_per_bounce_counts(si.batch_case())
        out = OUT_BATCH
    elif "--aircraft" in sys.argv:
        # the 1.5 M-triangle aircraft: every 45th of its 360 azimuths, 200,000
        # seeded rays of each (of ~9.6 M)
        w = si.aircraft_case()
        res = per_bounce_counts(w, list(range(0, w.n_angles, 45)), w.max_bounces, ray_sample=200_000, seed=0)
        out = OUT_AIRCRAFT
    else:
        w = si.trihedral_case()
        res = per_bounce_counts(w, list(range(0, w.n_angles, 10)), w.max_bounces)
        out = OUT
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
