"""Reference traversal work for the roofline of the trace kernels.

TEST INFRASTRUCTURE.  The algorithmic work of a closest-hit query is priced
on the oracle's own binned-SAH BVH (Algorithm 1 with the SAH cost, 4
triangles per leaf, 16 bins), not on the tree the GPU builds, so a worse GPU
tree cannot inflate the achieved rate.  For each bounce b the script runs the
oracle's fast mode with B_max = b and differences the cumulative counters,
giving per-bounce queries, box tests, triangle tests and hits on a fixed
sample of the trihedral sweep (every 10th angle of the 181).  Each count is
given over all rays and over the rays a primary-ray mask keeps (cells of
8 x 8 rays touched by a projected leaf box of the oracle's tree): the
masked rays are misses that need no traversal, so a masked sweep's work is
priced per unmasked query.

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


MASK_CELL = 8  # rays per side of a mask cell


def masked_rays(mesh, theta_deg, phi_deg, ds, eta=0.1):
    """Per ray of the angle's grid (ray order j*Nu + i): True when no leaf box
    of the oracle's tree, projected onto the aperture plane and widened by
    half a ray spacing plus a float32 rounding bound, touches the ray's cell
    of 8 x 8 rays.  Such a ray cannot pass a leaf's box test, so a
    primary-ray mask resolves it as a miss without traversal."""
    Nu, Nv, uc, vc, s0 = O.aperture(mesh.bbox, theta_deg, phi_deg, ds, eta)
    k, th, ph = O.frame(theta_deg, phi_deg)
    bx = mesh.leaf_boxes()
    lo, hi = bx[:, :3], bx[:, 3:]
    r = np.abs(mesh.bbox.reshape(2, 3)).max(0).sum()
    ro = abs(uc) + abs(vc) + abs(s0) + 0.5 * (Nu + Nv) * ds
    slack = 0.5 + 64.0 * 2.0 ** -24 * (r + ro) / ds
    mcu, mcv = -(-Nu // MASK_CELL), -(-Nv // MASK_CELL)

    def span(w, c, n):
        a, b = lo * w, hi * w
        f0 = (np.minimum(a, b).sum(1) - c) / ds + 0.5 * n - 0.5 - slack
        f1 = (np.maximum(a, b).sum(1) - c) / ds + 0.5 * n - 0.5 + slack
        i0 = np.ceil(np.maximum(f0, 0.0))
        i1 = np.floor(np.minimum(f1, n - 1.0))
        return i0, i1, (f1 >= 0) & (f0 <= n - 1) & (i0 <= i1)

    i0, i1, oku = span(ph, uc, Nu)  # u = phi_hat, v = theta_hat
    j0, j1, okv = span(th, vc, Nv)
    ok = oku & okv
    c0 = (i0[ok] // MASK_CELL).astype(np.int64)
    c1 = (i1[ok] // MASK_CELL).astype(np.int64) + 1
    r0 = (j0[ok] // MASK_CELL).astype(np.int64)
    r1 = (j1[ok] // MASK_CELL).astype(np.int64) + 1
    # covered cells: a 2-D difference array of the cell rectangles, summed
    D = np.zeros((mcv + 1, mcu + 1), np.int64)
    np.add.at(D, (r0, c0), 1)
    np.add.at(D, (r0, c1), -1)
    np.add.at(D, (r1, c0), -1)
    np.add.at(D, (r1, c1), 1)
    cov = D.cumsum(0).cumsum(1)[:mcv, :mcu] > 0
    jj, ii = np.divmod(np.arange(Nu * Nv), Nu)
    return ~cov[jj // MASK_CELL, ii // MASK_CELL]


def _diff(cum):
    out = []
    prev = (0, 0, 0, 0)
    for b, c in enumerate(cum, start=1):
        d = [c[i] - prev[i] for i in range(4)]
        out.append(dict(bounce=b, queries=d[0], box_tests=d[1], tri_tests=d[2], hits=d[3],
                        box_per_query=d[1] / max(d[0], 1), tri_per_query=d[2] / max(d[0], 1),
                        hits_per_query=d[3] / max(d[0], 1)))
        prev = c
    return out


def traverse_counts(jobs, bmax):
    """jobs: (mesh, theta, phi, freqs, samples_per_lambda, ds, ray ids).  For
    each bounce b the oracle runs with B_max = b and the cumulative counters
    are differenced.  Rays are split by the mask: the unmasked ones are traced
    for every bounce, the masked ones (misses by construction, checked) once,
    at the first bounce; all-ray counts are the sums."""
    split = []
    for mesh, th, ph, fr, spl, ds, ids in jobs:
        m = masked_rays(mesh, th, ph, ds)[ids]
        split.append((ids[~m], ids[m]))

    def run(mesh, th, ph, fr, spl, ds, ids, b):
        if len(ids) == 0:
            return 0, 0, 0, 0
        r = O.rcs_angle(mesh, th, ph, fr, spl, ds=ds, bmax=b, use_bvh=True, ray_subset=ids)
        return r["queries"], r["box_tests"], r["tri_tests"], int(r["nb"].sum())

    cum_u = []
    for b in range(1, bmax + 1):
        tot = np.zeros(4, np.int64)
        for job, (iu, _) in zip(jobs, split):
            tot += run(*job[:6], iu, b)
        cum_u.append(tuple(int(x) for x in tot))
    mk = np.zeros(4, np.int64)
    for job, (_, im) in zip(jobs, split):
        mk += run(*job[:6], im, 1)
    assert mk[3] == 0, "a masked ray hit"
    cum_a = [tuple(c[i] + int(mk[i]) for i in range(4)) for c in cum_u]
    n_masked = sum(len(im) for _, im in split)
    n_rays = sum(len(job[6]) for job in jobs)
    return dict(per_bounce=_diff(cum_a), per_bounce_unmasked=_diff(cum_u), rays=n_rays, masked_rays=n_masked,
                masked_fraction=n_masked / max(n_rays, 1))


def per_bounce_counts(w, angle_idx, bmax, ray_sample=None, seed=0):
    """ray_sample: trace only this many rays of each angle, drawn with a
    seeded generator (the per-query averages of a large grid)."""
    m = O.Mesh(w.V, w.T).build_bvh("sah", 4, 16)
    ds = O.C0 / float(np.max(w.freqs_hz)) / w.samples_per_lambda
    rng = np.random.default_rng(seed) if ray_sample else None
    jobs = []
    for i in angle_idx:
        Nu, Nv, *_ = O.aperture(m.bbox, w.theta_deg[i], w.phi_deg[i], ds)
        if ray_sample:
            ids = np.sort(rng.choice(Nu * Nv, size=min(ray_sample, Nu * Nv), replace=False))
        else:
            ids = np.arange(Nu * Nv)
        jobs.append((m, w.theta_deg[i], w.phi_deg[i], w.freqs_hz, w.samples_per_lambda, ds, ids))
    res = traverse_counts(jobs, bmax)
    return dict(workload=w.name, angles_sampled=len(angle_idx), tree="binned SAH, leaf<=4, 16 bins",
                ray_sample=ray_sample, **res)


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
    jobs = []
    for i, ids in zip(picks, subsets):
        sc, th, ph, fo, nf = items[i]
        if sc not in meshes:
            meshes[sc] = O.Mesh(w.scenes[sc].V, w.scenes[sc].T).build_bvh("sah", 4, 16)
        jobs.append((meshes[sc], th, ph, freqs[fo:fo + nf], w.samples_per_lambda, ds_of[i], ids))
    res = traverse_counts(jobs, w.max_bounces)
    return dict(workload=w.name, draws=draws, ray_sample=ray_sample, scenes_used=len(meshes),
                tree="binned SAH, leaf<=4, 16 bins", **res)


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
