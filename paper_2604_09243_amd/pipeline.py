"""Surrogate-plus-fallback pipeline: the sequence of library calls that
trains the network on an SBR sweep and fills a dense angle-frequency grid.
Orchestration only: the SBR sweeps, the network and the fill are library
calls; torch supplies device memory, reshapes sweep output into training
pairs and takes the go/no-go decision of ``anchored_fill`` (a comparison of
dB values)."""
import time

import numpy as np

from . import sbr


def training_pairs(A):
    """(targets) complex [n_angles * n_freq, 2] = (A_HH, A_VV) of a sweep
    result A [n_angles, n_freq, 2, 2]."""
    import torch
    return torch.stack([A[:, :, 0, 0], A[:, :, 1, 1]], dim=-1).reshape(-1, 2).contiguous()


def grid_points(theta_deg, phi_deg, freqs_hz):
    """Points [n_angles * n_freq, 3] (theta, phi, f), angle-major."""
    th = np.repeat(np.asarray(theta_deg, np.float64), len(freqs_hz))
    ph = np.repeat(np.asarray(phi_deg, np.float64), len(freqs_hz))
    f = np.tile(np.asarray(freqs_hz, np.float64), len(theta_deg))
    return np.stack([th, ph, f], axis=1)


def tile_probes(theta_deg, phi_deg, freqs_hz, tile_angles, tile_freqs, per_tile=2):
    """Held-out probe points of each tile: the direction half a tile past the
    tile's first direction (between two training directions when a tile
    spans one training step) and per_tile frequencies at the centres of equal
    sub-bands of the tile's frequency range."""
    th, ph, fr = (np.asarray(x, np.float64) for x in (theta_deg, phi_deg, freqs_hz))
    na, nf = len(th), len(fr)
    dirs = []
    for a0 in range(0, na, tile_angles):
        a1 = min(na, a0 + tile_angles)
        if a1 - a0 > 1:  # grid step inside the tile
            step_t = (th[a1 - 1] - th[a0]) / (a1 - 1 - a0)
            step_p = (ph[a1 - 1] - ph[a0]) / (a1 - 1 - a0)
        else:
            step_t = step_p = 0.0
        dirs.append((th[a0] + step_t * tile_angles / 2.0, ph[a0] + step_p * tile_angles / 2.0))
    freqs = []
    for f0 in range(0, nf, tile_freqs):
        f1 = min(nf, f0 + tile_freqs)
        lo, hi = fr[f0], fr[f1 - 1]
        for q in range(per_tile):
            freqs.append(lo + (hi - lo) * (q + 0.5) / per_tile)
    return np.array(dirs), np.array(freqs)


def surrogate_fill(ctx, bvh, train, query, ds, max_bounces, net_kw=None, train_kw=None, tile_angles=10,
                   tile_freqs=32, tol_db=0.5, floor_db=40.0, mode=sbr.MODE_VECTOR):
    """Whole pipeline.  ``train`` and ``query`` are (theta_deg, phi_deg,
    freqs_hz) of the training sweep and of the dense grid.  Returns (A
    [n_angles, n_freq, 2] complex device tensor, info dict with stage
    times, fallback statistics and the network)."""
    import torch
    net_kw = dict(net_kw or {})
    train_kw = dict(train_kw or {})
    t0 = time.perf_counter()
    th, ph, fr = train
    A, _, st = ctx.rcs_sweep(bvh, th, ph, fr, max_bounces, ds=ds, mode=mode)
    tg = training_pairs(A)
    scale = float(torch.sqrt(torch.mean(torch.abs(tg) ** 2)).item())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lo = np.array([min(np.min(th), np.min(query[0])), min(np.min(ph), np.min(query[1])),
                   min(np.min(fr), np.min(query[2]))])
    hi = np.array([max(np.max(th), np.max(query[0])), max(np.max(ph), np.max(query[1])),
                   max(np.max(fr), np.max(query[2]))])
    hi = np.where(hi > lo, hi, lo + 1.0)
    net = ctx.mlp(lo, hi, out_scale=scale, **net_kw)
    pts = torch.from_numpy(grid_points(th, ph, fr)).cuda()
    hist = net.train(pts, tg, **train_kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pdir, pfr = tile_probes(*query, tile_angles, tile_freqs)
    Aq, err, fb, fst = ctx.surrogate_fill(bvh, net, query[0], query[1], query[2], tile_angles, tile_freqs, pdir, pfr,
                                          ds, max_bounces, mode=mode, tol_db=tol_db, floor_db=floor_db)
    t3 = time.perf_counter()
    info = dict(s_train_data=t1 - t0, s_train=t2 - t1, s_fill=t3 - t2, s_total=t3 - t0, loss=hist,
                train_rays=st["rays"], tile_err=err, fallback=fb, fill=fst, net=net, scale=scale)
    return Aq, info


def _match(values, grid, tol):
    """Index in grid of each value (|difference| <= tol), or None if one is missing."""
    grid = np.asarray(grid, np.float64)
    out = []
    for v in np.asarray(values, np.float64):
        i = int(np.argmin(np.abs(grid - v)))
        if abs(grid[i] - v) > tol:
            return None
        out.append(i)
    return np.array(out)


def _sigma_db(A):
    import torch
    return 10.0 * torch.log10(torch.clamp(4.0 * np.pi * torch.abs(A) ** 2, min=1e-300))


def anchored_fill(ctx, bvh, train, query, ds, max_bounces, net_kw=None, train_kw=None, tile_freqs=32,
                  tol_db=0.5, floor_db=40.0, hopeless=0.5, mode=sbr.MODE_VECTOR):
    """Whole pipeline with anchors and an early decision, for a training set
    whose directions are grid directions and whose frequencies are grid
    frequencies (e.g. every 10th direction and every 8th frequency):

    1. the anchor sweep: SBR at the training directions for every grid
       frequency, one trace per direction; those grid rows are exact, and
       the training pairs are their training frequencies;
    2. training;
    3. the held-out check: the network against SBR at the anchor rows'
       other frequencies (not trained on; no SBR beyond step 1).  When more
       than ``hopeless`` of the (anchor, frequency tile) cells miss by more
       than tol_db (on points within floor_db of the largest), the network
       cannot win: the other directions are filled by plain SBR, so the
       pipeline costs one plain sweep plus the training;
    4. otherwise the directions between anchors are filled by
       sbr_surrogate_fill, one angle tile per run of directions between two
       anchors, probed at the run's middle.

    Returns (A [n_angles, n_freq, 2] complex device tensor, info dict).
    Falls back to ``surrogate_fill`` when the training set is not on the grid
    or the runs between anchors are uneven."""
    import torch
    net_kw = dict(net_kw or {})
    train_kw = dict(train_kw or {})
    th, ph, fr = (np.asarray(x, np.float64) for x in train)
    qth, qph, qfr = (np.asarray(x, np.float64) for x in query)
    na, nf = len(qth), len(qfr)
    dirs = np.stack([qth, qph], axis=1)
    a_idx = None
    if len(th) == len(ph):
        hits = [np.nonzero((np.abs(qth - t) <= 1e-9) & (np.abs(qph - p) <= 1e-9))[0] for t, p in zip(th, ph)]
        if all(len(h) for h in hits):
            a_idx = np.array([h[0] for h in hits])
    f_idx = _match(fr, qfr, 1e-3)
    runs = np.diff(np.concatenate([np.sort(a_idx), [na + (a_idx.min() if a_idx is not None else 0)]])) - 1 \
        if a_idx is not None else None
    if a_idx is None or f_idx is None or len(set(runs.tolist())) != 1 or runs[0] < 1 or np.sort(a_idx)[0] != 0:
        A, info = surrogate_fill(ctx, bvh, train, query, ds, max_bounces, net_kw=net_kw, train_kw=train_kw,
                                 tile_freqs=tile_freqs, tol_db=tol_db, floor_db=floor_db, mode=mode)
        info["decision"] = "unanchored"
        return A, info
    a_idx = np.sort(a_idx)
    run = int(runs[0])
    t0 = time.perf_counter()
    # 1. anchor sweep: every grid frequency at the training directions
    Aa, _, st = ctx.rcs_sweep(bvh, qth[a_idx], qph[a_idx], qfr, max_bounces, ds=ds, mode=mode)
    Aa = torch.stack([Aa[:, :, 0, 0], Aa[:, :, 1, 1]], dim=-1)  # [n_anchor, nf, 2]
    f_t = torch.from_numpy(f_idx).to(Aa.device)
    tg = Aa.index_select(1, f_t).reshape(-1, 2).contiguous()
    scale = float(torch.sqrt(torch.mean(torch.abs(tg) ** 2)).item())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # 2. training
    lo = np.array([qth.min(), qph.min(), qfr.min()])
    hi = np.array([qth.max(), qph.max(), qfr.max()])
    hi = np.where(hi > lo, hi, lo + 1.0)
    net = ctx.mlp(lo, hi, out_scale=scale, **net_kw)
    pts = torch.from_numpy(grid_points(qth[a_idx], qph[a_idx], qfr[f_idx])).cuda()
    hist = net.train(pts, tg, **train_kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # 3. held-out check at the anchor rows' other frequencies
    held = np.setdiff1d(np.arange(nf), f_idx)
    pred = net.predict(grid_points(qth[a_idx], qph[a_idx], qfr[held])).reshape(len(a_idx), len(held), 2)
    ref = Aa.index_select(1, torch.from_numpy(held).to(Aa.device))
    s_ref, s_net = _sigma_db(ref), _sigma_db(pred)
    lim = s_ref.amax() - floor_db
    err = torch.where(s_ref >= lim, torch.abs(s_net - s_ref), torch.zeros_like(s_ref)).amax(dim=2)  # [n_anchor, held]
    tile_of = torch.from_numpy(held // tile_freqs).to(err.device)
    n_ft = (nf + tile_freqs - 1) // tile_freqs
    cell = torch.zeros(len(a_idx), n_ft, dtype=err.dtype, device=err.device)
    cell.scatter_reduce_(1, tile_of.expand(len(a_idx), -1), err, reduce="amax")
    fail_frac = float((cell > tol_db).double().mean().item())
    t3 = time.perf_counter()
    # 4. the directions between anchors
    rest = np.setdiff1d(np.arange(na), a_idx)
    out = torch.empty(na, nf, 2, dtype=torch.complex128, device=Aa.device)
    out[torch.from_numpy(a_idx).to(out.device)] = Aa
    info = dict(loss=hist, net=net, scale=scale, anchors=len(a_idx), held_out_fail_frac=fail_frac,
                train_rays=st["rays"], s_anchor=t1 - t0, s_train=t2 - t1, s_check=t3 - t2)
    if fail_frac > hopeless:
        Ar, _, _ = ctx.rcs_sweep(bvh, qth[rest], qph[rest], qfr, max_bounces, ds=ds, mode=mode)
        out[torch.from_numpy(rest).to(out.device)] = torch.stack([Ar[:, :, 0, 0], Ar[:, :, 1, 1]], dim=-1)
        info.update(decision="plain", fallback=np.ones((len(rest) // run, n_ft), np.uint8),
                    tile_err=None, fill=dict(fallback_points=len(rest) * nf))
    else:
        pdir, pfr = tile_probes(qth[rest], qph[rest], qfr, run, tile_freqs)
        Aq, terr, fb, fst = ctx.surrogate_fill(bvh, net, qth[rest], qph[rest], qfr, run, tile_freqs, pdir, pfr,
                                               ds, max_bounces, mode=mode, tol_db=tol_db, floor_db=floor_db)
        out[torch.from_numpy(rest).to(out.device)] = Aq
        info.update(decision="surrogate", fallback=fb, tile_err=terr, fill=fst)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    info.update(s_fill=t4 - t3, s_total=t4 - t0)
    return out, info
