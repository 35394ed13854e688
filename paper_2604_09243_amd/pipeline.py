"""Surrogate-plus-fallback pipeline: the sequence of library calls that
trains the network on an SBR sweep and fills a dense angle-frequency grid.
Orchestration only: every computation is a library call (torch supplies
device memory and reshapes the sweep output into training pairs)."""
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
