"""The primary-ray mask: a per-angle map of 8 x 8-ray cells marked by the
projected leaf boxes of the tree.  Rays of empty cells are resolved as
misses without traversal, which is exact because a ray reaches a leaf only
through that leaf's box test.  Every case compares a run with the mask
against one with SBR_OPT_NO_MASK, bit for bit, and checks that masked rays
are still counted as first-bounce queries."""
import sys

import numpy as np
import pytest

import sbr_inputs as si

pytestmark = pytest.mark.gpu

C0 = 299_792_458.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_2604_09243_amd import Context
    return Context(0)


def both(run):
    """run(flags) -> (A, sigma, stats); returns the masked and unmasked results."""
    from paper_2604_09243_amd import sbr
    A1, S1, st1 = run(0)
    A0, S0, st0 = run(sbr.OPT_NO_MASK)
    return (A1.cpu().numpy(), S1.cpu().numpy(), st1), (A0.cpu().numpy(), S0.cpu().numpy(), st0)


def check_same(m, u, min_frac=0.0):
    (A1, S1, st1), (A0, S0, st0) = m, u
    assert np.array_equal(A1.view(np.float64), A0.view(np.float64))
    assert np.array_equal(S1, S0)
    assert st0["masked"] == 0
    assert st1["queries"] == st0["queries"] and st1["hits"] == st0["hits"] and st1["valid"] == st0["valid"]
    assert st1["masked"] >= min_frac * st1["rays"]
    # a masked ray is a miss: never more masked rays than first-bounce misses
    assert st1["masked"] <= st1["rays"] - st1["hits"][1]
    return st1["masked"] / st1["rays"]


@pytest.mark.parametrize("builder", [0, 1, 2])
def test_trihedral_sweep_identical_with_mask(torch, ctx, builder):
    w = si.trihedral_case()
    say("case trihedral 181 angles, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    m, u = both(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                         samples_per_lambda=w.samples_per_lambda, flags=fl))
    frac = check_same(m, u, min_frac=0.05)
    say("masked fraction", frac)
    bvh.free()


def test_wavefront_schedule_identical_with_mask(torch, ctx):
    from paper_2604_09243_amd import sbr
    w = si.trihedral_case(n_phi=19)
    say("case trihedral 19 angles, wavefront schedule")
    bvh = ctx.build_bvh(w.V, w.T)
    m, u = both(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                         samples_per_lambda=w.samples_per_lambda, flags=fl | sbr.OPT_WAVEFRONT))
    check_same(m, u, min_frac=0.05)
    # and both equal the streaming schedule with the mask, which claims only
    # the live tiles and counts the others' rays as masked: the same count as
    # the wavefront schedule's ray-by-ray one
    A, _, st = ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                             samples_per_lambda=w.samples_per_lambda)
    assert np.array_equal(A.cpu().numpy().view(np.float64), m[0].view(np.float64))
    assert st["masked"] == m[2]["masked"] and st["queries"] == m[2]["queries"]
    bvh.free()


@pytest.mark.parametrize("tile_w", [4, 8, 16, 64])
def test_live_tiles_any_tile_width_and_chunking(torch, ctx, tile_w):
    """The live-tile list at every tile shape (a tile spans 1 x 2, 1, 2 or
    8 x 1 mask cells) and at chunks of one or a few angles: the results equal
    the unmasked sweep bit for bit and the masked count equals the
    ray-by-ray count of the wavefront schedule."""
    from paper_2604_09243_amd import sbr
    w = si.aircraft_case()
    idx = np.arange(0, w.n_angles, 90)
    say("case aircraft 4 azimuths, tile_w", tile_w)
    bvh = ctx.build_bvh(w.V, w.T, builder=1)
    run = lambda fl, **kw: ctx.rcs_sweep(bvh, w.theta_deg[idx], w.phi_deg[idx], w.freqs_hz, w.max_bounces,
                                         samples_per_lambda=w.samples_per_lambda, flags=fl, **kw)
    _, _, wf = run(sbr.OPT_WAVEFRONT)
    for chunk in (16, 24):
        tune = sbr.make_tune(tile_w=tile_w, chunk_log2=chunk)
        m, u = both(lambda fl: run(fl, tune=tune))
        check_same(m, u, min_frac=0.2)
        assert m[2]["masked"] == wf["masked"] and m[2]["queries"] == wf["queries"]
    bvh.free()


@pytest.mark.parametrize("builder", [0, 1])
def test_aircraft_angles_identical_with_mask(torch, ctx, builder):
    w = si.aircraft_case()
    idx = np.arange(0, w.n_angles, 45)
    say("case aircraft 8 azimuths, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    m, u = both(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg[idx], w.phi_deg[idx], w.freqs_hz, w.max_bounces,
                                         samples_per_lambda=w.samples_per_lambda, flags=fl))
    frac = check_same(m, u, min_frac=0.2)
    say("masked fraction", frac)
    bvh.free()


def test_mask_with_one_leaf_tree_and_tiny_grids(torch, ctx):
    """A two-triangle plate (the whole tree one leaf) at normal and grazing
    incidence, and grids smaller than one mask cell."""
    V = np.array([[-0.1, -0.1, 0.0], [0.1, -0.1, 0.0], [0.1, 0.1, 0.0], [-0.1, 0.1, 0.0]], np.float32)
    T = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    bvh = ctx.build_bvh(V, T, builder=1)
    th = np.array([0.0, 30.0, 89.0, 90.0, 120.0])
    ph = np.array([0.0, 17.0, 45.0, 0.0, 200.0])
    for ds in (C0 / 10e9 / 10, 0.15):
        say("case plate, ds", ds)
        m, u = both(lambda fl: ctx.rcs_sweep(bvh, th, ph, [10e9], 3, ds=ds, flags=fl | 4))
        check_same(m, u)
    bvh.free()


def test_batch_identical_with_mask(torch, ctx):
    from paper_2604_09243_amd import sbr
    w = si.batch_case(n_scenes=6, tri_range=(2000, 20000), angle_range=(3, 8), nf_range=(1, 4),
                      f_range=(2.0e9, 6.0e9))
    say("case batch of 6 scenes")
    bvhs = [ctx.build_bvh(s.V, s.T) for s in w.scenes]
    scn = ctx.pack_scenes(bvhs)
    for b in bvhs:
        b.free()
    res = []
    for fl in (0, sbr.OPT_NO_MASK):
        for eager in (0, sbr.OPT_NO_GRAPH, sbr.OPT_WAVEFRONT):
            b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                          flags=fl | eager)
            outs = []
            for rep in range(2):
                A, S, st = b.run()
                outs.append((A.cpu().numpy().copy(), S.cpu().numpy().copy(), dict(st)))
            assert np.array_equal(outs[0][0].view(np.float64), outs[1][0].view(np.float64))
            res.append(outs[1])
            b.close()
    for r in res[1:]:
        assert np.array_equal(r[0].view(np.float64), res[0][0].view(np.float64))
        assert r[2]["queries"] == res[0][2]["queries"]
    assert all(r[2]["masked"] > 0 for r in res[:3]) and all(r[2]["masked"] == 0 for r in res[3:])
    # live-tile lists (graph and eager streaming) and the ray-by-ray wavefront count agree
    assert res[0][2]["masked"] == res[1][2]["masked"] == res[2][2]["masked"]
    say("masked fraction", res[0][2]["masked"] / res[0][2]["rays"])
    scn.free()
