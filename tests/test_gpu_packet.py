"""Packet traversal of primary tiles: the parallel primary rays of a tile walk
the tree together, every lane testing each visited node with its own ray.
A lane reaches every leaf its own walk would, so the closest hit (the
minimum of (t, id) under the hit rule, Algorithm 2) cannot change: each case
compares a sweep with SBR_OPT_PACKET against the same sweep without it
(every ray on its own, the default), bit for bit, with equal query and hit
counts."""
import sys

import numpy as np
import pytest

import sbr_inputs as si

pytestmark = pytest.mark.gpu


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


def check_same(run):
    from paper_2604_09243_amd import sbr
    A1, S1, st1 = run(sbr.OPT_PACKET)
    A0, S0, st0 = run(0)
    assert np.array_equal(A1.cpu().numpy().view(np.float64), A0.cpu().numpy().view(np.float64))
    assert np.array_equal(S1.cpu().numpy(), S0.cpu().numpy())
    for k in ("queries", "hits", "valid", "masked", "rays"):
        assert st1[k] == st0[k], k
    return st1


@pytest.mark.parametrize("builder", [0, 1, 2])
def test_trihedral_sweep(torch, ctx, builder):
    w = si.trihedral_case()
    say("case trihedral 181 angles, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    check_same(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                        samples_per_lambda=w.samples_per_lambda, flags=fl))
    bvh.free()


@pytest.mark.parametrize("builder", [1, 2])
def test_aircraft_azimuths(torch, ctx, builder):
    w = si.aircraft_case()
    idx = np.arange(0, w.n_angles, 45)
    say("case aircraft 8 azimuths, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    for extra in (0, 64):  # with the primary-ray mask and without (every tile traced)
        check_same(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg[idx], w.phi_deg[idx], w.freqs_hz, w.max_bounces,
                                            samples_per_lambda=w.samples_per_lambda, flags=fl | extra))
    bvh.free()


@pytest.mark.parametrize("tile_w", [4, 16, 64])
def test_tile_shapes_and_partial_refills(torch, ctx, tile_w):
    """Other tile shapes, and refills below a whole wave (waves then mix rays
    of several tiles and bounces: they take the per-lane walk whenever a
    lane is not a primary ray of the wave's direction)."""
    from paper_2604_09243_amd import sbr
    w = si.trihedral_case(n_phi=37)
    say("case trihedral 37 angles, tile_w", tile_w)
    bvh = ctx.build_bvh(w.V, w.T, builder=1)
    for refill in (64, 16):
        tune = sbr.make_tune(tile_w=tile_w, refill_min=refill)
        check_same(lambda fl: ctx.rcs_sweep(bvh, w.theta_deg, w.phi_deg, w.freqs_hz, w.max_bounces,
                                            samples_per_lambda=w.samples_per_lambda, flags=fl, tune=tune))
    bvh.free()


def test_batch(torch, ctx):
    from paper_2604_09243_amd import sbr
    w = si.batch_case(n_scenes=6, tri_range=(2000, 20000), angle_range=(3, 8), nf_range=(1, 4),
                      f_range=(2.0e9, 6.0e9))
    say("case batch of 6 scenes")
    bvhs = [ctx.build_bvh(s.V, s.T) for s in w.scenes]
    scn = ctx.pack_scenes(bvhs)
    for b in bvhs:
        b.free()
    out = []
    for fl in (sbr.OPT_PACKET, 0):
        b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda, flags=fl)
        A, S, st = b.run()
        out.append((A.cpu().numpy().copy(), dict(st)))
        b.close()
    assert np.array_equal(out[0][0].view(np.float64), out[1][0].view(np.float64))
    assert out[0][1]["queries"] == out[1][1]["queries"]
    scn.free()
