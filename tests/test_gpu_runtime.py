"""The device block cache behind BVH arrays and build scratch: blocks handed
back by sbr_free_bvh are reused by later builds of any mesh and builder, and
a sweep over a tree built into reused blocks gives the same bits as over the
first tree of that mesh (stale contents never leak into a build)."""
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


def sweep(ctx, bvh, th, ph):
    A, _, _ = ctx.rcs_sweep(bvh, th, ph, [10e9, 11e9], 5, ds=C0 / 11e9 / 8)
    return A.cpu().numpy()


def test_builds_into_reused_blocks_match_fresh_builds(torch, ctx):
    say("case block cache reuse")
    th, ph = np.array([54.74, 60.0, 40.0]), np.array([45.0, 20.0, 70.0])
    meshes = [si.trihedral(1.0, 8), si.trihedral(0.5, 16), si.trihedral(1.0, 4)]
    ref = {}
    for i, (V, T) in enumerate(meshes):
        for builder in (0, 1, 2):
            b = ctx.build_bvh(V, T, builder=builder)
            ref[(i, builder)] = sweep(ctx, b, th, ph)
            b.free()
    # interleaved builds and frees of other sizes: every tree lands in blocks
    # last used by another tree (or by another build's scratch)
    rng = np.random.default_rng(3)
    live = []
    for rep in range(12):
        i, builder = int(rng.integers(len(meshes))), int(rng.integers(3))
        V, T = meshes[i]
        b = ctx.build_bvh(V, T, builder=builder)
        assert np.array_equal(sweep(ctx, b, th, ph), ref[(i, builder)]), (rep, i, builder)
        live.append(b)
        if len(live) > 2:
            live.pop(int(rng.integers(len(live)))).free()
    for b in live:
        b.free()
    say("reused builds agree bit for bit")
