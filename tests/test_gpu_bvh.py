"""The three BVH builders (GPU linear BVH, host binned SAH, GPU PLOC
clustering) produce valid layouts over the same triangles, and the sweep
results do not depend on the tree: the closest hit is the smallest (t, id)
whatever order the nodes are visited in, and the PO sums are exact integer
sums, so A is bitwise the same for every builder and leaf size."""
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


def _tiny(n):
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.2], [0.5, 0.5, 1.0]], np.float32)
    T = np.array([[0, 1, 2], [1, 3, 2], [0, 1, 4], [1, 3, 4], [2, 3, 4]], np.int32)[:n]
    return V, T


MESHES = {
    # n <= leaf size, and just above it
    "tiny2": lambda: _tiny(2),
    "tiny5": lambda: _tiny(5),
    # clustering finished inside one workgroup (at most 2048 clusters)
    "trihedral16": lambda: si.trihedral(1.0, 16),
    "soup2048": lambda: si.random_triangles(2048, seed=5, box=1.0, size=0.2),
    # whole-array steps first, then the workgroup
    "soup2049": lambda: si.random_triangles(2049, seed=6, box=1.0, size=0.2),
    "sphere20480": lambda: si.icosphere(5),
    "soup60000": lambda: si.random_triangles(60000, seed=7, box=2.0, size=0.05),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_layouts_valid_for_every_builder(torch, ctx, name):
    V, T = MESHES[name]()
    say("case layout", name, len(T))
    for builder in (0, 1, 2):
        for leaf in (1, 2, 4):
            b = ctx.build_bvh(V, T, leaf_size=leaf, builder=builder)
            b.validate()
            assert b.n_live == len(T)
            assert 1 <= b.n_nodes <= max(1, len(T) - 1)
            assert b.depth >= 1
            if builder == 2:
                # the build is deterministic
                b2 = ctx.build_bvh(V, T, leaf_size=leaf, builder=builder)
                assert (b2.n_nodes, b2.depth) == (b.n_nodes, b.depth)
                b2.free()
            say(name, "builder", builder, "leaf", leaf, "nodes", b.n_nodes, "depth", b.depth)
            b.free()


@pytest.mark.parametrize("name", ["trihedral16", "sphere20480"])
def test_sweeps_identical_across_builders(torch, ctx, name):
    V, T = MESHES[name]()
    say("case sweep across builders", name)
    th, ph = np.array([54.74, 60.0, 90.0]), np.array([45.0, 20.0, 0.0])
    ref = None
    for builder in (0, 1, 2):
        for leaf in (1, 4):
            b = ctx.build_bvh(V, T, leaf_size=leaf, builder=builder)
            b.validate()
            A, _, st = ctx.rcs_sweep(b, th, ph, [10e9], 5, ds=C0 / 10e9 / 6)
            A = A.cpu().numpy()
            if ref is None:
                ref = (A, st["queries"], st["hits"])
            assert np.array_equal(A, ref[0]), (builder, leaf)
            assert st["queries"] == ref[1] and list(st["hits"]) == list(ref[2])
            b.free()
