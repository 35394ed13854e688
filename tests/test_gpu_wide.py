"""The four-wide copy of the tree (SBR_OPT_BVH4, a traversal study): sweeps
and caller-ray traces that walk it give the same bits as the binary tree, on
every builder, with and without the stack spill (the aircraft's trees need
it), on the float64 study traversal too, and the copy passes the layout
check once built."""
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


def sweep_pair(ctx, bvh, w, flags=0, idx=None):
    from paper_2604_09243_amd import sbr
    th = w.theta_deg if idx is None else w.theta_deg[idx]
    ph = w.phi_deg if idx is None else w.phi_deg[idx]
    out = []
    for fl in (flags | sbr.OPT_BVH4, flags):
        A, S, st = ctx.rcs_sweep(bvh, th, ph, w.freqs_hz, w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                                 flags=fl)
        out.append((A.cpu().numpy(), S.cpu().numpy(), st))
    return out


def check_equal(a, b):
    (A4, S4, st4), (A2, S2, st2) = a, b
    assert np.array_equal(A4.view(np.float64), A2.view(np.float64))
    assert np.array_equal(S4, S2)
    for key in ("queries", "valid", "trapped", "hits", "masked", "queries_bounce"):
        assert st4[key] == st2[key], key


@pytest.mark.parametrize("builder", [0, 1, 2])
def test_trihedral_sweep_same_on_both_trees(torch, ctx, builder):
    w = si.trihedral_case()
    say("case trihedral 181 angles, wide vs binary, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    a, b = sweep_pair(ctx, bvh, w)
    bvh.validate()  # the wide copy exists now
    check_equal(a, b)
    say("queries", a[2]["queries"])
    bvh.free()


@pytest.mark.parametrize("builder", [1, 2])
def test_aircraft_azimuths_same_on_both_trees(torch, ctx, builder):
    w = si.aircraft_case()
    say("case aircraft 8 azimuths, wide vs binary, builder", builder)
    bvh = ctx.build_bvh(w.V, w.T, builder=builder)
    a, b = sweep_pair(ctx, bvh, w, idx=np.arange(0, 360, 45))
    bvh.validate()
    check_equal(a, b)
    say("queries", a[2]["queries"], "valid", a[2]["valid"])
    bvh.free()


def test_float64_traversal_same_on_both_trees(torch, ctx):
    from paper_2604_09243_amd import sbr
    w = si.trihedral_case(n_phi=19)
    say("case trihedral 19 angles, float64 traversal, wide vs binary")
    bvh = ctx.build_bvh(w.V, w.T)
    a, b = sweep_pair(ctx, bvh, w, flags=sbr.OPT_FP64_TRAVERSE)
    check_equal(a, b)
    bvh.free()


@pytest.mark.parametrize("builder", [0, 1, 2])
def test_caller_rays_same_on_both_trees(torch, ctx, orc, builder):
    """Random origins and directions around an icosphere and a trihedral:
    every result array of sbr_trace, with the per-bounce ids."""
    from paper_2604_09243_amd import sbr
    rng = np.random.default_rng(40 + builder)
    dev = torch.device("cuda", 0)
    for name, (V, T), lo, hi in (("sphere", si.icosphere(4), -1.0, 1.0), ("trihedral", si.trihedral(1.0, 8), 0.0, 1.0)):
        say("case caller rays", name, "builder", builder)
        bvh = ctx.build_bvh(V, T, builder=builder)
        n = 20_000
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        # aimed at a point of the object's box from 3 m away
        o = rng.uniform(lo, hi, size=(n, 3)) - 3.0 * d
        eh = np.cross(d, [0.3, 0.5, 0.8])
        eh /= np.linalg.norm(eh, axis=1, keepdims=True)
        ev = np.cross(eh, d)
        t = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev) for x in (o, d, eh, ev)]
        k = (0.0, 0.0, -1.0)
        r4 = ctx.trace(bvh, *t, 6, k, want_path=True, stats=True, flags=sbr.OPT_BVH4)
        r2 = ctx.trace(bvh, *t, 6, k, want_path=True, stats=True)
        torch.cuda.synchronize()
        for key, v in r4.items():
            if key == "stats":
                continue
            assert torch.equal(v, r2[key]), (name, key)
        assert r4["stats"]["queries"] == r2["stats"]["queries"]
        assert int((r4["n_bounce"] > 0).sum()) > n // 5
        bvh.free()
