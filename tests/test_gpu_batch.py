"""Batched sweeps over many scenes in one persistent launch per chunk,
replayed from a captured HIP graph: parity with the oracle on every item of a
reduced batch and on sampled items of the full 64-scene batch, bitwise
agreement with per-scene sweeps, across graph replays, eager runs and launch
parameters, and the error paths."""
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


def build_set(ctx, w):
    bvhs = [ctx.build_bvh(s.V, s.T) for s in w.scenes]
    return bvhs, ctx.pack_scenes(bvhs)


def sweeps_of(ctx, bvhs, w, **kw):
    """Per-scene sbr_rcs_sweep results stacked in batch row order."""
    out = []
    for b, s in zip(bvhs, w.scenes):
        A, _, _ = ctx.rcs_sweep(b, s.theta_deg, s.phi_deg, s.freqs_hz, w.max_bounces,
                                samples_per_lambda=w.samples_per_lambda, **kw)
        out.append(A.cpu().numpy().reshape(-1, 2, 2))
    return np.concatenate(out)


def check_item_vs_oracle(orc, mesh, s, A_rows, bmax, spl):
    """Complex error <= 1e-4 of the item's max, dB within 0.05 within 40 dB."""
    r = orc.rcs_angle(mesh, s[0], s[1], s[2], ds=C0 / float(np.max(s[2])) / spl, bmax=bmax, use_bvh=True)
    A_o = r["A"]
    amax = np.abs(A_o).max()
    if amax == 0.0:
        assert np.abs(A_rows).max() == 0.0
        return 0.0
    err = np.abs(A_rows - A_o) / np.maximum(np.abs(A_o), 1e-3 * amax)
    assert err.max() <= 1e-4, err.max()
    so = 10 * np.log10(np.maximum(4 * np.pi * np.abs(A_o) ** 2, 1e-300))
    sg = 10 * np.log10(np.maximum(4 * np.pi * np.abs(A_rows) ** 2, 1e-300))
    sel = so >= so.max() - 40
    assert np.abs(so - sg)[sel].max() <= 0.05
    return err.max()


@pytest.fixture(scope="module")
def small(torch, ctx):
    w = si.batch_case(n_scenes=5, tri_range=(2000, 8000), angle_range=(2, 5), nf_range=(1, 3),
                      f_range=(2.0e9, 5.0e9))
    bvhs, scn = build_set(ctx, w)
    return w, bvhs, scn


def test_small_batch_matches_oracle_item_by_item(torch, ctx, orc, small):
    w, bvhs, scn = small
    say("case small batch vs oracle")
    items = w.items()
    fr = w.freqs()
    b = ctx.batch(scn, items, fr, w.max_bounces, samples_per_lambda=w.samples_per_lambda)
    A, S, st = b.run()
    A = A.cpu().numpy()
    info = b.info()
    assert info["n_items"] == len(items) and info["n_rows"] == sum(it[4] for it in items)
    assert st["angles"] == len(items) and st["rays"] == info["rays"]
    meshes = [orc.Mesh(s.V, s.T).build_bvh() for s in w.scenes]
    worst = 0.0
    for i, (sc, th, ph, off, nf) in enumerate(items):
        r0 = b.row_offset[i]
        worst = max(worst, check_item_vs_oracle(orc, meshes[sc], (th, ph, fr[off:off + nf]), A[r0:r0 + nf],
                                                w.max_bounces, w.samples_per_lambda))
    say("items", len(items), "worst complex error", worst)
    # sigma is 10 log10(4 pi |A|^2)
    Sg = S.cpu().numpy()
    ref = 10 * np.log10(np.maximum(4 * np.pi * np.abs(A) ** 2, 1e-300))
    sel = np.abs(A) > 0
    assert np.allclose(Sg[sel], ref[sel], rtol=0, atol=1e-9)


def test_small_batch_equals_per_scene_sweeps_and_replays(torch, ctx, small):
    w, bvhs, scn = small
    say("case small batch replays")
    from paper_2604_09243_amd import sbr
    b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda)
    ref = sweeps_of(ctx, bvhs, w)
    outs = []
    for rep in range(4):
        A, _, _ = b.run(stats=(rep % 2 == 0))
        outs.append(A.cpu().numpy().copy())
        # eager work on the same stream between replays
        x = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert b.info()["graph_ready"] == 1
    for o in outs:
        assert np.array_equal(o, ref)
    e = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                  flags=sbr.OPT_NO_GRAPH)
    A, _, st = e.run()
    assert np.array_equal(A.cpu().numpy(), ref)
    assert st["ms_trace"] > 0 and st["ms_po"] > 0
    # launch parameters and chunking change nothing
    for kw in (dict(tile_w=4, chunk_log2=16), dict(claim_tiles=1, refill_min=1), dict(tile_w=32, blocks_per_cu=2),
               dict(schedule=1)):
        b.set_tune(sbr.make_tune(**kw))
        assert b.info()["graph_ready"] == 0
        A, _, _ = b.run()
        assert np.array_equal(A.cpu().numpy(), ref), kw
    assert b.info()["n_chunks"] >= 1
    t = b.autotune()
    A, _, _ = b.run()
    assert np.array_equal(A.cpu().numpy(), ref)
    say("autotuned", t.as_dict())


def test_batch_paper_mode_and_flags(torch, ctx, small):
    w, bvhs, scn = small
    say("case batch paper mode")
    from paper_2604_09243_amd import sbr
    for mode, flags in ((sbr.MODE_PAPER, 0), (sbr.MODE_VECTOR, sbr.OPT_DROP_TRAPPED | sbr.OPT_PAPER_PATH)):
        b = ctx.batch(scn, w.items(), w.freqs(), w.max_bounces, samples_per_lambda=w.samples_per_lambda,
                      mode=mode, flags=flags)
        A, _, _ = b.run()
        ref = sweeps_of(ctx, bvhs, w, mode=mode, flags=flags)
        assert np.array_equal(A.cpu().numpy(), ref)


def test_batch_errors(torch, ctx, small):
    w, bvhs, scn = small
    say("case batch errors")
    from paper_2604_09243_amd import sbr
    fr = w.freqs()
    bad = [[(len(w.scenes), 10.0, 0.0, 0, 1)],         # scene index out of range
           [(0, 10.0, 0.0, len(fr) - 1, 2)],            # frequencies outside the array
           [(0, 10.0, 0.0, 0, 0)]]                      # no frequency
    for items in bad:
        with pytest.raises(sbr.SbrError) as e:
            ctx.batch(scn, items, fr, 5)
        assert e.value.status == sbr.ERR_INVALID_ARG
    with pytest.raises(sbr.SbrError) as e:
        ctx.batch(scn, [(0, 10.0, 0.0, 0, 1, C0 / fr[0] / 4)], fr, 5)   # coarser than lambda/5
    assert e.value.status == sbr.ERR_SAMPLING
    with pytest.raises(sbr.SbrError):
        ctx.pack_scenes([scn])                          # a set of sets
    with pytest.raises(sbr.SbrError):
        ctx.rcs_sweep(scn, [10.0], [0.0], [3e9], 5)     # sets serve batches only
    one = ctx.batch(bvhs[0], [(0, 10.0, 0.0, 0, 1)], fr, 5)   # a single BVH is a one-scene batch
    A, _, _ = one.run()
    assert A.shape == (1, 2, 2)


@pytest.fixture(scope="module")
def full(torch, ctx):
    """The 64-scene batch on host SAH trees, run once."""
    w = si.batch_case()
    bvhs, scn = build_set(ctx, w)
    assert scn.n_scenes == 64 and 8e6 < scn.n_tris < 9e6
    items, fr = w.items(), w.freqs()
    b = ctx.batch(scn, items, fr, w.max_bounces, samples_per_lambda=w.samples_per_lambda)
    A1, _, st = b.run()
    return dict(w=w, bvhs=bvhs, scn=scn, items=items, fr=fr, b=b, A=A1.cpu().numpy().copy(), st=st)


def test_full_batch_64_scenes(torch, ctx, full):
    say("case full 64-scene batch")
    w, bvhs, items, b, A1, st = full["w"], full["bvhs"], full["items"], full["b"], full["A"], full["st"]
    info = b.info()
    assert info["max_item_rays"] > 50 * info["min_item_rays"]
    A2, _, st2 = b.run()
    assert np.array_equal(A1, A2.cpu().numpy())
    say("rays", st["rays"], "queries", st["queries"], "graph ms", st["ms_total"], "items", len(items),
        "chunks", info["n_chunks"])
    assert st["queries"] == st2["queries"]
    # per-scene sweeps agree bit for bit on 8 scenes spread over the batch
    pick = list(range(0, 64, 8))
    off = 0
    rows = {}
    for si_, s in enumerate(w.scenes):
        n = len(s.theta_deg) * len(s.freqs_hz)
        rows[si_] = (off, n)
        off += n
    for k in pick:
        s = w.scenes[k]
        A, _, _ = ctx.rcs_sweep(bvhs[k], s.theta_deg, s.phi_deg, s.freqs_hz, w.max_bounces,
                                samples_per_lambda=w.samples_per_lambda)
        r0, n = rows[k]
        assert np.array_equal(A.cpu().numpy().reshape(-1, 2, 2), A1[r0:r0 + n]), k


def test_full_batch_identical_across_builders(torch, ctx, full):
    """Every one of the 154,028 result rows is the same on the GPU LBVH, the
    host SAH and the GPU PLOC trees: the closest hit is the minimum over all
    triangles, whatever tree finds it."""
    say("case full batch across builders")
    from paper_2604_09243_amd import sbr
    w, items, fr, A1 = full["w"], full["items"], full["fr"], full["A"]
    assert len(A1) == 154_028
    for builder in (sbr.BUILD_LBVH, sbr.BUILD_PLOC):
        bvhs = [ctx.build_bvh(s.V, s.T, builder=builder) for s in w.scenes]
        scn = ctx.pack_scenes(bvhs)
        for x in bvhs:
            x.free()
        b = ctx.batch(scn, items, fr, w.max_bounces, samples_per_lambda=w.samples_per_lambda)
        A, _, _ = b.run()
        A = A.cpu().numpy()
        bad = np.flatnonzero(np.any(A != A1, axis=(1, 2)))
        say("builder", builder, "rows differing from the SAH trees", len(bad))
        assert len(bad) == 0, bad[:20]
        b.close()
        scn.free()


# Items whose rows differed between trees before the hit rule's box test
# made the closest hit tree-independent (found by comparing the three trees'
# batches; the oracle, brute-force-pinned, decides them here).
TREE_SENSITIVE_ITEMS = (5988, 7238)


@pytest.mark.parametrize("group", [0, 1, 2, 3])
def test_full_batch_oracle_parity(torch, orc, full, group):
    """Oracle parity on the first item of each of 16 scenes (a quarter of the
    64 per test), and on the tree-sensitive items of those scenes."""
    w, items, fr, b, A1 = full["w"], full["items"], full["fr"], full["b"], full["A"]
    scenes = range(16 * group, 16 * group + 16)
    say("case full batch oracle parity, scenes", scenes[0], "to", scenes[-1])
    worst = 0.0
    for k in scenes:
        s = w.scenes[k]
        m = orc.Mesh(s.V, s.T).build_bvh()
        mine = [i for i, it in enumerate(items) if it[0] == k]
        for i in [mine[0]] + [i for i in TREE_SENSITIVE_ITEMS if items[i][0] == k]:
            sc, th, ph, o, nf = items[i]
            r0 = b.row_offset[i]
            e = check_item_vs_oracle(orc, m, (th, ph, fr[o:o + nf]), A1[r0:r0 + nf], w.max_bounces,
                                     w.samples_per_lambda)
            worst = max(worst, e)
    say("worst complex error", worst)


@pytest.mark.parametrize("item,ray", [(5988, 4667867), (7238, 1895418)])
def test_tree_sensitive_rays_on_every_builder(torch, ctx, orc, item, ray):
    """The two rays whose closest hit depended on the tree before the hit
    rule's box test: every GPU builder's tree gives the oracle's brute-force
    result (ids at every bounce, hit point, phase path)."""
    from paper_2604_09243_amd import sbr
    say("case tree-sensitive ray of item", item)
    w = si.batch_case(n_scenes=64)
    items, fr = w.items(), w.freqs()
    sc, th, ph, off, nf = items[item]
    s = w.scenes[sc]
    m = orc.Mesh(s.V, s.T)
    ds = C0 / float(np.max(fr[off:off + nf])) / w.samples_per_lambda
    o, d, _, _ = orc.gen_rays(m.bbox, th, ph, ds)
    k, tv, pv = orc.frame(th, ph)
    o = o[ray:ray + 1]
    r = orc.trace(m, o, d, pv, tv, k, w.max_bounces, want_path=True)
    dev = torch.device("cuda", 0)
    t = [torch.from_numpy(np.ascontiguousarray(np.broadcast_to(x, (1, 3)).astype(np.float32))).to(dev)
         for x in (o, d, pv, tv)]
    for builder in (sbr.BUILD_LBVH, sbr.BUILD_SAH, sbr.BUILD_PLOC):
        bvh = ctx.build_bvh(s.V, s.T, builder=builder)
        g = {kk: v.cpu().numpy() for kk, v in ctx.trace(bvh, *t, w.max_bounces, k, want_path=True).items()}
        assert np.array_equal(r["tri_path"], g["tri_path"]), builder
        assert np.array_equal(r["x_last"], g["x_last"]) and np.array_equal(r["D"], g["D"]), builder
        bvh.free()
