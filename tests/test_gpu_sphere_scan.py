"""Sphere frequency scan against the Mie series (the paper's sphere
validation, Sec. 5.1, reduced): a unit PEC sphere (icosphere, 327,680
triangles) traced once at the paper's fixed ray spacing (2.05 m / 22,000)
with 40 frequencies spanning kr = 10 ... 12,000, and a ray-spacing study at
kr = 1000.  The paper places the onset of the optical region near kr = 30
and the onset of aliasing near a spacing of lambda / 8.4 (golden values in
tests/golden/paper_numbers.json); the thresholds below sit between the
errors measured on either side of those onsets, in the paper's own PO mode
(first-hit obliquity).  Mie values: tests/golden/sphere_scan_mie.json."""
import json
import os
import sys

import numpy as np
import pytest

import sbr_inputs as si

pytestmark = pytest.mark.gpu

C0 = 299_792_458.0
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


@pytest.fixture(scope="module")
def mie():
    return json.load(open(os.path.join(GOLDEN, "sphere_scan_mie.json")))


@pytest.fixture(scope="module")
def sphere(ctx):
    V, T = si.meshes.icosphere(7, 1.0)
    bvh = ctx.build_bvh(V, T, builder=1)
    yield bvh
    bvh.free()


def test_scan_optical_onset_near_kr_30(torch, ctx, mie, sphere):
    from paper_2604_09243_amd import sbr
    paper = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    kr = np.array(mie["kr_scan"])
    ds = paper["sphere_aperture_m"] / paper["sphere_rays_per_side"]
    say("case sphere scan, kr 10..12000, ds", ds)
    A, S, st = ctx.rcs_sweep(sphere, [0.0], [0.0], kr * C0 / (2 * np.pi), 5, ds=ds, mode=sbr.MODE_PAPER)
    S = S.cpu().numpy()[0]
    assert np.array_equal(S[:, 0, 0], S[:, 1, 1])  # co-polar only in this mode
    err = np.abs(S[:, 0, 0] - np.array(mie["mie_scan_dbsm"]))
    onset = paper["sphere_optical_onset_kr"]
    res, opt = kr < onset, (kr >= onset) & (kr <= 2400)
    say("rays", st["rays"], "max error below kr 30: %.3f dB, kr 30-2400: %.3f dB" % (err[res].max(), err[opt].max()))
    assert err[opt].max() <= 0.2
    assert err[res].max() >= 0.3
    # the whole scan is one trace: one ray per grid point, PO over 40 frequencies
    assert st["angles"] == 1 and S.shape[0] == 40


def test_spacing_aliasing_onset_near_lambda_over_8(torch, ctx, mie, sphere):
    from paper_2604_09243_amd import sbr
    f = mie["kr_spacing"] * C0 / (2 * np.pi)
    lam = C0 / f
    ref = mie["mie_spacing_dbsm"]
    th, ph = [0.0, 30.0, 60.0], [0.0, 10.0, 20.0]  # a sphere: the same sigma from every direction
    worst = {}
    for spl in (40, 20, 10, 8, 6, 5):
        say("case spacing lambda /", spl)
        for mode in (sbr.MODE_PAPER, sbr.MODE_VECTOR):
            _, S, _ = ctx.rcs_sweep(sphere, th, ph, [f], 5, ds=lam / spl, mode=mode)
            worst[(spl, mode)] = float(np.abs(S.cpu().numpy()[:, 0, 0, 0] - ref).max())
    say({"/".join(map(str, k)): round(v, 3) for k, v in worst.items()})
    P, Vm = sbr.MODE_PAPER, sbr.MODE_VECTOR
    # fine sampling converges to Mie in both modes
    assert worst[(40, P)] <= 0.15 and worst[(40, Vm)] <= 0.15
    # PAPER mode: clean down to lambda/10, aliasing from lambda/8 on
    assert max(worst[(20, P)], worst[(10, P)]) <= 0.2
    assert max(worst[(8, P)], worst[(6, P)], worst[(5, P)]) >= 0.25
    # VECTOR mode (the field carried to the last facet) aliases on the grazing
    # rim already at coarser-than-lambda/20 spacings
    assert worst[(10, Vm)] >= 0.4
