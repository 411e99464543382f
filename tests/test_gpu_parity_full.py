"""Parity at the benchmark configurations' full sizes, through the C ABI.

  - guided 512 x 512 heightfield (132k triangles, max depth 10): a whole
    schedule of 3 classic and 3 MARS iterations at 1 spp over every pixel,
    the octree, visits, accumulators, factors and directional distributions
    after every update and the radiance of every camera sample;
  - bidirectional 1280 x 720 interior (1.04M triangles; with one light-path
    budget and with per-length budgets) and the learned-cache workload's
    1920 x 1080 interior (2.08M triangles), max path length 12: the octree
    grown by both sides over two classic iterations over every pixel, then a
    MARS iteration on it, compared on sampled pixels;
  - the Cornell box's MARS schedule: its image mean within 3 sigma of a
    65,536 spp render of the oracle (tests/golden/cornell64_d5_mean.json).
Bars as in test_gpu_parity.py."""
import json
import math
import os

import numpy as np
import pytest

import scenegen
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
RTOL_RAD = 1e-4


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_20429_amd import api
    c = api.Context(0)
    yield c
    c.close()


def say(*a):
    print("[gpu-test]", *a, flush=True)


def _params(**kw):
    from paper_2410_20429_amd import api
    return api.iter_params(**kw), orc.Oracle.params(**kw)


def _cmp_radiance(a, b, what):
    err = np.abs(a - b) / np.maximum(np.abs(b), 1e-3)
    bad = np.flatnonzero(np.any(err > RTOL_RAD, axis=-1))
    assert bad.size == 0, (what, len(bad), float(err.max()), a[bad[0]], b[bad[0]])


def _cmp_vertices(dg, do):
    assert len(dg) == len(do), (len(dg), len(do))
    kg = np.sort(dg, order=["root", "depth", "stream_lo", "stream_hi"])
    ko = np.sort(do, order=["root", "depth", "stream_lo", "stream_hi"])
    for f in ("root", "depth", "stream_lo", "stream_hi", "cell", "gamma"):
        assert np.array_equal(kg[f], ko[f]), f
    assert np.array_equal(kg["beta"].view(np.uint32), ko["beta"].view(np.uint32))
    assert np.array_equal(kg["T"].view(np.uint32), ko["T"].view(np.uint32))


def _cmp_cache(g, o, guided=False):
    assert g.ncells == o.ncells
    assert np.array_equal(g.nodes(), o.nodes())
    cg, co = g.cells(), o.cells()
    assert np.array_equal(cg["visits"], co["visits"])
    assert np.array_equal(cg["depth"], co["depth"])
    assert np.allclose(cg["acc"], co["acc"], rtol=1e-9, atol=1e-12)
    fa, fb = cg["factors"], co["factors"]
    # binary64 sums in another order may round to a neighbouring binary32
    assert np.allclose(fa, fb, rtol=1e-6, atol=0)
    assert np.mean(fa.view(np.uint32) != fb.view(np.uint32)) < 1e-3
    if guided:
        pg, cdg = g.hist()
        po, cdo = o.hist()
        assert np.allclose(pg, po, rtol=1e-6, atol=1e-9)
        assert np.allclose(cdg, cdo, rtol=1e-6, atol=1e-9)


def test_guided_full_schedule(ctx):
    from paper_2410_20429_amd import api
    sc = scenegen.make_heightfield_scene(seed=1)
    say("guided full schedule:", sc["width"], "x", sc["height"], sc["V"].shape[0], "tris")
    g = api.Scene(ctx, sc, mode=api.MODE_PT_GUIDED, max_depth=10, max_cells=54054)
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=10, max_cells=54054)
    for it in range(6):
        alloc = orc.ALLOC_CLASSIC if it < 3 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=1, alloc=alloc, stat_clamp=50.0, debug_depth=2)
        say("guided full schedule, iteration", it)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance(), f"iteration {it}")
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        assert sg.total_rays() == so.total_rays()
        _cmp_cache(g, o, guided=True)
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-9 * uo.V_I
        assert ug.n_cells_after == uo.n_cells_after
        _cmp_cache(g, o, guided=True)
        assert np.allclose(g.itilde(), o.itilde(), rtol=1e-6, atol=0)
    assert g.ncells > 1000
    g.release()


def _grown_then_sampled(ctx, sc, n_pix, seed, lp_lengths=False):
    """Two classic iterations over every pixel on both sides (the octree and
    the factors grow from their statistics), then a MARS iteration compared
    on n_pix sampled pixels (with per-length light-path budgets: the class
    cells too)."""
    from paper_2410_20429_amd import api
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12, lp_lengths=lp_lengths)
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=12, lp_classes=3 if lp_lengths else 1)
    for it in range(2):
        pg, po = _params(iteration=it, spp=1, stat_clamp=0.0)
        say("grow octree, classic iteration", it)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        assert sg.total_rays() == so.total_rays()
        _cmp_radiance(g.sample_radiance(), o.sample_radiance(), f"classic iteration {it}")
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-9 * uo.V_I
        _cmp_cache(g, o)
        if lp_lengths:
            xg, xo = g.cells_x(), o.cells_x()
            assert np.allclose(xg["acc"], xo["acc"], rtol=1e-9, atol=1e-12)
            assert np.allclose(xg["factors"], xo["factors"], rtol=1e-6, atol=0)
    assert g.ncells >= 64
    rng = np.random.default_rng(seed)
    pix = rng.choice(sc["width"] * sc["height"], n_pix, replace=False)
    o.set_pixel_subset(pix)
    pg, po = _params(iteration=2, spp=1, alloc=api.ALLOC_MARS, stat_clamp=0.0, debug_depth=3)
    say("MARS iteration on the grown octree,", n_pix, "sampled pixels")
    g.render_iteration(pg)
    o.render_iteration(po)
    _cmp_radiance(g.sample_radiance()[pix], o.sample_radiance()[pix], "MARS iteration")
    dg = g.debug_vertices()
    dg = dg[np.isin(dg["root"], pix)]
    do = o.debug_vertices()
    _cmp_vertices(dg, do)
    assert np.any(dg["gamma"][:, 2] > 1)  # splitting of light-path samples happened
    if lp_lengths:
        kg = np.sort(dg, order=["root", "depth", "stream_lo", "stream_hi"])
        ko = np.sort(do, order=["root", "depth", "stream_lo", "stream_hi"])
        assert np.array_equal(kg["gamma_x"], ko["gamma_x"])
        assert np.array_equal(kg["beta_x"].view(np.uint32), ko["beta_x"].view(np.uint32))
    g.release()


def test_bdpt_grown_octree_sampled(ctx):
    sc = scenegen.make_interior(seed=1)
    say("bidirectional interior", sc["width"], "x", sc["height"], sc["V"].shape[0], "tris")
    _grown_then_sampled(ctx, sc, 1024, 29)


def test_bdpt_lp_lengths_grown_octree_sampled(ctx):
    sc = scenegen.make_interior(seed=1)
    say("bidirectional interior, per-length light paths", sc["width"], "x", sc["height"])
    _grown_then_sampled(ctx, sc, 512, 37, lp_lengths=True)


def test_learned_scene_grown_octree_sampled(ctx):
    sc = scenegen.make_interior(seed=3, width=1920, height=1080, n_pieces=4500)
    say("learned-cache scene", sc["width"], "x", sc["height"], sc["V"].shape[0], "tris")
    _grown_then_sampled(ctx, sc, 512, 31)


def test_cornell_image_mean_vs_oracle_64k(ctx):
    """The Cornell box's MARS schedule (1 classic + 4 MARS iterations of 1 spp,
    max depth 5): the mean of every camera sample's radiance is within 3
    sigma of the oracle's 65,536 spp render with counts of one (MARS is
    unbiased for any counts)."""
    from paper_2410_20429_amd import api
    ref = json.load(open(os.path.join(HERE, "golden", "cornell64_d5_mean.json")))
    sc = scenegen.make_cornell(64, 64)
    L = []
    for rep in range(16):  # independent schedules (random-stream seeds) for the spread
        g = api.Scene(ctx, sc, max_depth=5, seed=1000 + rep)
        for it in range(5):
            p = api.iter_params(iteration=it, spp=1,
                                alloc=api.ALLOC_CLASSIC if it < 1 else api.ALLOC_MARS)
            g.render_iteration(p)
            L.append(g.sample_radiance().astype(np.float64).mean(0))
            g.update(p)
        g.release()
    L = np.array(L)
    se = np.sqrt(L.var(0, ddof=1) / len(L) + np.array(ref["stderr_rgb"]) ** 2)
    z = (L.mean(0) - np.array(ref["mean_rgb"])) / se
    say("image mean", L.mean(0), "oracle 64k spp", ref["mean_rgb"], "z", z)
    assert np.all(np.abs(z) < 3.0), z
