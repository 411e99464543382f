"""Parity of the HIP path (through the C ABI) with the CPU oracle on the same
seeded inputs.  Bars: bit-exact for integers (cells, rounded counts, octree
nodes, visit counts) and for the binary32 building blocks; per-pixel
radiance within 1e-4 relative; binary64 accumulators within 1e-9 relative
(their summation order differs: atomics on the GPU)."""
import math
import os

import numpy as np
import pytest

import scenegen
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

RTOL_RAD = 1e-4


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_20429_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _api():
    from paper_2410_20429_amd import api
    return api


def say(*a):
    print("[gpu-test]", *a, flush=True)


def _pair(ctx, sc, **kw):
    api = _api()
    g = api.Scene(ctx, sc, **kw)
    okw = {k: v for k, v in kw.items() if k not in ("queue_capacity", "tile_roots")}
    o = orc.Oracle(sc, **okw)
    return g, o


def _params(**kw):
    return _api().iter_params(**kw), orc.Oracle.params(**kw)


def _cmp_radiance(a, b, rtol=RTOL_RAD):
    err = np.abs(a - b) / np.maximum(np.abs(b), 1e-3)
    bad = np.argwhere(err > rtol)
    assert bad.size == 0, (len(bad), err.max(), a[bad[0][0]], b[bad[0][0]])


def _cmp_vertices(dg, do, exact_T=True):
    assert len(dg) == len(do), (len(dg), len(do))
    kg = np.sort(dg, order=["root", "depth", "stream_lo", "stream_hi"])
    ko = np.sort(do, order=["root", "depth", "stream_lo", "stream_hi"])
    for f in ("root", "depth", "stream_lo", "stream_hi", "cell", "gamma"):
        assert np.array_equal(kg[f], ko[f]), f
    assert np.array_equal(kg["beta"].view(np.uint32), ko["beta"].view(np.uint32))
    if exact_T:
        assert np.array_equal(kg["T"].view(np.uint32), ko["T"].view(np.uint32))


# ---------------------------------------------------------------------------
# building blocks, bit-exact
# ---------------------------------------------------------------------------
def test_probe_philox_bitexact(ctx):
    say("probe philox")
    rng = np.random.default_rng(0)
    inp = rng.integers(0, 2 ** 32, (20000, 6), dtype=np.uint64).astype(np.uint32)
    out = ctx.probe(0, inp, (20000, 4), np.uint32)
    ref = np.array([orc.philox(r[:2], r[2:]) for r in inp[:2000]])
    assert np.array_equal(out[:2000], ref)


def test_probe_sincos_bitexact(ctx):
    say("probe sincos")
    u = (np.arange(0, 1 << 24, 97, dtype=np.int64) / float(1 << 24)).astype(np.float32)
    out = ctx.probe(1, u, (u.shape[0], 2), np.float32)
    idx = np.linspace(0, len(u) - 1, 3000).astype(int)
    ref = np.array([orc.sincos2pi(float(u[i])) for i in idx], np.float32)
    assert np.array_equal(out[idx].view(np.uint32), ref.view(np.uint32))


def test_probe_alg1_bitexact(ctx):
    say("probe alg1")
    rng = np.random.default_rng(1)
    b = rng.uniform(0.0, 20.0, (5000, 3)).astype(np.float32)
    u = (rng.integers(0, 1 << 24, 5000) / float(1 << 24)).astype(np.float32)
    inp = np.concatenate([b, u[:, None]], 1).astype(np.float32)
    out = ctx.probe(2, inp, (5000, 3), np.uint32)
    ref = np.array([orc.alg1(r[:3], r[3]) for r in inp])
    assert np.array_equal(out, ref)


# ---------------------------------------------------------------------------
# Cornell box, depth <= 2: radiance per camera sample and per-vertex decisions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("center", [True, False])
def test_cornell_depth2_parity(ctx, center):
    sc = scenegen.make_cornell(64, 64)
    g, o = _pair(ctx, sc, max_depth=2)
    for it in range(3):
        say("cornell D2 iteration", it, "center", center)
        alloc = orc.ALLOC_CLASSIC if it == 0 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=4, alloc=alloc, center_jitter=center, debug_depth=2)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        assert sg.total_rays() == so.total_rays()
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-6 * uo.V_I
        assert np.array_equal(g.nodes(), o.nodes())


# ---------------------------------------------------------------------------
# full MARS schedule on the Cornell box (max depth 5): every iteration's
# decisions, radiance, cells, factors, octree and pixel estimates
# ---------------------------------------------------------------------------
def _cmp_cells(g, o, exact_factors=True):
    cg, co = g.cells(), o.cells()
    assert np.array_equal(cg["visits"], co["visits"])
    assert np.array_equal(cg["depth"], co["depth"])
    a, b = cg["acc"], co["acc"]
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12)
    fa, fb = cg["factors"], co["factors"]
    if exact_factors:
        mism = np.sum(fa.view(np.uint32) != fb.view(np.uint32))
        assert mism <= 2, mism  # float64 sums of different order may round differently (rare)
    assert np.allclose(fa, fb, rtol=1e-6, atol=0)


@pytest.mark.parametrize("aware", [True, False])
def test_cornell_mars_schedule_parity(ctx, aware):
    sc = scenegen.make_cornell(64, 64)
    g, o = _pair(ctx, sc, max_depth=5)
    for it in range(5):
        say("cornell D5 iteration", it, "aware", aware)
        alloc = orc.ALLOC_CLASSIC if it == 0 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=1, alloc=alloc, budget_aware=aware, debug_depth=5)
        g.render_iteration(pg)
        o.render_iteration(po)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        _cmp_cells(g, o)
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-9 * uo.V_I
        assert ug.C_I == uo.C_I
        assert np.array_equal(g.nodes(), o.nodes())
        assert np.array_equal(g.itilde().view(np.uint32), o.itilde().view(np.uint32))
        _cmp_cells(g, o)
    np.testing.assert_allclose(g.image(0), o.image(0), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(g.image(1), o.image(1), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(g.count_map(), o.count_map(), rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# guided technique (small heightfield scene, GGX): directional histograms
# ---------------------------------------------------------------------------
def test_guided_schedule_parity(ctx):
    sc = scenegen.make_heightfield_scene(seed=2, width=40, height=33, grid=24, n_boxes=12)
    g, o = _pair(ctx, sc, mode=orc.MODE_PT_GUIDED, max_depth=6)
    for it in range(5):
        say("guided iteration", it)
        alloc = orc.ALLOC_CLASSIC if it < 2 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=2, alloc=alloc, debug_depth=6)
        g.render_iteration(pg)
        o.render_iteration(po)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        g.update(pg)
        o.update(po)
        _cmp_cells(g, o)
        pmg, cdg = g.hist()
        pmo, cdo = o.hist()
        assert np.allclose(pmg, pmo, rtol=1e-6) and np.allclose(cdg, cdo, rtol=1e-6)
        assert np.array_equal(g.nodes(), o.nodes())


# ---------------------------------------------------------------------------
# EARS allocation (one shared count per vertex): the same schedule parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["pt", "guided", "bdpt"])
def test_ears_schedule_parity(ctx, mode):
    extra = {}
    if mode == "pt":
        sc, kw, warm = scenegen.make_cornell(48, 40), dict(max_depth=5), 1
    elif mode == "guided":
        sc = scenegen.make_heightfield_scene(seed=2, width=40, height=33, grid=24, n_boxes=12)
        kw, warm = dict(mode=orc.MODE_PT_GUIDED, max_depth=6), 2
    else:
        sc, kw, warm = scenegen.make_cornell(40, 36), dict(mode=orc.MODE_BDPT, max_depth=5), 2
        extra = dict(stat_clamp=0.0)
    g, o = _pair(ctx, sc, **kw)
    for it in range(5):
        say("EARS", mode, "iteration", it)
        alloc = orc.ALLOC_CLASSIC if it < warm else orc.ALLOC_EARS
        pg, po = _params(iteration=it, spp=2, alloc=alloc, debug_depth=kw["max_depth"], **extra)
        g.render_iteration(pg)
        o.render_iteration(po)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        dg, do = g.debug_vertices(), o.debug_vertices()
        _cmp_vertices(dg, do)
        if alloc == orc.ALLOC_EARS:
            # one shared factor: BSDF and guided counts at half the NEE count
            # (guided), the BSDF count equal to it (plain PT)
            # (below the classic RR depth, where a cell without data falls
            # back to counts of the same shape)
            b = do["beta"]
            half = np.float32(0.5) if mode == "guided" else np.float32(1.0)
            on = (b[:, 1] > 0) & (do["depth"] < 5)
            assert on.any() and np.array_equal(b[on, 0], half * b[on, 1])
            if mode == "bdpt":
                assert np.array_equal(b[on, 2], b[on, 1])
        g.update(pg)
        o.update(po)
        _cmp_cells(g, o)
        assert np.array_equal(g.nodes(), o.nodes())
    np.testing.assert_allclose(g.image(1), o.image(1), rtol=1e-5, atol=1e-7)


# ---------------------------------------------------------------------------
# update kernel and refinement on identical inputs: bit-identical
# ---------------------------------------------------------------------------
def test_fixed_point_update_bitexact(ctx):
    sc = scenegen.make_cornell(16, 16)
    g, o = _pair(ctx, sc, max_depth=3)
    for it in range(3):  # grow the octree identically
        pg, po = _params(iteration=it, spp=8)
        g.render_iteration(pg); o.render_iteration(po)
        g.update(pg); o.update(po)
    n = g.ncells
    assert n == o.ncells and n > 8
    rng = np.random.default_rng(5)
    acc = np.zeros((n, 3, 8))
    acc[:, :, 6] = rng.integers(0, 50, (n, 3))
    acc[:, :, 7] = acc[:, :, 6] * rng.uniform(1, 9, (n, 3))
    m = rng.lognormal(0, 2, (n, 3, 3))
    acc[:, :, 0:3] = m * acc[:, :, 6:7]
    acc[:, :, 3:6] = (m * m + rng.lognormal(0, 2, (n, 3, 3))) * acc[:, :, 6:7]
    fac = rng.uniform(0, 3, (n, 2, 3, 3)).astype(np.float32)
    for x in (g, o):
        x.write_cells(factors=fac, acc=acc)
        x.update_cells_only(0.37, 11.5)
    fa, fb = g.cells()["factors"], o.cells()["factors"]
    assert np.array_equal(fa.view(np.uint32), fb.view(np.uint32))


def test_refinement_identical(ctx):
    sc = scenegen.make_cornell(16, 16)
    g, o = _pair(ctx, sc, max_depth=3, max_cells=3000)
    rng = np.random.default_rng(8)
    for r in range(5):
        n = g.ncells
        vis = rng.integers(0, 80, n).astype(np.uint32)
        for x in (g, o):
            x.write_cells(visits=vis)
        a, b = g.refine_only(), o.refine_only()
        assert a == b
        assert np.array_equal(g.nodes(), o.nodes())
        assert np.array_equal(g.cells()["depth"], o.cells()["depth"])


# ---------------------------------------------------------------------------
# closed forms on the GPU alone
# ---------------------------------------------------------------------------
def test_furnace_gpu(ctx):
    api = _api()
    sc = scenegen.make_furnace(64, 64)
    g = api.Scene(ctx, sc, max_depth=5)
    L = []
    for it in range(8):
        say("furnace iteration", it)
        p = api.iter_params(iteration=it, spp=8, alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        g.render_iteration(p)
        if it:
            L.append(g.sample_radiance()[:, 1].copy())
        g.update(p)
    L = np.concatenate(L)
    z = (L.mean() - 1.9375) / (L.std() / math.sqrt(len(L)))
    assert abs(z) < 4.0, (L.mean(), z)


def test_unbiased_fixed_counts_gpu(ctx):
    api = _api()
    sc = scenegen.make_cornell(48, 48)
    ref = api.Scene(ctx, sc, max_depth=3)
    ref.set_fixed_counts(np.array([[1.0, 1.0, 0.0]]))
    g = api.Scene(ctx, sc, max_depth=3)
    for it in range(2):
        p = api.iter_params(iteration=100 + it, spp=4)
        g.render_iteration(p)
        g.update(p)
    rng = np.random.default_rng(3)
    n = g.ncells
    g.set_fixed_counts(np.stack([rng.uniform(0.05, 3, n), rng.uniform(0.05, 20, n), np.zeros(n)], 1))
    ma, mb = [], []
    for it in range(16):
        say("unbiased iteration", it)
        ref.render_iteration(api.iter_params(iteration=it, spp=16, alloc=api.ALLOC_FIXED))
        ma.append(ref.sample_radiance().mean(0))
        g.render_iteration(api.iter_params(iteration=500 + it, spp=16, alloc=api.ALLOC_FIXED,
                                           fixed_scale=bool(it % 2)))
        mb.append(g.sample_radiance().mean(0))
    a, b = np.array(ma), np.array(mb)
    z = (a.mean(0) - b.mean(0)) / np.sqrt(a.var(0) / len(a) + b.var(0) / len(b))
    assert np.all(np.abs(z) < 4.0), z


# ---------------------------------------------------------------------------
# host-forced failure handling and state
# ---------------------------------------------------------------------------
def test_overflow_rerun_gives_identical_results(ctx):
    api = _api()
    sc = scenegen.make_cornell(32, 32)
    a = api.Scene(ctx, sc, max_depth=5)
    b = api.Scene(ctx, sc, max_depth=5, queue_capacity=700, tile_roots=512)
    retries = 0
    for it in range(3):
        say("overflow iteration", it)
        p = api.iter_params(iteration=it, spp=2, alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        a.render_iteration(p)
        sb = b.render_iteration(p)
        retries += sb.overflow_retries
        assert np.array_equal(a.sample_radiance().view(np.uint32), b.sample_radiance().view(np.uint32))
        a.update(p)
        b.update(p)
        assert np.array_equal(a.nodes(), b.nodes())
    # the halving happened, and later iterations start from the tile that fitted
    assert retries > 0 and b.query()[1] < 512


def test_shadow_queue_overflow_rerun_gives_identical_results(ctx):
    """Ray queues roomy, shadow queues (NEE samples and connections) small:
    the shadow queues overflow, the tile halves and the bidirectional
    results equal those of roomy queues bit for bit."""
    api = _api()
    sc = scenegen.make_interior(seed=3, n_pieces=12, tess=1, width=32, height=24)
    a = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=6)
    b = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=6)
    b.configure(queue_capacity=1 << 16, tile_roots=768, shadow_capacity=2048)
    assert b.query_queues()[:2] == (1 << 16, 2048)
    retries = 0
    for it in range(3):
        say("shadow overflow iteration", it)
        p = api.iter_params(iteration=it, spp=2, stat_clamp=0.0,
                            alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        sa = a.render_iteration(p)
        sb = b.render_iteration(p)
        retries += sb.overflow_retries
        assert sa.total_rays() == sb.total_rays()
        assert np.array_equal(a.sample_radiance().view(np.uint32), b.sample_radiance().view(np.uint32))
        a.update(p)
        b.update(p)
        assert np.array_equal(a.nodes(), b.nodes())
    assert retries > 0 and b.query()[1] < 768
    # the peaks per camera sample of the two queues
    _, _, pr, ps = b.query_queues()
    assert ps > pr > 0.0


def test_single_tree_overflow_is_reported(ctx):
    api = _api()
    sc = scenegen.make_cornell(8, 8)
    s = api.Scene(ctx, sc, max_depth=5, queue_capacity=8, tile_roots=4)
    s.set_fixed_counts(np.array([[3.0, 20.0, 0.0]]))
    with pytest.raises(api.MarsError) as e:
        s.render_iteration(api.iter_params(spp=1, alloc=api.ALLOC_FIXED))
    assert e.value.code == -5


def test_checkpoint_resume_identical(ctx, tmp_path):
    api = _api()
    sc = scenegen.make_cornell(32, 32)
    a = api.Scene(ctx, sc, max_depth=4)
    b = api.Scene(ctx, sc, max_depth=4)
    for it in range(3):
        p = api.iter_params(iteration=it, spp=1, alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        a.render_iteration(p)
        a.update(p)
    path = tmp_path / "ck.bin"
    a.checkpoint_save(path)
    b.checkpoint_load(path)
    p = api.iter_params(iteration=3, spp=1, alloc=api.ALLOC_MARS)
    a.render_iteration(p)
    b.render_iteration(p)
    assert np.array_equal(a.sample_radiance().view(np.uint32), b.sample_radiance().view(np.uint32))
    a.update(p)
    b.update(p)
    assert np.array_equal(a.nodes(), b.nodes())
    assert np.array_equal(a.image(0), b.image(0))


def test_determinism_two_runs(ctx):
    api = _api()
    sc = scenegen.make_heightfield_scene(seed=4, width=32, height=32, grid=20, n_boxes=8)
    outs = []
    for rep in range(2):
        s = api.Scene(ctx, sc, mode=api.MODE_PT_GUIDED, max_depth=6)
        api.run_schedule(s, 4, warmup=1, spp=2)
        outs.append((s.nodes(), s.cells()["visits"], s.image(0)))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)


def test_argument_errors(ctx):
    api = _api()
    sc = scenegen.make_cornell(8, 8)
    bad = dict(sc)
    bad["V"] = sc["V"].copy()
    bad["V"][0, 0] = np.nan
    with pytest.raises(api.MarsError) as e:
        api.Scene(ctx, bad)
    assert e.value.code == -6
    s = api.Scene(ctx, sc, max_depth=3)
    with pytest.raises(api.MarsError):
        s.render_iteration(api.iter_params(spp=0))
    with pytest.raises(api.MarsError):
        s.render_iteration(api.iter_params(alloc=api.ALLOC_FIXED))
    with pytest.raises(api.MarsError):
        s.update()


# ---------------------------------------------------------------------------
# edge cases: ragged image, no emitter, single triangle, depth 1
# ---------------------------------------------------------------------------
def test_edge_cases(ctx):
    api = _api()
    # ragged sizes
    sc = scenegen.make_cornell(33, 17)
    g, o = _pair(ctx, sc, max_depth=3)
    pg, po = _params(spp=3, debug_depth=3)
    g.render_iteration(pg); o.render_iteration(po)
    _cmp_radiance(g.sample_radiance(), o.sample_radiance())
    # no emitter: black image, NEE has nothing to sample
    dark = dict(scenegen.make_cornell(16, 16))
    dark["mats"] = dark["mats"].copy()
    dark["mats"][:, 5:8] = 0
    s = api.Scene(ctx, dark, max_depth=4)
    s.render_iteration(api.iter_params(spp=2))
    assert np.all(s.sample_radiance() == 0)
    # single triangle (the BVH is one leaf)
    # winding normal (v1-v0)x(v2-v0) points at the camera, so the emitter is seen
    tri = {"V": np.array([[-1, -1, 2, 0, 1, 2, 1, -1, 2]], np.float32),
           "tri_mat": np.array([0], np.uint32),
           "mats": np.array([[0, .5, .5, .5, 0, 2, 2, 2]], np.float32),
           "camera": np.array([0, 0, 0, 0, 0, 1, 0, 1, 0, 60], np.float32),
           "width": 9, "height": 7}
    g, o = _pair(ctx, tri, max_depth=2)
    pg, po = _params(spp=2)
    g.render_iteration(pg); o.render_iteration(po)
    _cmp_radiance(g.sample_radiance(), o.sample_radiance())
    assert g.sample_radiance().max() > 0
    # depth 1: emission only
    g, o = _pair(ctx, scenegen.make_cornell(16, 16), max_depth=1)
    g.render_iteration(pg); o.render_iteration(po)
    _cmp_radiance(g.sample_radiance(), o.sample_radiance())


# ---------------------------------------------------------------------------
# full size (512 x 512 guided heightfield, ~132k triangles, max depth 10) in
# the launch configuration of the benchmark: sampled pixels against the
# oracle, for a classic iteration and for MARS counts from seeded factors
# ---------------------------------------------------------------------------
def test_full_size_sampled_pixels(ctx):
    api = _api()
    sc = scenegen.make_heightfield_scene(seed=1)
    say("full size upload", sc["V"].shape[0], "tris")
    g = api.Scene(ctx, sc, mode=api.MODE_PT_GUIDED, max_depth=10)
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=10)
    rng = np.random.default_rng(17)
    pix = rng.choice(sc["width"] * sc["height"], 400, replace=False)
    o.set_pixel_subset(pix)
    roots = pix  # spp = 1
    pg, po = _params(iteration=0, spp=1, debug_depth=3)
    say("full size classic iteration")
    g.render_iteration(pg)
    o.render_iteration(po)
    _cmp_radiance(g.sample_radiance()[roots], o.sample_radiance()[roots])
    dg = g.debug_vertices()
    dg = dg[np.isin(dg["root"], roots)]
    _cmp_vertices(dg, o.debug_vertices())
    # MARS counts: seeded pixel estimates, factors and a directional
    # distribution written identically into both (root cell only)
    it = rng.uniform(0.05, 2.0, (sc["height"], sc["width"], 3)).astype(np.float32)
    fac = rng.uniform(0.0, 4.0, (1, 2, 3, 3)).astype(np.float32)
    w = rng.random(64) ** 2
    pm = (0.9 * w / w.sum() + 0.1 / 64).astype(np.float32)[None]
    cdf = np.cumsum(pm.astype(np.float64), 1).astype(np.float32)
    cdf[:, -1] = 1
    for x in (g, o):
        x.set_itilde(it)
        x.write_cells(factors=fac)
        x.set_hist(pm, cdf)
    pg, po = _params(iteration=1, spp=1, alloc=api.ALLOC_MARS, debug_depth=3)
    say("full size MARS iteration")
    g.render_iteration(pg)
    o.render_iteration(po)
    _cmp_radiance(g.sample_radiance()[roots], o.sample_radiance()[roots])
    dg = g.debug_vertices()
    dg = dg[np.isin(dg["root"], roots)]
    _cmp_vertices(dg, o.debug_vertices())


# ---------------------------------------------------------------------------
# bidirectional mode (Sec. 5): light subpaths, NEE, light-path connections
# with the full-path budget-aware balance heuristic
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scene", ["cornell", "interior"])
def test_bdpt_schedule_parity(ctx, scene):
    if scene == "cornell":
        sc, D = scenegen.make_cornell(40, 36), 5
    else:
        sc, D = scenegen.make_interior(seed=2, n_pieces=40, tess=2, width=48, height=27), 6
    g, o = _pair(ctx, sc, mode=orc.MODE_BDPT, max_depth=D)
    for it in range(5):
        say("bdpt", scene, "iteration", it)
        alloc = orc.ALLOC_CLASSIC if it < 2 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=2, alloc=alloc, stat_clamp=0.0, debug_depth=D)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        assert (sg.rays_light, sg.rays_conn, sg.rays_shadow, sg.rays_ext) == \
               (so.rays_light, so.rays_conn, so.rays_shadow, so.rays_ext)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        _cmp_cells(g, o)
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-9 * max(uo.V_I, 1e-30)
        assert ug.n_excluded == uo.n_excluded
        assert np.array_equal(g.nodes(), o.nodes())
        _cmp_cells(g, o)


def test_bdpt_furnace_gpu(ctx):
    api = _api()
    sc = scenegen.make_furnace(48, 48)
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=5)
    L = []
    for it in range(6):
        p = api.iter_params(iteration=it, spp=4, stat_clamp=0.0,
                            alloc=api.ALLOC_CLASSIC if it < 2 else api.ALLOC_MARS)
        g.render_iteration(p)
        L.append(g.sample_radiance()[:, 0].copy())
        g.update(p)
    L = np.concatenate(L)
    z = (L.mean() - 1.9375) / (L.std() / math.sqrt(len(L)))
    assert abs(z) < 4.0, (L.mean(), z)


def test_bdpt_full_size_sampled_pixels(ctx):
    """1280 x 720 interior, ~1M triangles, max path length 12: sampled
    pixels of a classic iteration and of a MARS iteration with seeded
    factors, against the oracle (which traces every light subpath)."""
    api = _api()
    sc = scenegen.make_interior(seed=1)
    say("bdpt full size upload", sc["V"].shape[0], "tris")
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12)
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=12)
    rng = np.random.default_rng(23)
    pix = rng.choice(sc["width"] * sc["height"], 200, replace=False)
    o.set_pixel_subset(pix)
    for it, alloc in ((0, orc.ALLOC_CLASSIC), (1, orc.ALLOC_MARS)):
        if alloc == orc.ALLOC_MARS:
            itl = rng.uniform(0.05, 2.0, (sc["height"], sc["width"], 3)).astype(np.float32)
            fac = rng.uniform(0.0, 3.0, (1, 2, 3, 3)).astype(np.float32)
            for x in (g, o):
                x.set_itilde(itl)
                x.write_cells(factors=fac)
        pg, po = _params(iteration=it, spp=1, alloc=alloc, stat_clamp=0.0, debug_depth=3)
        say("bdpt full size iteration", it)
        g.render_iteration(pg)
        o.render_iteration(po)
        _cmp_radiance(g.sample_radiance()[pix], o.sample_radiance()[pix])
        dg = g.debug_vertices()
        dg = dg[np.isin(dg["root"], pix)]
        _cmp_vertices(dg, o.debug_vertices())


# ---------------------------------------------------------------------------
# independent rounding of each count (the scheme Alg. 1 replaces): the same
# decisions and radiance as the oracle over MARS schedules
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [orc.MODE_PT, orc.MODE_PT_GUIDED, orc.MODE_BDPT])
def test_independent_rounding_schedule_parity(ctx, mode):
    sc = scenegen.make_cornell(40, 36)
    g, o = _pair(ctx, sc, mode=mode, max_depth=4)
    kc = 0.0 if mode == orc.MODE_BDPT else 50.0
    for it in range(4):
        say("independent rounding, mode", mode, "iteration", it)
        alloc = orc.ALLOC_CLASSIC if it < 1 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=2, alloc=alloc, stat_clamp=kc, debug_depth=4,
                         rounding=1)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        assert sg.total_rays() == so.total_rays()
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        _cmp_vertices(g.debug_vertices(), o.debug_vertices())
        g.update(pg)
        o.update(po)
        assert np.array_equal(g.nodes(), o.nodes())
