"""Separate light-path budgets per light-vertex index (y_1, y_2, y_3+) in the
bidirectional HIP path, through the C ABI, against the oracle: a schedule of
classic and MARS iterations with every vertex's five counts, rounded counts
and radiance, the cells and the per-class cells after every update; random
written class factors; the argument checks; checkpoint resume and batched
iterations (graph and stream pool) against per-scene calls, bit for bit but
for the order of binary64 atomic sums.
Bars as in test_gpu_parity.py."""
import numpy as np
import pytest

import scenegen
from oracle import oracle as orc
from test_gpu_parity import _cmp_cells, _cmp_radiance, _cmp_vertices, _params, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_20429_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _pair(ctx, sc, depth, **kw):
    from paper_2410_20429_amd import api
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=depth, lp_lengths=True, **kw)
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=depth, lp_classes=3, **kw)
    return g, o


def _cmp_cells_x(g, o):
    cg, co = g.cells_x(), o.cells_x()
    assert np.allclose(cg["acc"], co["acc"], rtol=1e-9, atol=1e-12)
    fa, fb = cg["factors"], co["factors"]
    assert np.sum(fa.view(np.uint32) != fb.view(np.uint32)) <= 2
    assert np.allclose(fa, fb, rtol=1e-6, atol=0)


def _cmp_vertices_x(dg, do):
    kg = np.sort(dg, order=["root", "depth", "stream_lo", "stream_hi"])
    ko = np.sort(do, order=["root", "depth", "stream_lo", "stream_hi"])
    assert np.array_equal(kg["gamma_x"], ko["gamma_x"])
    assert np.array_equal(kg["beta_x"].view(np.uint32), ko["beta_x"].view(np.uint32))


@pytest.mark.parametrize("scene", ["cornell", "interior"])
@pytest.mark.parametrize("aware", [True, False])
def test_lp_lengths_schedule_parity(ctx, scene, aware):
    if scene == "cornell":
        sc, D = scenegen.make_cornell(40, 36), 5
    else:
        sc, D = scenegen.make_interior(seed=2, n_pieces=40, tess=2, width=48, height=27), 7
    g, o = _pair(ctx, sc, D)
    classes_used = False
    for it in range(6):
        say("per-length light paths", scene, "aware", aware, "iteration", it)
        alloc = orc.ALLOC_CLASSIC if it < 2 else orc.ALLOC_MARS
        pg, po = _params(iteration=it, spp=2, alloc=alloc, stat_clamp=0.0, debug_depth=D,
                         budget_aware=aware)
        sg = g.render_iteration(pg)
        so = o.render_iteration(po)
        assert (sg.rays_light, sg.rays_conn, sg.rays_shadow, sg.rays_ext, sg.samples) == \
               (so.rays_light, so.rays_conn, so.rays_shadow, so.rays_ext, so.samples)
        _cmp_radiance(g.sample_radiance(), o.sample_radiance())
        dg, do = g.debug_vertices(), o.debug_vertices()
        _cmp_vertices(dg, do)
        _cmp_vertices_x(dg, do)
        classes_used |= bool(np.any(dg["gamma_x"] != dg["gamma"][:, 2:3]))
        _cmp_cells(g, o)
        _cmp_cells_x(g, o)
        np.testing.assert_allclose(g.count_map(), o.count_map(), rtol=1e-6, atol=0)
        ug, uo = g.update(pg), o.update(po)
        assert abs(ug.V_I - uo.V_I) <= 1e-9 * max(uo.V_I, 1e-30)
        assert np.array_equal(g.nodes(), o.nodes())
        _cmp_cells(g, o)
        _cmp_cells_x(g, o)
    assert classes_used   # the three classes drew different counts somewhere
    g.release()


def test_lp_lengths_written_factors_parity(ctx):
    """Random class factors written into both sides (counts far from the
    fixed point's): one MARS iteration, every decision and the radiance."""
    sc = scenegen.make_cornell(24, 20)
    g, o = _pair(ctx, sc, 6)
    for it in range(2):
        pg, po = _params(iteration=it, spp=4, stat_clamp=0.0)
        g.render_iteration(pg)
        o.render_iteration(po)
        g.update(pg)
        o.update(po)
    rng = np.random.default_rng(13)
    n = g.ncells
    f = np.exp(rng.uniform(-4.0, 2.0, (n, 2, 3, 3))).astype(np.float32)
    fx = np.exp(rng.uniform(-4.0, 2.0, (n, 2, 2, 3))).astype(np.float32)
    for s in (g, o):
        s.write_cells(factors=f)
        s.write_cells_x(factors=fx)
    pg, po = _params(iteration=9, spp=4, alloc=orc.ALLOC_MARS, stat_clamp=0.0, debug_depth=6)
    sg = g.render_iteration(pg)
    so = o.render_iteration(po)
    assert sg.total_rays() == so.total_rays()
    _cmp_radiance(g.sample_radiance(), o.sample_radiance())
    dg, do = g.debug_vertices(), o.debug_vertices()
    _cmp_vertices(dg, do)
    _cmp_vertices_x(dg, do)
    assert np.any(dg["gamma_x"][:, 1] > 1)   # y_3+ connections split
    _cmp_cells(g, o)
    _cmp_cells_x(g, o)
    g.release()


def test_lp_lengths_argument_checks(ctx):
    from paper_2410_20429_amd import api
    sc = scenegen.make_cornell(8, 8)
    with pytest.raises(api.MarsError):
        api.Scene(ctx, sc, mode=api.MODE_PT, max_depth=4, lp_lengths=True)
    with pytest.raises(api.MarsError):
        api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=4, lp_lengths=True, mlp=True)
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=4, lp_lengths=True)
    with pytest.raises(api.MarsError):
        g.render_iteration(api.iter_params(alloc=api.ALLOC_EARS))
    with pytest.raises(api.MarsError):
        g.render_iteration(api.iter_params(rounding=1))
    g.release()
    one = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=4)
    with pytest.raises(api.MarsError):
        one.cells_x()
    one.release()


def test_lp_lengths_checkpoint_resume_identical(ctx, tmp_path):
    """The class factors travel with the checkpoint: a resumed scene renders
    the next MARS iteration bit for bit like the uninterrupted one."""
    from paper_2410_20429_amd import api
    sc = scenegen.make_cornell(32, 32)
    a = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=5, lp_lengths=True)
    b = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=5, lp_lengths=True)
    for it in range(4):
        p = api.iter_params(iteration=it, spp=2, stat_clamp=0.0,
                            alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        a.render_iteration(p)
        a.update(p)
    assert np.any(a.cells_x()["factors"] >= 0)
    path = tmp_path / "ck_lp.bin"
    a.checkpoint_save(path)
    b.checkpoint_load(path)
    assert np.array_equal(a.cells_x()["factors"].view(np.uint32),
                          b.cells_x()["factors"].view(np.uint32))
    p = api.iter_params(iteration=4, spp=2, alloc=api.ALLOC_MARS, stat_clamp=0.0)
    a.render_iteration(p)
    b.render_iteration(p)
    assert np.array_equal(a.sample_radiance().view(np.uint32), b.sample_radiance().view(np.uint32))
    a.release()
    b.release()


@pytest.mark.parametrize("graph", [True, False])
def test_lp_lengths_batch_equals_eager(ctx, graph):
    """Per-length scenes in a batch (captured graphs or the stream pool)
    equal their per-scene twins bit for bit after every iteration."""
    from paper_2410_20429_amd import api
    scenes = [scenegen.make_cornell(20, 18), scenegen.make_interior(seed=4, n_pieces=30, tess=1,
                                                                    width=24, height=16)]
    G = [api.Scene(ctx, s, mode=api.MODE_BDPT, max_depth=6, lp_lengths=True) for s in scenes]
    E = [api.Scene(ctx, s, mode=api.MODE_BDPT, max_depth=6, lp_lengths=True) for s in scenes]
    for it in range(4):
        say("per-length batch iteration", it, "graph", graph)
        p = api.iter_params(iteration=it, spp=2, stat_clamp=0.0,
                            alloc=api.ALLOC_CLASSIC if it < 2 else api.ALLOC_MARS)
        api.iterate_batch(G, p, update=True, graph=graph)
        for g, e in zip(G, E):
            e.render_iteration(p)
            e.update(p)
            assert np.array_equal(g.sample_radiance().view(np.uint32),
                                  e.sample_radiance().view(np.uint32))
            assert np.array_equal(g.nodes(), e.nodes())
            xg, xe = g.cells_x(), e.cells_x()
            assert np.array_equal(xg["factors"].view(np.uint32), xe["factors"].view(np.uint32))
            # binary64 atomics add in either order
            assert np.allclose(xg["acc"], xe["acc"], rtol=1e-12, atol=0)
    for s in G + E:
        s.release()
