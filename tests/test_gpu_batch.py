"""Batched iterations (one captured launch graph over many scenes) and the
queue / tile autotuner, through the C ABI.

Every batched scene has an eager twin rendered with the per-scene calls and
a CPU oracle twin.  Bars: the batch equals the eager path bit for bit
(sample radiance, images, count maps, octree, visit counts, factors, update
statistics), after every replay of the graph with eager work and
synchronisation in between; against the oracle, per-sample radiance within
1e-4 relative and identical octrees."""
import numpy as np
import pytest

import scenegen
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

MODES = {"guided": orc.MODE_PT_GUIDED, "bdpt": orc.MODE_BDPT, "pt": orc.MODE_PT}


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


def _small_batch(seed=3, n=4):
    b = scenegen.make_batch(seed=seed, n=n, tris_lo=200, tris_hi=3000, res=(16, 24, 33),
                            depth_lo=4, depth_hi=7)
    c = scenegen.make_cornell(20, 18)
    c["mode"], c["max_depth"] = "pt", 5
    return b + [c]


def _twins(ctx, scenes, with_oracle=True, **kw):
    api = _api()
    G, E, O = [], [], []
    for sc in scenes:
        m, D = MODES[sc["mode"]], sc["max_depth"]
        G.append(api.Scene(ctx, sc, mode=m, max_depth=D, **kw))
        E.append(api.Scene(ctx, sc, mode=m, max_depth=D, **kw))
        if with_oracle:
            O.append(orc.Oracle(sc, mode=m, max_depth=D))
    return G, E, O


def _params(it, warm=2, alloc=None):
    api = _api()
    alloc = orc.ALLOC_MARS if alloc is None else alloc
    kw = dict(iteration=it, spp=2, alloc=orc.ALLOC_CLASSIC if it < warm else alloc,
              stat_clamp=0.0, clamp_hi=8.0)
    return api.iter_params(**kw), orc.Oracle.params(**kw)


def _same(a, b, what):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.dtype.kind == "f":
        ok = np.array_equal(a.view(np.uint32 if a.itemsize == 4 else np.uint64),
                            b.view(np.uint32 if b.itemsize == 4 else np.uint64))
    else:
        ok = np.array_equal(a, b)
    assert ok, (what, np.abs(a.astype(np.float64) - b.astype(np.float64)).max())


def _cmp_twins(g, e, updated=True):
    api = _api()
    _same(g.sample_radiance(), e.sample_radiance(), "radiance")
    _same(g.image(api.IMAGE_LAST), e.image(api.IMAGE_LAST), "last image")
    _same(g.count_map(), e.count_map(), "count map")
    if updated:
        _same(g.image(api.IMAGE_MEAN), e.image(api.IMAGE_MEAN), "mean image")
        _same(g.image(api.IMAGE_IVW), e.image(api.IMAGE_IVW), "ivw image")
        assert g.ncells == e.ncells
        _same(g.nodes(), e.nodes(), "nodes")
        cg, ce = g.cells(), e.cells()
        _same(cg["factors"], ce["factors"], "factors")
        _same(cg["visits"], ce["visits"], "visits")


def _cmp_oracle(g, o):
    a, b = g.sample_radiance(), o.sample_radiance()
    err = np.abs(a - b) / np.maximum(np.abs(b), 1e-3)
    assert err.max() <= 1e-4, err.max()
    assert np.array_equal(g.nodes(), o.nodes())


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_eager_and_oracle(ctx, graph):
    api = _api()
    scenes = _small_batch()
    G, E, O = _twins(ctx, scenes)
    for it in range(5):
        say("batch iteration", it, "graph", graph)
        pg, po = _params(it)
        its, ups = api.iterate_batch(G, pg, update=True, graph=graph)
        for k, (g, e, o) in enumerate(zip(G, E, O)):
            se = e.render_iteration(pg)
            ue = e.update(pg)
            o.render_iteration(po)
            o.update(po)
            si = its[k]
            assert (si.rays_ext, si.rays_shadow, si.rays_light, si.rays_conn, si.vertices,
                    si.samples) == (se.rays_ext, se.rays_shadow, se.rays_light, se.rays_conn,
                                    se.vertices, se.samples), k
            u = ups[k]
            assert (u.V_I, u.C_I, u.n_cells_before, u.n_cells_after, u.n_excluded) == \
                   (ue.V_I, ue.C_I, ue.n_cells_before, ue.n_cells_after, ue.n_excluded), k
            _cmp_twins(g, e)
            _cmp_oracle(g, o)


def test_batch_ears_equals_eager_and_oracle(ctx):
    # the EARS count rule through the captured batch (its update writes the
    # shared factors, signalled by the iteration's allocation mode)
    api = _api()
    scenes = _small_batch(seed=5)
    G, E, O = _twins(ctx, scenes)
    for it in range(4):
        say("batch EARS iteration", it)
        pg, po = _params(it, alloc=orc.ALLOC_EARS)
        api.iterate_batch(G, pg, update=True, graph=True)
        for g, e, o in zip(G, E, O):
            e.render_iteration(pg)
            e.update(pg)
            o.render_iteration(po)
            o.update(po)
            _cmp_twins(g, e)
            _cmp_oracle(g, o)


def test_render_batch_totals(ctx):
    api = _api()
    scenes = _small_batch(seed=4)
    G, E, _ = _twins(ctx, scenes, with_oracle=False)
    for it in range(3):
        pg, _ = _params(it, warm=1)
        tot = api.render_batch(G, pg)
        ref = [e.render_iteration(pg) for e in E]
        assert tot.rays_ext == sum(r.rays_ext for r in ref)
        assert tot.rays_shadow == sum(r.rays_shadow for r in ref)
        assert tot.rays_light == sum(r.rays_light for r in ref)
        assert tot.samples == sum(r.samples for r in ref)
        for g, e in zip(G, E):
            _cmp_twins(g, e, updated=False)
            g.update(pg)
            e.update(pg)
            _cmp_twins(g, e)


def test_batch_overflow_reruns_scene(ctx):
    """A scene whose queues overflow inside the graph skips its update there
    and is rendered again with tile halving: the result still equals the
    eager twin (which halves its tiles the same way)."""
    api = _api()
    # first: a BDPT interior, whose shadow queues hold a connection per light
    # vertex, on queues of 1024 entries per level
    first = scenegen.make_interior(seed=2, n_pieces=10, tess=1, width=24, height=24)
    first["mode"], first["max_depth"] = "bdpt", 6
    scenes = [first] + _small_batch(seed=5, n=2)
    G, E, O = _twins(ctx, scenes)
    for x in (G[0], E[0]):
        x.configure(queue_capacity=1024, tile_roots=1024)
    for it in range(4):
        say("overflow iteration", it)
        pg, po = _params(it, warm=1)
        its, _ = api.iterate_batch(G, pg, update=True)
        for k, (g, e, o) in enumerate(zip(G, E, O)):
            se = e.render_iteration(pg)
            e.update(pg)
            o.render_iteration(po)
            o.update(po)
            _cmp_twins(g, e)
            _cmp_oracle(g, o)
            if k == 0 and it == 0:
                assert se.overflow_retries > 0, "the small queue never overflowed"
                assert its[0].overflow_retries > 0
    # the eager path starts later iterations from the tile that fitted; the
    # batch keeps the configured tile and re-runs a scene when it overflows
    assert G[0].query()[1] == 1024 and E[0].query()[1] < 1024


def test_batch_full_size_equals_eager(ctx):
    """A batch at full configuration sizes (the 512x512 guided heightfield
    of 132k triangles, depth 10, and the 1280x720 bidirectional interior of
    1.04M triangles, depth 12) equals its per-scene twins bit for bit over a
    classic and two MARS iterations, through the captured graphs."""
    api = _api()
    hf = scenegen.make_heightfield_scene(seed=1)
    hf["mode"], hf["max_depth"] = "guided", 10
    it_ = scenegen.make_interior(seed=1)
    it_["mode"], it_["max_depth"] = "bdpt", 12
    G, E, _ = _twins(ctx, [hf, it_], with_oracle=False)
    for x in (G[1], E[1]):
        x.configure(queue_capacity=4 << 20, tile_roots=230400, shadow_capacity=64 << 20)
    for it in range(3):
        say("full-size batch iteration", it)
        p = api.iter_params(iteration=it, spp=1, stat_clamp=0.0,
                            alloc=api.ALLOC_CLASSIC if it == 0 else api.ALLOC_MARS)
        its, _ = api.iterate_batch(G, p, update=True)
        for k, (g, e) in enumerate(zip(G, E)):
            se = e.render_iteration(p)
            e.update(p)
            assert its[k].total_rays() == se.total_rays(), k
            _cmp_twins(g, e)
    for s_ in G + E:
        s_.release()


def _cap(tile, e):
    """Queue capacity the autotuner derives from a tile and the measured peak."""
    c = int(np.ceil(tile * max(1.0, e) * 1.5))
    return min(max((c + 4095) // 4096 * 4096, 4096), 0xFFFF0000)


def _floor(roots, e):
    """Smallest tile the autotuner plans: ~2^18 queue entries at the peak."""
    t = int(np.ceil(262144.0 / max(1.0, e)))
    return min(roots, (max(t, 4096) + 63) // 64 * 64)


def _qbytes(scene, cap, scap):
    # per level: 168 B per ray-queue entry (BDPT adds the 32 B camera-vertex
    # record), 16 B per shadow value; the 32 B shadow rays hold one level
    per = 168 + (32 if scene.mode == orc.MODE_BDPT else 0)
    return (scene.max_depth + 2) * (cap * per + scap * 16) + scap * 32


def test_autotune_and_cache(ctx, tmp_path):
    api = _api()
    scenes = _small_batch(seed=6, n=4)
    big = scenegen.make_cornell(512, 512)
    big["mode"], big["max_depth"] = "pt", 5
    scenes.append(big)
    G, E, _ = _twins(ctx, scenes, with_oracle=False)
    p0, _ = _params(0)
    roots = [g.W * g.H * p0.spp for g in G]
    cache = str(tmp_path / "tune.txt")
    say("autotune, roomy budget")
    res = api.autotune(G, p0, mem_budget=4 << 30, cache_path=cache)
    lines = [ln for ln in open(cache).read().split("\n") if ln.strip()]
    assert len(lines) == len(G)
    for g, r, (cap, tile, e, scap, es) in zip(G, roots, res):
        assert g.query()[:2] == (cap, tile)
        assert g.query_queues()[:2] == (cap, scap)
        assert e >= 1.0 and es >= 1.0 and _floor(r, max(e, es)) <= tile <= r
        assert cap == _cap(tile, e) and scap == _cap(tile, es)
    # a budget that only fits the large scene at its smallest tile
    pk = [(e, es) for _, _, e, _, es in res]
    fl = _floor(roots[-1], max(pk[-1]))
    assert fl < roots[-1]
    need = _qbytes(G[-1], _cap(fl, pk[-1][0]), _cap(fl, pk[-1][1])) + sum(
        _qbytes(g, _cap(r, e), _cap(r, es)) for g, r, (e, es) in zip(G[:-1], roots[:-1], pk[:-1]))
    # probe again at whole-iteration tiles so the measured peaks repeat
    for g, r, (e, es) in zip(G, roots, pk):
        g.configure(queue_capacity=_cap(r, e), tile_roots=r, shadow_capacity=_cap(r, es))
    say("autotune, tight budget", need)
    res_t = api.autotune(G, p0, mem_budget=need + (1 << 20))
    assert res_t[-1][1] == fl
    assert sum(_qbytes(g, c, sc_) for g, (c, _, _, sc_, _) in zip(G, res_t)) <= need + (1 << 20)
    with pytest.raises(api.MarsError) as err:
        api.autotune(G, p0, mem_budget=1 << 20)
    assert err.value.code == -2
    # cached classes are applied without probing
    res2 = api.autotune(E, p0, mem_budget=4 << 30, cache_path=cache)
    assert [(c, t, sc_) for c, t, _, sc_, _ in res2] == [(c, t, sc_) for c, t, _, sc_, _ in res]
    for g, (c, t, _, sc_, _) in zip(G, res):
        g.configure(queue_capacity=c, tile_roots=t, shadow_capacity=sc_)
    # tuned batches still equal their eager twins
    for it in range(1, 4):
        say("tuned batch iteration", it)
        pg, _ = _params(it)
        api.iterate_batch(G, pg, update=True)
        for e in E:
            e.render_iteration(pg)
            e.update(pg)
    for g, e in zip(G, E):
        _cmp_twins(g, e)


def test_batch_argument_errors(ctx):
    api = _api()
    sc = scenegen.make_cornell(8, 8)
    a = api.Scene(ctx, sc, max_depth=3)
    b = api.Scene(ctx, sc, max_depth=3, mlp=True)
    p = api.iter_params(spp=1)
    with pytest.raises(api.MarsError) as e:
        api.iterate_batch([a, a], p)
    assert e.value.code == -1
    with pytest.raises(api.MarsError) as e:
        api.iterate_batch([a, b], p)
    assert e.value.code == -1
    with pytest.raises(api.MarsError) as e:
        api.iterate_batch([a], api.iter_params(spp=1, debug_depth=2))
    assert e.value.code == -1
    with pytest.raises(api.MarsError):
        a.configure(queue_capacity=1024, tile_roots=4096)
    # a batch with the learned-cache scene still renders through render_batch
    api.render_batch([a, b], p)
