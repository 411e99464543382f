"""Learned cache, render side, on the GPU (through the C ABI) against
oracle/mlp_cache.py: the training targets and weights the update computes
from the cells, and the pooled counts learned-cache iterations draw with.
Every input is seeded and synthetic and is written into both sides."""
import numpy as np
import pytest

import scenegen
from oracle import mlp_cache as MC
from oracle import mlp_ref as M
from oracle import oracle as orc

pytestmark = pytest.mark.gpu
F = np.float32


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_20429_amd import api
    c = api.Context(0)
    yield c
    c.close()


def say(*a):
    print("[gpu-test]", *a, flush=True)


def _grow_same_octree(g, o, rng, rounds=3):
    """Identical octrees on both sides from written visit counts."""
    for _ in range(rounds):
        vis = rng.integers(0, 120, g.ncells).astype(np.uint32)
        g.write_cells(visits=vis)
        o.write_cells(visits=vis)
        g.refine_only()
        o.refine_only()
    assert g.ncells == o.ncells and np.array_equal(g.nodes(), o.nodes())


@pytest.mark.parametrize("mode", ["guided", "bdpt"])
def test_mlp_targets_parity(ctx, mode):
    from paper_2410_20429_amd import api
    say("mlp targets", mode)
    sc = scenegen.make_cornell(24, 20)    # ragged: 480 pixels
    m = api.MODE_PT_GUIDED if mode == "guided" else api.MODE_BDPT
    g = api.Scene(ctx, sc, mode=m, max_depth=3, max_cells=4000, mlp=True)
    o = orc.Oracle(sc, mode=m, max_depth=3, max_cells=4000)
    rng = np.random.default_rng(17)
    _grow_same_octree(g, o, rng)
    nc = g.ncells
    fac = rng.lognormal(-1.0, 1.5, (nc, 2, 3, 3)).astype(F)
    fac[:, 1] *= rng.uniform(0, 1, (nc, 3, 3)).astype(F)
    fac[rng.random(nc) < 0.1, 0, 1, 0] = -1.0          # no data for NEE in some cells
    acc = np.zeros((nc, 3, 8))
    acc[:, :, 6] = rng.integers(0, 90, (nc, 3))
    g.write_cells(factors=fac, acc=acc)
    o.write_cells(factors=fac, acc=acc)
    It = rng.uniform(0.005, 2.0, (sc["height"], sc["width"], 3)).astype(F)
    g.set_itilde(It)
    n = 6001
    P = rng.uniform(-0.05, 1.05, (n, 3)).astype(F)       # some outside the cube's clamp
    nrm = rng.normal(size=(n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(F)
    T = rng.lognormal(-1.0, 1.0, (n, 3)).astype(F)
    T[:50] = 0.0                                         # a dead path: no target
    pix = rng.integers(0, sc["width"] * sc["height"], n).astype(np.uint32)
    g.mlp_write_records(P, nrm, T, pix)
    g.mlp_targets_only()
    x6, tg, wg = g.mlp_train_set()
    assert x6.shape == (n, 6)
    # oracle: the same vertices through the oracle's own octree lookup
    cells = np.array([o.octree_lookup(p)[0] for p in P])
    oc = o.cells()
    y, w = MC.targets(cells, T, It.reshape(-1, 3)[pix], oc["factors"], oc["acc"][:, :, 6],
                      [True, True, True])
    x6o = MC.inputs(P, nrm, *MC.octree_box(sc["V"]))
    np.testing.assert_array_equal(x6, x6o)
    np.testing.assert_array_equal(wg, w)
    assert np.all(wg[:50] == 0) and (wg > 0).mean() > 0.5
    err = np.abs(tg.astype(np.float64) - y) / np.maximum(1.0, np.abs(y))
    assert err.max() < 2e-6, err.max()
    g.release()


def _depth1_vertices(ctx, mode, params, case):
    """GPU learned-cache counts and the oracle's pooled counts of every
    depth-1 vertex of one iteration with pixel-centre rays."""
    from paper_2410_20429_amd import api
    sc = scenegen.make_cornell(24, 20)
    m = api.MODE_PT_GUIDED if mode == "guided" else api.MODE_BDPT
    g = api.Scene(ctx, sc, mode=m, max_depth=3, max_cells=4000, mlp=True)
    o = orc.Oracle(sc, mode=m, max_depth=3, max_cells=4000)
    kc = 0.0 if m == api.MODE_BDPT else 50.0
    for i in range(3):
        alloc = api.ALLOC_CLASSIC if i == 0 else api.ALLOC_MARS
        kw = dict(iteration=i, spp=4, alloc=alloc, stat_clamp=kc)
        g.render_iteration(api.iter_params(**kw))
        g.update()
        o.render_iteration(orc.Oracle.params(**kw))
        o.update()
    g.set_mlp_params(params)
    spp = 2
    g.render_iteration(api.iter_params(iteration=3, spp=spp, alloc=api.ALLOC_MLP, stat_clamp=kc,
                                       center_jitter=True, debug_depth=1))
    o.render_iteration(orc.Oracle.params(iteration=3, spp=spp, alloc=orc.ALLOC_MARS,
                                         stat_clamp=kc, center_jitter=True, debug_depth=1))
    dg = np.sort(g.debug_vertices(), order="root")
    do = np.sort(o.debug_vertices(), order="root")
    assert len(dg) == len(do) > 0 and np.array_equal(dg["root"], do["root"])
    np.testing.assert_array_equal(dg["cell"], do["cell"])
    np.testing.assert_array_equal(dg["T"], do["T"])
    pix = (do["root"] // spp).astype(np.int64)
    It = o.itilde().reshape(-1, 3)[pix]
    if case == "constant":
        y = np.tile(params[M.N_PARAMS - 16:M.N_PARAMS - 13].astype(np.float64), (len(do), 1))
    else:
        W = sc["width"]
        V = sc["V"].astype(F).reshape(-1, 3, 3)
        P, nrm = [], []
        for r in do["root"]:
            px = int(r // spp)
            org, d = o.camera_ray(px % W, px // W)
            t, prim = o.intersect(org, d)
            P.append(org + F(t) * d)
            e1 = (V[prim, 1] - V[prim, 0]).astype(np.float64)
            e2 = (V[prim, 2] - V[prim, 0]).astype(np.float64)
            c = np.cross(e1, e2)
            nrm.append((c / np.linalg.norm(c)).astype(F))
        x6 = MC.inputs(np.array(P, F), np.array(nrm, F), *MC.octree_box(sc["V"]))
        y, _ = M.forward(params.astype(np.float64), x6)
    exp = MC.pooled_count(do["beta"], y, do["T"], It, 0.05, 20.0)
    g.release()
    return dg["beta"].astype(np.float64), exp, do["beta"].astype(np.float64), y


@pytest.mark.parametrize("mode", ["guided", "bdpt"])
def test_mlp_pooled_counts_constant_network(ctx, mode):
    """A network whose weights are all zero outputs its biases: the pooled
    counts then follow from the octree's counts, T and I~ alone, so every
    depth-1 count must equal the oracle's within binary32 rounding."""
    say("mlp pooled counts, constant network", mode)
    params = np.zeros(M.N_PARAMS, F)
    params[M.N_PARAMS - 16:M.N_PARAMS - 13] = [0.7, -1.2, 2.5]
    got, exp, boct, _ = _depth1_vertices(ctx, mode, params, "constant")
    np.testing.assert_allclose(got, exp, rtol=3e-6, atol=0)
    assert np.any(np.abs(got - boct) > 1e-3 * boct)      # the network changed the counts


@pytest.mark.parametrize("mode", ["guided", "bdpt"])
def test_mlp_pooled_counts_random_network(ctx, mode):
    """A random network: the counts follow the oracle's pooled formula on the
    reference network's outputs at the vertex's position and geometric
    normal, within the bfloat16 forward pass's tolerance (outputs within
    2% of their range, so the geometric mean within half of that)."""
    say("mlp pooled counts, random network", mode)
    params = M.init_params(21)
    params[M.N_PARAMS - 16:M.N_PARAMS - 13] = [0.3, -0.5, 0.8]
    got, exp, boct, y = _depth1_vertices(ctx, mode, params, "random")
    tol = 0.5 * 2e-2 * np.abs(y).max() + 1e-6
    active = boct > 0
    d = np.abs(np.log(got[active]) - np.log(exp[active]))
    assert d.max() < tol, (d.max(), tol)
    assert np.all(got[~active] == 0)
