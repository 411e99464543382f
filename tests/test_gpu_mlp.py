"""Learned cache on the GPU (through the C ABI) against the binary64
reference network: matrix-core lane layout, forward, gradient, Adam, and the
render loop with network-predicted counts."""
import math

import numpy as np
import pytest

import scenegen
from oracle import mlp_ref as M
from oracle import oracle as orc

pytestmark = pytest.mark.gpu


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


def _bf16_bits(x):
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def test_mfma_probe_layout(ctx):
    say("mfma probe")
    rng = np.random.default_rng(0)
    A = rng.normal(size=(16, 16)).astype(np.float32)
    B = rng.normal(size=(16, 16)).astype(np.float32)
    inp = np.concatenate([_bf16_bits(A).ravel(), _bf16_bits(B).ravel()])
    D = ctx.probe(3, inp, (1, 256), np.float32).reshape(16, 16)
    ref = M.bf16(A) @ M.bf16(B)
    np.testing.assert_allclose(D, ref, rtol=1e-5, atol=1e-5)


def _inputs(rng, n):
    return np.concatenate([rng.random((n, 3)), rng.uniform(-1, 1, (n, 3))], 1).astype(np.float32)


@pytest.fixture(scope="module")
def mlp_scene(ctx):
    api = _api()
    return api.Scene(ctx, scenegen.make_cornell(16, 16), max_depth=3, mlp=True)


def test_mlp_forward_parity(mlp_scene):
    say("mlp forward")
    rng = np.random.default_rng(1)
    params = M.init_params(7)
    params[M.N_PARAMS - 16:M.N_PARAMS - 13] = [0.3, -0.2, 0.5]  # output biases
    mlp_scene.set_mlp_params(params)
    np.testing.assert_array_equal(mlp_scene.mlp_params(), params)
    x = _inputs(rng, 1000)
    y = mlp_scene.mlp_forward(x)
    yr, _ = M.forward(params.astype(np.float64), x)
    scale = np.abs(yr).max()
    assert np.abs(y - yr).max() < 2e-2 * scale, (np.abs(y - yr).max(), scale)
    assert np.corrcoef(y.ravel(), yr.ravel())[0, 1] > 0.9995


def test_mlp_gradient_parity(mlp_scene):
    say("mlp gradient")
    rng = np.random.default_rng(2)
    params = M.init_params(9)
    mlp_scene.set_mlp_params(params)
    n = 777  # ragged: not a multiple of the 16-sample tile
    x = _inputs(rng, n)
    tgt = rng.normal(size=(n, 3)).astype(np.float32)
    w = rng.random((n, 3)).astype(np.float32)
    w[rng.random((n, 3)) < 0.2] = 0.0
    loss, g = mlp_scene.mlp_grad(x, tgt, w)
    lref, gref = M.loss_and_grad(params.astype(np.float64), x.astype(np.float64),
                                 tgt.astype(np.float64), w.astype(np.float64))
    assert abs(loss - lref) < 1e-3 * lref
    cos = float(np.dot(g, gref) / (np.linalg.norm(g) * np.linalg.norm(gref)))
    assert cos > 0.999, cos
    for name, sl in _slices():
        a, b = g[sl], gref[sl]
        assert np.abs(a - b).max() < 2e-2 * np.abs(b).max() + 1e-12, name
    assert np.all(g[M.N_PARAMS - 16 + 3:] == 0) and np.all(M.unpack(g)["W4"][3:] == 0)


def _slices():
    o = 0
    for name, shp in M.SHAPES:
        n = int(np.prod(shp))
        yield name, slice(o, o + n)
        o += n


def test_mlp_adam_matches_reference(mlp_scene):
    say("mlp adam")
    rng = np.random.default_rng(3)
    params = M.init_params(11)
    mlp_scene.set_mlp_params(params)
    w, m, v = params.copy(), np.zeros_like(params), np.zeros_like(params)
    for step in range(1, 4):
        g = (rng.normal(size=params.shape) * 1e-2).astype(np.float32)
        g[M.N_PARAMS - 13:] = 0
        mlp_scene.mlp_apply_grad(g, lr=1e-3)
        w, m, v = M.adam_step(w, g, m, v, step, lr=1e-3)
    got = mlp_scene.mlp_params()
    np.testing.assert_allclose(got, w, rtol=1e-6, atol=1e-9)


def test_mlp_training_fits_smooth_target(ctx):
    """Adam on a fixed synthetic set lowers the loss by an order of magnitude
    (targets are a smooth function of position and normal)."""
    api = _api()
    s = api.Scene(ctx, scenegen.make_cornell(8, 8), max_depth=2, mlp=True)
    rng = np.random.default_rng(4)
    n = 8192
    x = _inputs(rng, n)
    tgt = np.stack([np.sin(3 * x[:, 0]) + x[:, 4], np.cos(2 * x[:, 1]) - x[:, 3], x[:, 2] * x[:, 5]],
                   1).astype(np.float32)
    w = np.ones((n, 3), np.float32)
    l0, _ = s.mlp_grad(x, tgt, w)
    for it in range(300):
        _, g = s.mlp_grad(x, tgt, w)
        s.mlp_apply_grad(g, lr=3e-3)
    l1, _ = s.mlp_grad(x, tgt, w)
    say("fit loss", l0, "->", l1)
    assert l1 < 0.1 * l0


def _relmse(img, ref, eps=1e-2):
    d = img.astype(np.float64) - ref
    return float(np.mean(np.mean(d * d / (ref * ref + eps), axis=-1)))


def test_mlp_render_unbiased_and_gain(ctx):
    """Octree MARS and learned-cache MARS on the Cornell box: the image mean
    agrees with a counts-of-one reference (unbiased for any counts), and the
    learned cache's efficiency 1/(relMSE x rays) of its inverse-variance
    weighted image, against an independent 4096 spp reference, is at least
    the octree's (rays rather than seconds: deterministic)."""
    api = _api()
    sc = scenegen.make_cornell(64, 64)
    ref = api.Scene(ctx, sc, max_depth=5)
    ref.set_fixed_counts(np.array([[1.0, 1.0, 0.0]]))
    mref, img = [], np.zeros((64, 64, 3))
    for it in range(64):
        ref.render_iteration(api.iter_params(iteration=900 + it, spp=64, alloc=api.ALLOC_FIXED))
        mref.append(ref.sample_radiance().mean(0))
        img += ref.image(api.IMAGE_LAST)
    img /= 64
    ref.release()
    effs, means, errs, rays = {}, {}, {}, {}
    for mode in ("octree", "mlp"):
        s = api.Scene(ctx, sc, max_depth=5, mlp=(mode == "mlp"))
        mm, r = [], 0
        for it in range(14):
            alloc = api.ALLOC_CLASSIC if it < 1 else api.ALLOC_MARS
            if mode == "mlp" and it >= 4:
                alloc = api.ALLOC_MLP
            p = api.iter_params(iteration=it, spp=4, alloc=alloc)
            r += s.render_iteration(p).total_rays()
            if it >= 6:
                mm.append(s.sample_radiance().mean(0))
            s.update(p)
            if mode == "mlp" and it >= 1:
                s.mlp_train(steps=16, batch=8192, lr=2e-3)
        errs[mode] = _relmse(s.image(api.IMAGE_IVW), img)
        rays[mode] = r
        effs[mode] = 1.0 / (errs[mode] * r)
        means[mode] = np.array(mm)
        s.release()
    say("relMSE octree", errs["octree"], "mlp", errs["mlp"], "rays", rays,
        "efficiency ratio", effs["mlp"] / effs["octree"])
    a = np.array(mref)
    for mode in ("octree", "mlp"):
        b = means[mode]
        z = (a.mean(0) - b.mean(0)) / np.sqrt(a.var(0) / len(a) + b.var(0) / len(b))
        assert np.all(np.abs(z) < 4.5), (mode, z)
    assert effs["mlp"] >= 1.0 * effs["octree"], (errs, rays)


def test_mlp_bdpt_furnace_unbiased(ctx):
    """Bidirectional MARS with the learned cache in the white furnace, with a
    network whose counts vary strongly over the scene: the MIS weights of
    every strategy evaluate the count function the samples are drawn with
    (the network's at the camera vertices, from their records, and at the
    light vertices for the strategies that would have reached them from the
    camera side), so the weights of a path sum to one and the estimate keeps
    the closed-form mean."""
    api = _api()
    sc = scenegen.make_furnace(48, 48)
    g = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=5, mlp=True)
    params = M.init_params(11)
    p = M.unpack(params)
    p["W4"][:3] *= 10.0  # log-count outputs with a spread of about +-2
    g.set_mlp_params(M.pack(p).astype(np.float32))
    L = []
    for it in range(10):
        alloc = api.ALLOC_CLASSIC if it < 1 else (api.ALLOC_MARS if it < 2 else api.ALLOC_MLP)
        par = api.iter_params(iteration=it, spp=4, stat_clamp=0.0, alloc=alloc, clamp_hi=6.0)
        g.render_iteration(par)
        if it >= 2:
            L.append(g.sample_radiance()[:, 0].copy())
        g.update(par)
    L = np.concatenate(L)
    z = (L.mean() - 1.9375) / (L.std() / math.sqrt(len(L)))
    say("bdpt furnace with the learned cache: mean", L.mean(), "z", z)
    assert abs(z) < 4.0, (L.mean(), z)
