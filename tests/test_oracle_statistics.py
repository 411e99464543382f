"""Pins of the oracle's statistics: the per-cell records of the primary
estimates <L_r,t> and their costs (Sec. 4.1 "Local estimates"), the image
variance estimate V_I (Sec. 4.1 "Image estimates"), the training of the
guided directional histogram, and the form of the budget-aware balance
heuristic (Sec. 3 "Proxy model"; supplement A.1).

Each test names the mistakes it is built to catch.  None of them re-types
the oracle's formula: the expected values come from closed forms of the
white furnace, from counting arguments over the path tree, from independent
Monte Carlo estimates over many iterations, or from a quadrature of the
emitter's incident radiance."""
import math

import numpy as np
import pytest

import scenegen
from oracle import oracle as orc

LR_D2 = 0.5    # furnace (Le = 1, a = 0.5): reflected radiance with one bounce left
LR_D3 = 0.75   # ... with two bounces left: a Le + a^2 Le


def _zs(samples, expected):
    s = np.asarray(samples, np.float64)
    return (s.mean() - expected) / max(s.std(ddof=1) / math.sqrt(len(s)), 1e-12)


# ---------------------------------------------------------------------------
# budget-aware balance heuristic: every weight is beta_t p_t over one common
# denominator, so w_t / (beta_t p_t) is the same for every technique of the
# sum, and each sample contributes f / sum_k beta_k p_k.
# Catches: weights of the form beta^2 p or sqrt(beta) p (which still sum to
# one), an NEE density left out of the direct denominator or put into the
# indirect one, the indicator form in place of the budget-aware one.
# ---------------------------------------------------------------------------
def test_mis_weight_is_beta_p_over_one_denominator():
    rng = np.random.default_rng(11)
    for _ in range(500):
        beta = rng.uniform(0.05, 20.0, 3).astype(np.float32)
        p = rng.uniform(0.01, 5.0, 3).astype(np.float32)
        wd, wi = orc.mis(1, beta, p)
        bp = beta.astype(np.float64) * p
        np.testing.assert_allclose(wd / bp, np.full(3, 1.0 / bp.sum()), rtol=2e-6)
        np.testing.assert_allclose(wi[[0, 2]] / bp[[0, 2]], np.full(2, 1.0 / (bp[0] + bp[2])),
                                   rtol=2e-6)
        assert wi[1] == 0.0
        # budget-unaware: indicators in place of the counts
        wd, wi = orc.mis(0, beta, p)
        np.testing.assert_allclose(wd / p, np.full(3, 1.0 / p.astype(np.float64).sum()),
                                   rtol=2e-6)
        np.testing.assert_allclose(wi[[0, 2]] / p[[0, 2]],
                                   np.full(2, 1.0 / (float(p[0]) + float(p[2]))), rtol=2e-6)
    # a disabled technique (count 0) takes no share in either form
    for aware in (0, 1):
        wd, wi = orc.mis(aware, np.array([2.0, 0.0, 0.5], np.float32),
                         np.array([0.3, 1.0, 0.7], np.float32))
        assert wd[1] == 0.0 and abs(wd.sum() - 1.0) < 1e-6 and abs(wi.sum() - 1.0) < 1e-6


# ---------------------------------------------------------------------------
# Sample-statistic records in the white furnace at D = 2 with fixed counts.
# Every vertex at depth 1 reflects a Le = 0.5 in expectation; its samples
# are the only records (depth-2 vertices draw none).  For every cell the
# per-technique means of the records sum to 0.5, and every sample costs
# exactly one ray (an NEE shadow ray, or a continuation ray that ends the
# path).  Catches: records of v / beta_t instead of v, a dropped MIS weight
# or emission term, costs that count more or fewer rays.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [orc.MODE_PT, orc.MODE_PT_GUIDED, orc.MODE_BDPT])
def test_records_furnace_depth2(mode):
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, mode=mode, max_depth=2, max_cells=4000)
    for i in range(4):  # refine until many cells see the camera's vertices
        p = orc.Oracle.params(iteration=40 + i, spp=4, stat_clamp=0.0)
        o.render_iteration(p)
        o.update(p)
    n = o.ncells
    assert n > 8
    rng = np.random.default_rng(5)
    third = np.zeros(n) if mode == orc.MODE_PT else rng.uniform(0.3, 2.5, n)
    beta = np.stack([rng.uniform(0.3, 2.5, n), rng.uniform(0.3, 2.5, n), third], 1)
    o.set_fixed_beta(beta)
    p = orc.Oracle.params(iteration=7, spp=48, alloc=orc.ALLOC_FIXED, stat_clamp=0.0)
    o.render_iteration(p)
    acc = o.cells()["acc"]          # [cell][tech][sum3, sum2_3, n, cost]
    nt = acc[:, :, 6]
    techs = [0, 1] if mode == orc.MODE_PT else [0, 1, 2]
    if mode == orc.MODE_BDPT:
        techs = [0, 1]  # at D = 2 no connection fits: a light vertex needs a third segment
        assert np.all(nt[:, 2] == 0) or np.all(acc[:, 2, 0] == 0)
    zs = []
    for c in range(n):
        if np.any(nt[c, techs] < 60):
            continue
        mean = sum(acc[c, t, 0] / nt[c, t] for t in techs)
        var = sum((acc[c, t, 3] / nt[c, t] - (acc[c, t, 0] / nt[c, t]) ** 2) / nt[c, t]
                  for t in techs)
        zs.append((mean - LR_D2) / math.sqrt(max(var, 1e-18)))
        for t in techs:
            assert acc[c, t, 7] == nt[c, t], (c, t)  # one ray per sample
    zs = np.array(zs)
    assert len(zs) >= 8
    assert np.max(np.abs(zs)) < 4.5, zs
    assert np.mean(zs ** 2) < 2.0, zs


# ---------------------------------------------------------------------------
# The same records at D = 3 over the whole path tree, by counting.  With
# global fixed counts beta and N camera samples, the vertices at depth 1 (N
# of them, each reflecting 0.75) and depth 2 (N b of them, each reflecting
# 0.5) give
#     sum_t (sum of records of t) / beta_t = N (0.75 + 0.5 b),
# where b = beta_B + beta_G / 2 is the expected number of continuations per
# vertex: the guided distribution starts uniform over the sphere, and the
# half of its directions below the surface ends the sample without a ray.
# NEE samples cost one ray each; a continuation at depth 1 costs 1 plus the
# samples of its depth-2 vertex, one at depth 2 (or one that ended at once)
# costs 1:
#     sum cost_B = N beta_B (1 + beta_N + beta_B + beta_G) + N b beta_B,
#     n_B        = N beta_B (1 + b),
#     sum cost_G = N beta_G/2 (1 + beta_N + beta_B + beta_G) + N beta_G/2 + N b beta_G.
# Catches: records divided by beta, costs without the subtree's rays (or
# with the parent's own ray counted twice), records of the secondary instead
# of the primary estimate.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [orc.MODE_PT, orc.MODE_PT_GUIDED])
def test_records_furnace_depth3_counts(mode):
    sc = scenegen.make_furnace(24, 24)
    o = orc.Oracle(sc, mode=mode, max_depth=3, max_cells=1)
    bB, bN = 0.6, 1.7
    bG = 0.0 if mode == orc.MODE_PT else 0.9
    o.set_fixed_beta(np.array([[bB, bN, bG]]))
    N = 24 * 24 * 8
    val, cB, cN, cG, nB, nN = [], [], [], [], [], []
    for it in range(10):
        o.render_iteration(orc.Oracle.params(iteration=it, spp=8, alloc=orc.ALLOC_FIXED,
                                             stat_clamp=0.0))
        a = o.cells()["acc"].sum(0)   # [tech][8], grey furnace: channel 0
        s = a[0, 0] / bB + a[1, 0] / bN + (a[2, 0] / bG if bG > 0 else 0.0)
        val.append(s / N)
        cB.append(a[0, 7] / a[0, 6])
        cN.append(a[1, 7] / a[1, 6])
        nB.append(a[0, 6] / N)
        nN.append(a[1, 6] / N)
        if bG > 0:
            cG.append(a[2, 7] / a[2, 6])
    b = bB + 0.5 * bG
    sub = 1 + bN + bB + bG          # rays of a continuation sample started at depth 1
    assert abs(_zs(val, LR_D3 + 0.5 * b)) < 4.5, (np.mean(val), LR_D3 + 0.5 * b)
    assert abs(_zs(nB, bB * (1 + b))) < 4.5
    assert abs(_zs(nN, bN * (1 + b))) < 4.5
    exp_cB = (bB * sub + b * bB) / (bB * (1 + b))
    assert abs(_zs(cB, exp_cB)) < 4.5, (np.mean(cB), exp_cB)
    assert np.all(np.array(cN) == 1.0)
    if bG > 0:
        exp_cG = (0.5 * bG * sub + 0.5 * bG + b * bG) / (bG * (1 + b))
        assert abs(_zs(cG, exp_cG)) < 4.5, (np.mean(cG), exp_cG)


# ---------------------------------------------------------------------------
# Bidirectional records at D = 3, from the vertices at depth 1 only.  With
# full-path MIS a vertex's own samples carry only the strategies that sample
# it from the camera side, so the identity holds at depth 1, where every
# strategy t >= 2 does: sum_t (records of t) / beta_t = 0.75 N, the light-
# path records being the weighted contributions of whole light subpaths.
# Costs: an NEE sample one ray; a light-path sample its connection rays (one
# here: a connection from depth 1 reaches y_1 only); a BSDF sample 1 plus
# the samples of its depth-2 vertex, each of which costs one ray or, for a
# light-path sample with no connection that fits, the minimum of one:
# C_B = 1 + beta_B + beta_N + beta_L.
# Catches: the light-path records divided by beta or missing their MIS
# weight, the light subpath's throughput left out, connection costs counted
# per light vertex that cannot be reached.
# ---------------------------------------------------------------------------
def test_records_furnace_bdpt_depth3():
    sc = scenegen.make_furnace(24, 24)
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=3, max_cells=1)
    o.set_record_depth(1)
    bB, bN, bL = 0.7, 1.3, 1.6
    o.set_fixed_beta(np.array([[bB, bN, bL]]))
    N = 24 * 24 * 8
    val, cB, cL, nL = [], [], [], []
    for it in range(10):
        o.render_iteration(orc.Oracle.params(iteration=it, spp=8, alloc=orc.ALLOC_FIXED,
                                             stat_clamp=0.0))
        a = o.cells()["acc"].sum(0)
        val.append((a[0, 0] / bB + a[1, 0] / bN + a[2, 0] / bL) / N)
        assert a[1, 7] == a[1, 6]
        cB.append(a[0, 7] / a[0, 6])
        cL.append(a[2, 7] / a[2, 6])
        nL.append(a[2, 6] / N)
    assert abs(_zs(val, LR_D3)) < 4.5, (np.mean(val), LR_D3)
    assert abs(_zs(cB, 1 + bB + bN + bL)) < 4.5, (np.mean(cB), 1 + bB + bN + bL)
    assert abs(np.mean(cL) - 1.0) < 1e-3, np.mean(cL)
    assert abs(_zs(nL, bL)) < 4.5


# ---------------------------------------------------------------------------
# V_I against an independent estimate of the image's relative per-sample
# variance: the furnace has the same expectation in every pixel, so the
# box-filtered I~ converges to it; the mean of V_I over iterations must equal
# the per-pixel sample variance over all iterations divided by the squared
# pixel mean, averaged over pixels and channels, within 3%.  Catches: a
# missing or doubled 1/spp, the channel sum without its 1/3, the deviation
# divided by I~ once instead of squared, the pixel mean taken over the
# included pixels wrongly.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [orc.MODE_PT, orc.MODE_PT_GUIDED])
def test_vi_matches_independent_variance(mode):
    W = H = 24
    spp = 4
    sc = scenegen.make_furnace(W, H)
    o = orc.Oracle(sc, mode=mode, max_depth=3, max_cells=1)
    o.set_fixed_beta(np.array([[0.7, 1.3, 0.0 if mode == orc.MODE_PT else 0.8]]))
    vis, Ls = [], []
    n_iter, skip = 48, 8
    for it in range(n_iter):
        p = orc.Oracle.params(iteration=it, spp=spp, alloc=orc.ALLOC_FIXED, stat_clamp=0.0)
        o.render_iteration(p)
        Ls.append(o.sample_radiance().reshape(H * W, spp, 3).astype(np.float64))
        us = o.update(p)
        assert us.n_excluded == 0
        if it >= skip:
            vis.append(us.V_I)
    S = np.concatenate(Ls[skip:], axis=1)                  # [pixel][samples][ch]
    mu = np.concatenate(Ls, axis=1).mean(1)                # all iterations' samples
    rel = (S.var(1, ddof=1) / mu ** 2).mean()
    assert abs(np.mean(vis) / rel - 1.0) < 0.03, (np.mean(vis), rel)


# ---------------------------------------------------------------------------
# Histogram training (guided technique): a continuation sample in direction
# w adds lum(L_i(w)) / (beta_B p_B(w) + beta_G p_G(w)) to bin(w); since the
# continuation samples have that density, the bins estimate the integral of
# the incident luminance over each bin's solid angle, summed over vertices.
# Direct light only (D = 2) from a quad emitter above a floor, one cell,
# fixed counts and a non-uniform starting distribution: the learned pmf
# (0.9 learned + 0.1 uniform) must match a midpoint quadrature of the
# emitter's solid angle per bin.  Catches: the luminance added without the
# density of continuation samples, a bin taken from the outgoing direction,
# the uniform share mixed in with the wrong weight.  (Dividing by each
# technique's own density instead is also unbiased for the integral, up to
# the factor beta_B + beta_G, and gives the same normalised distribution.)
# ---------------------------------------------------------------------------
def _floor_and_emitter(width, height, le=3.0):
    rect = (0.1, -0.4, 1.0, 1.0, 0.6)  # x0, y0, size x, size y, height
    mats = [scenegen._mat(scenegen.LAMBERT, 0.8),
            scenegen._mat(scenegen.LAMBERT, 0.0, le=(le, le, le))]
    tris, tm = [], []
    t = scenegen._quad((-3, -3, 0), (6, 0, 0), (0, 6, 0))          # floor, normal +z
    tris += t
    tm += [0] * len(t)
    x0, y0, sx, sy, h = rect
    t = scenegen._quad((x0, y0, h), (0, sy, 0), (sx, 0, 0))       # emitter, normal -z
    tris += t
    tm += [1] * len(t)
    cam = [0.0, 0.0, 0.3, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 60.0]
    return scenegen._finish(tris, tm, mats, cam, width, height, "floor_emitter"), rect


def _bin_quadrature(points, rect, le, n=48):
    x0, y0, sx, sy, h = rect
    Q = np.zeros(64)
    us = (np.arange(n) + 0.5) / n
    for bz in range(4, 8):          # the emitter is above the floor: z > 0
        z = -1.0 + 0.25 * (bz + us)
        for bp in range(8):
            phi = (bp + us) * (math.pi / 4)
            Z, PH = np.meshgrid(z, phi, indexing="ij")
            s = np.sqrt(1 - Z * Z)
            d = np.stack([s * np.cos(PH), s * np.sin(PH), Z], -1).reshape(-1, 3)
            dA = (0.25 / n) * ((math.pi / 4) / n)
            tot = 0.0
            for x in points:
                t = (h - x[2]) / d[:, 2]
                hx = x[0] + t * d[:, 0]
                hy = x[1] + t * d[:, 1]
                inside = (hx >= x0) & (hx <= x0 + sx) & (hy >= y0) & (hy <= y0 + sy)
                tot += inside.sum()
            Q[bz * 8 + bp] = le * tot * dA
    return Q


def test_histogram_training_matches_quadrature():
    W = H = 12
    sc, rect = _floor_and_emitter(W, H)
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=2, max_cells=1, split_visits=1 << 30)
    o.set_fixed_beta(np.array([[0.6, 1.0, 1.4]]))
    rng = np.random.default_rng(3)
    w = rng.random(64) ** 3 + 0.02
    pm = (w / w.sum()).astype(np.float32)[None]
    cdf = np.cumsum(pm.astype(np.float64), 1).astype(np.float32)
    cdf[:, -1] = 1.0
    o.set_hist(pm, cdf)
    # primary hit points of the pixel-centre rays on the floor z = 0
    pts = []
    for py in range(H):
        for px in range(W):
            org, d = o.camera_ray(px, py)
            t = -float(org[2]) / float(d[2])
            pts.append(org.astype(np.float64) + t * d.astype(np.float64))
    Q = _bin_quadrature(np.array(pts), rect, 3.0)
    expect = Q / Q.sum()
    learned = []
    for it in range(8):
        p = orc.Oracle.params(iteration=it, spp=96, alloc=orc.ALLOC_FIXED, center_jitter=True,
                              stat_clamp=0.0)
        o.render_iteration(p)
        o.update(p)
        assert o.ncells == 1
        pmo, cdfo = o.hist()
        learned.append((pmo[0].astype(np.float64) - 0.1 / 64) / 0.9)
        assert abs(float(cdfo[0, -1]) - 1.0) < 1e-6
    L = np.array(learned)
    m, se = L.mean(0), L.std(0, ddof=1) / math.sqrt(len(L))
    big = expect > 0.02
    assert big.sum() >= 6
    z = (m - expect) / np.maximum(se, 1e-9)
    assert np.all(np.abs(z[big]) < 4.5 + 0.01 / np.maximum(se[big], 1e-9)), (m[big], expect[big])
    assert np.all(np.abs(m - expect) < 0.01), np.abs(m - expect).max()
    # bins the emitter cannot reach learn nothing
    assert np.all(np.abs(m[expect == 0]) < 1e-6)
