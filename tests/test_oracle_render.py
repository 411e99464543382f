"""Pins of the oracle's renderer: closed forms (white furnace), brute-force
quadrature of direct light, unbiasedness under arbitrary counts, and
independent re-computations with library routines."""
import math

import numpy as np
import pytest
import scipy.ndimage

import scenegen
from oracle import oracle as orc


def _gather(o, params_list):
    out = []
    for p in params_list:
        o.render_iteration(p)
        out.append(o.sample_radiance().copy())
    return np.concatenate(out)


def _zscore(x, expected):
    se = x.std() / math.sqrt(len(x))
    if se == 0.0:
        # noiseless estimates (one segment): exact or infinitely far
        return 0.0 if abs(x.mean() - expected) < 1e-5 else math.inf
    return (x.mean() - expected) / se


# ---------------------------------------------------------------------------
# White furnace: closed enclosure, Le = 1, albedo a = 0.5 everywhere: every
# pixel's expectation is Le (1 - a^D) / (1 - a) for D segments, whatever the
# counts (classic RR, MARS, arbitrary fixed counts with or without T/I~).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("D", [1, 3, 5])
def test_furnace_classic(D):
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, max_depth=D)
    L = _gather(o, [orc.Oracle.params(iteration=i, spp=8, rr_start=2) for i in range(6)])[:, 0]
    exp = (1 - 0.5 ** D) / 0.5
    assert abs(_zscore(L, exp)) < 4.0 or abs(L.mean() - exp) < 1e-5


def test_furnace_mars_iterations():
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, max_depth=5)
    Ls = []
    for i in range(6):
        p = orc.Oracle.params(iteration=i, spp=4,
                              alloc=orc.ALLOC_CLASSIC if i < 1 else orc.ALLOC_MARS)
        o.render_iteration(p)
        if i >= 1:
            Ls.append(o.sample_radiance()[:, 1].copy())
        o.update(p)
    L = np.concatenate(Ls)
    assert abs(_zscore(L, 1.9375)) < 4.0
    assert o.ncells > 1


def test_furnace_random_fixed_counts():
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, max_depth=4)
    for i in range(2):  # refine the octree so that per-cell counts differ
        p = orc.Oracle.params(iteration=100 + i, spp=8)
        o.render_iteration(p)
        o.update(p)
    rng = np.random.default_rng(4)
    beta = np.stack([rng.uniform(0.05, 2.5, o.ncells), rng.uniform(0.05, 20, o.ncells),
                     np.zeros(o.ncells)], 1)
    o.set_fixed_beta(beta)
    for scale in (False, True):
        ps = [orc.Oracle.params(iteration=i, spp=4, alloc=orc.ALLOC_FIXED, fixed_scale=scale,
                                clamp_lo=0.05, clamp_hi=20.0) for i in range(4)]
        L = _gather(o, ps)[:, 2]
        assert abs(_zscore(L, (1 - 0.5 ** 4) / 0.5)) < 4.0, scale


# ---------------------------------------------------------------------------
# Direct light (depth <= 2) in the Cornell box by 256x256 midpoint quadrature
# over the emitter, with visibility computed analytically against the box.
# ---------------------------------------------------------------------------
def _slab(o, d, lo, hi, tmax):
    t0, t1 = 1e-9, tmax
    for a in range(3):
        if abs(d[a]) < 1e-12:
            if o[a] < lo[a] or o[a] > hi[a]:
                return False
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return t0 <= t1


def _cornell_first_hit(o, d, box_lo, box_hi):
    best = (np.inf, None, None)
    planes = [(1, 0.0, np.array([0, 1, 0.])), (1, 1.0, np.array([0, -1, 0.])),
              (2, 1.0, np.array([0, 0, -1.])), (0, 0.0, np.array([1, 0, 0.])),
              (0, 1.0, np.array([-1, 0, 0.]))]
    albedo = {0: np.array([.7, .7, .7]), 3: np.array([.7, .2, .2]), 4: np.array([.2, .7, .2])}
    for k, (ax, val, n) in enumerate(planes):
        if abs(d[ax]) < 1e-12:
            continue
        t = (val - o[ax]) / d[ax]
        p = o + t * d
        if t > 1e-9 and np.all(p >= -1e-9) and np.all(p <= 1 + 1e-9) and t < best[0]:
            best = (t, n, albedo.get(k, albedo[0]))
    # box faces
    for ax in range(3):
        for side, val in ((0, box_lo[ax]), (1, box_hi[ax])):
            if abs(d[ax]) < 1e-12:
                continue
            t = (val - o[ax]) / d[ax]
            p = o + t * d
            other = [a for a in range(3) if a != ax]
            if t > 1e-9 and all(box_lo[a] - 1e-9 <= p[a] <= box_hi[a] + 1e-9 for a in other):
                if t < best[0]:
                    n = np.zeros(3)
                    n[ax] = -1 if side == 0 else 1
                    best = (t, n, albedo[0])
    return best


@pytest.mark.parametrize("pix", [(10, 40), (32, 50), (50, 45), (20, 20), (45, 58), (5, 60)])
def test_direct_light_quadrature(pix):
    sc = scenegen.make_cornell(64, 64)
    o = orc.Oracle(sc, max_depth=2)
    px, py = pix
    org, dirn = o.camera_ray(px, py)
    org = org.astype(np.float64)
    dirn = dirn.astype(np.float64)
    lx, ly, lz, sx, sz = sc["light_rect"]
    blo, bhi = sc["occluder_box"][:3], sc["occluder_box"][3:]
    t, n, alb = _cornell_first_hit(org, dirn, blo, bhi)
    x = org + t * dirn
    if np.dot(n, dirn) > 0:
        n = -n
    N = 256
    us = (np.arange(N) + 0.5) / N
    U, Vv = np.meshgrid(us, us, indexing="ij")
    Y = np.stack([lx + sx * U, np.full_like(U, ly), lz + sz * Vv], -1).reshape(-1, 3)
    dv = Y - x
    r2 = (dv * dv).sum(-1)
    w = dv / np.sqrt(r2)[:, None]
    cx = np.maximum(w @ n, 0)
    cl = np.maximum(w @ np.array([0, -1.0, 0]) * -1, 0)
    vis = np.array([not _slab(x + 1e-6 * n, wi, blo, bhi, math.sqrt(rr) - 1e-6) if c > 0 else False
                    for wi, rr, c in zip(w, r2, cx * cl)])
    integrand = 15.0 * cx * cl / r2 * vis
    Lr = integrand.sum() * (sx * sz / (N * N)) * alb / math.pi
    # Monte Carlo with pixel-centre rays
    samples = []
    for it in range(64):
        p = orc.Oracle.params(iteration=it, spp=16, center_jitter=True)
        o.render_iteration(p)
        L = o.sample_radiance().reshape(64, 64, 16, 3)
        samples.append(L[py, px])
    S = np.concatenate(samples)
    se = S.std(0) / math.sqrt(len(S))
    z = np.abs(S.mean(0) - Lr) / np.maximum(se, 1e-7)
    assert np.all((z < 4.5) | (np.abs(S.mean(0) - Lr) < 1e-4 * np.maximum(Lr, 1))), (S.mean(0), Lr, se)


# ---------------------------------------------------------------------------
# Unbiasedness under arbitrary counts (supplement A.1 "Unbiasedness"):
# random per-cell fixed counts give the same image mean as counts of 1.
# Guided sampling with an arbitrary directional distribution too.
# ---------------------------------------------------------------------------
def _image_means(o, ps):
    m = []
    for p in ps:
        o.render_iteration(p)
        L = o.sample_radiance()
        m.append(L.mean(0))
    return np.array(m)


def test_unbiased_random_fixed_counts_cornell():
    sc = scenegen.make_cornell(32, 32)
    ref = orc.Oracle(sc, max_depth=3)
    ref.set_fixed_beta(np.array([[1.0, 1.0, 0.0]]))
    mref = _image_means(ref, [orc.Oracle.params(iteration=i, spp=32, alloc=orc.ALLOC_FIXED)
                              for i in range(16)])
    o = orc.Oracle(sc, max_depth=3)
    for i in range(2):
        p = orc.Oracle.params(iteration=50 + i, spp=4)
        o.render_iteration(p)
        o.update(p)
    rng = np.random.default_rng(9)
    beta = np.stack([rng.uniform(0.05, 3.0, o.ncells), rng.uniform(0.05, 20, o.ncells),
                     np.zeros(o.ncells)], 1)
    o.set_fixed_beta(beta)
    m = _image_means(o, [orc.Oracle.params(iteration=200 + i, spp=8, alloc=orc.ALLOC_FIXED)
                         for i in range(16)])
    for ch in range(3):
        a, b = mref[:, ch], m[:, ch]
        z = (a.mean() - b.mean()) / math.sqrt(a.var() / len(a) + b.var() / len(b))
        assert abs(z) < 4.0, (ch, a.mean(), b.mean(), z)


def test_guided_arbitrary_distribution_unbiased():
    sc = scenegen.make_cornell(32, 32)
    ref = orc.Oracle(sc, max_depth=3)
    mref = _image_means(ref, [orc.Oracle.params(iteration=i, spp=32) for i in range(12)])
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=3)
    rng = np.random.default_rng(1)
    w = rng.random(64) ** 4
    pm = (0.9 * w / w.sum() + 0.1 / 64).astype(np.float32)[None]
    cdf = np.cumsum(pm.astype(np.float64), 1).astype(np.float32)
    cdf[:, -1] = 1
    o.set_hist(pm, cdf)
    m = _image_means(o, [orc.Oracle.params(iteration=300 + i, spp=32) for i in range(12)])
    for ch in range(3):
        a, b = mref[:, ch], m[:, ch]
        z = (a.mean() - b.mean()) / math.sqrt(a.var() / len(a) + b.var() / len(b))
        assert abs(z) < 4.0, (ch, a.mean(), b.mean(), z)


# ---------------------------------------------------------------------------
# Determinism: repeated rendering gives identical results, independent of
# the number of threads (statistics are merged in a fixed order).
# ---------------------------------------------------------------------------
def test_determinism_across_threads():
    sc = scenegen.make_cornell(32, 32)
    res = []
    for nt in (1, 4):
        orc.set_threads(nt)
        o = orc.Oracle(sc, max_depth=5)
        orc.run_schedule(o, 4, warmup=1)
        c = o.cells()
        res.append((o.image(0), o.itilde(), c["factors"], c["acc"], o.nodes()))
    orc.set_threads(0)
    for a, b in zip(*res):
        assert a.shape == b.shape and np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Octree lookup against integer cell coordinates floor(q * 2^depth), and the
# refinement rule (visits > 32, depth < 8, budget).
# ---------------------------------------------------------------------------
def test_octree_lookup_and_refine():
    sc = scenegen.make_cornell(32, 32)
    o = orc.Oracle(sc, max_depth=5, max_cells=400)
    for i in range(4):
        p = orc.Oracle.params(iteration=i, spp=2)
        o.render_iteration(p)
        before = o.cells()
        n_before = o.ncells
        o.update(p)
        eligible = int(np.sum((before["visits"] > 32) & (before["depth"] < 8)))
        n_split = min(eligible, (400 - n_before) // 7)
        assert o.ncells == n_before + 7 * n_split
    assert o.ncells <= 400
    nodes = o.nodes()
    V = sc["V"].reshape(-1, 3)
    lo = V.min(0).astype(np.float64)
    hi = V.max(0).astype(np.float64)
    ext = (hi - lo).max()
    side = ext * (1 + 2e-4)
    olo = ((lo + hi) * 0.5 - 0.5 * side).astype(np.float32)
    inv = np.float32(1.0 / side)
    rng = np.random.default_rng(0)
    P = rng.uniform(-0.05, 1.05, (3000, 3)).astype(np.float32)
    leaf_depth = o.cells()["depth"]
    for p in P:
        cell, d = o.octree_lookup(p)
        q = np.clip((p - olo) * inv, 0, np.float32(1 - 2 ** -24)).astype(np.float64)
        iq = np.floor(q * 256).astype(np.int64)  # integer coordinates at the finest level
        node, depth = 0, 0
        while not (nodes[node] & 0x80000000):
            sh = 7 - depth
            child = ((iq[0] >> sh) & 1) | (((iq[1] >> sh) & 1) << 1) | (((iq[2] >> sh) & 1) << 2)
            node = int(nodes[node]) + int(child)
            depth += 1
        assert (nodes[node] & 0x7FFFFFFF) == cell and depth == d
        assert leaf_depth[cell] == d  # recorded depth of the leaf = its depth in the tree


# ---------------------------------------------------------------------------
# Image estimates: I~ equals a 3x3 'nearest' uniform filter of the mean image
# (scipy), floored; V_I is zero for a noiseless image.
# ---------------------------------------------------------------------------
def test_itilde_is_box_filter_of_mean():
    sc = scenegen.make_cornell(24, 20)
    o = orc.Oracle(sc, max_depth=3)
    for i in range(3):
        p = orc.Oracle.params(iteration=i, spp=2)
        o.render_iteration(p)
        o.update(p)
    mean = o.image(0).astype(np.float64)
    ref = scipy.ndimage.uniform_filter(mean, size=(3, 3, 1), mode="nearest")
    floor = np.maximum(1e-3 * mean.reshape(-1, 3).mean(0), 1e-6)
    ref = np.maximum(ref, floor)
    np.testing.assert_allclose(o.itilde(), ref, rtol=2e-6, atol=1e-9)


def test_vi_zero_without_noise():
    sc = scenegen.make_furnace(16, 16)
    o = orc.Oracle(sc, max_depth=1)
    p = orc.Oracle.params(spp=2)
    o.render_iteration(p)
    us = o.update(p)
    assert us.V_I < 1e-6
    assert abs(us.C_I - 1.0) < 1e-12  # one camera ray per sample, nothing else


# ---------------------------------------------------------------------------
# Intersection against an independent float64 ray/triangle test
# ---------------------------------------------------------------------------
def test_intersection_matches_brute_force():
    sc = scenegen.make_heightfield_scene(seed=3, grid=24, n_boxes=20)
    o = orc.Oracle(sc, max_depth=2)
    V = sc["V"].astype(np.float64).reshape(-1, 3, 3)
    rng = np.random.default_rng(1)
    bad = 0
    for _ in range(300):
        org = rng.uniform([-1, 0.3, -1], [1, 1.2, 1])
        d = rng.normal(size=3)
        d[1] = -abs(d[1])
        d /= np.linalg.norm(d)
        t, prim = o.intersect(org, d)
        e1 = V[:, 1] - V[:, 0]
        e2 = V[:, 2] - V[:, 0]
        pv = np.cross(d, e2)
        det = (e1 * pv).sum(1)
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1 / det
            s = org - V[:, 0]
            u = (s * pv).sum(1) * inv
            q = np.cross(s, e1)
            v = (q @ d) * inv
            tt = (e2 * q).sum(1) * inv
        ok = (u >= 0) & (v >= 0) & (u + v <= 1) & (tt > 0) & np.isfinite(tt)
        if not ok.any():
            bad += t is not None
            continue
        k = np.argmin(np.where(ok, tt, np.inf))
        if t is None or abs(t - tt[k]) > 1e-4 * max(1, tt[k]):
            bad += 1
    assert bad <= 1


# ---------------------------------------------------------------------------
# BDPT (Sec. 5): the full-path balance heuristic sums to one over the
# strategies of any path; the estimator matches the furnace closed form and
# the unidirectional mean under classic, MARS and random fixed counts.
# ---------------------------------------------------------------------------
def _random_paths(o, sc, rng, n, kmax):
    V = sc["V"].reshape(-1, 3, 3).astype(np.float64)
    light = [i for i in range(len(sc["tri_mat"])) if sc["mats"][sc["tri_mat"][i]][5] > 0]
    out = []
    while len(out) < n:
        k = int(rng.integers(1, kmax + 1))
        cam = np.asarray(sc["camera"][:3], np.float64)
        P, prims = [cam], [0]
        org, d = o.camera_ray(int(rng.integers(0, sc["width"])), int(rng.integers(0, sc["height"])),
                              *rng.random(2))
        ok = True
        for _ in range(k - 1):
            t, pr = o.intersect(org, d)
            if t is None:
                ok = False
                break
            x = org + t * d
            P.append(x)
            prims.append(pr)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            org = (x + 1e-4 * d).astype(np.float32)
        if not ok:
            continue
        lt = light[int(rng.integers(0, len(light)))]
        a, b = sorted(rng.random(2))
        y = V[lt, 0] * a + V[lt, 1] * (b - a) + V[lt, 2] * (1 - b)
        P.append(y)
        prims.append(lt)
        out.append((np.array(P), np.array(prims)))
    return out


@pytest.mark.parametrize("aware", [True, False])
def test_bdpt_weights_partition_of_unity(aware):
    sc = scenegen.make_cornell(16, 16)
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=8)
    for i in range(2):  # build a non-trivial cache so that counts vary per vertex
        p = orc.Oracle.params(iteration=i, spp=4, alloc=orc.ALLOC_CLASSIC if i == 0 else orc.ALLOC_MARS,
                              stat_clamp=0)
        o.render_iteration(p)
        o.update(p)
    p = orc.Oracle.params(alloc=orc.ALLOC_MARS, budget_aware=aware, stat_clamp=0)
    rng = np.random.default_rng(3)
    checked = 0
    for P, prims in _random_paths(o, sc, rng, 300, 7):
        w = o.bdpt_weights(p, P, prims, [0.2, 0.2, 0.2])
        s = float(np.sum(w.astype(np.float64)))
        if s == 0.0:
            continue  # the emitter faces away: no strategy generates this path
        assert abs(s - 1.0) < 2e-5, (s, w)
        assert np.all(w >= 0)
        checked += 1
    assert checked > 100


def test_furnace_bdpt():
    sc = scenegen.make_furnace(24, 24)
    for D in (3, 5):
        o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=D)
        Ls = []
        for i in range(6):
            p = orc.Oracle.params(iteration=i, spp=4, stat_clamp=0,
                                  alloc=orc.ALLOC_CLASSIC if i < 2 else orc.ALLOC_MARS)
            o.render_iteration(p)
            Ls.append(o.sample_radiance()[:, 0].copy())
            o.update(p)
        L = np.concatenate(Ls)
        assert abs(_zscore(L, (1 - 0.5 ** D) / 0.5)) < 4.0, D


@pytest.mark.parametrize("aware", [True, False])
def test_bdpt_unbiased_against_pt(aware):
    sc = scenegen.make_cornell(24, 24)
    ref = orc.Oracle(sc, mode=orc.MODE_PT, max_depth=4)
    mref = _image_means(ref, [orc.Oracle.params(iteration=i, spp=32, stat_clamp=0) for i in range(12)])
    o = orc.Oracle(sc, mode=orc.MODE_BDPT, max_depth=4)
    for i in range(2):
        p = orc.Oracle.params(iteration=50 + i, spp=4, stat_clamp=0)
        o.render_iteration(p)
        o.update(p)
    rng = np.random.default_rng(21)
    n = o.ncells
    o.set_fixed_beta(np.stack([rng.uniform(0.05, 2.0, n), rng.uniform(0.05, 6, n),
                               rng.uniform(0.05, 4, n)], 1))
    m = _image_means(o, [orc.Oracle.params(iteration=200 + i, spp=16, alloc=orc.ALLOC_FIXED,
                                           budget_aware=aware, stat_clamp=0, fixed_scale=bool(i % 2))
                         for i in range(12)])
    for ch in range(3):
        a, b = mref[:, ch], m[:, ch]
        z = (a.mean() - b.mean()) / math.sqrt(a.var() / len(a) + b.var() / len(b))
        assert abs(z) < 4.0, (ch, a.mean(), b.mean(), z)


# ---------------------------------------------------------------------------
# The naive rounding Alg. 1 replaces (each count rounded with its own
# uniform) is unbiased too: MARS iterations in the furnace keep the closed
# form, in the unidirectional and the bidirectional renderer.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [orc.MODE_PT, orc.MODE_BDPT])
def test_furnace_independent_rounding(mode):
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, mode=mode, max_depth=4)
    L = []
    for i in range(6):
        p = orc.Oracle.params(iteration=i, spp=4, stat_clamp=0.0, rounding=1,
                              alloc=orc.ALLOC_CLASSIC if i < 1 else orc.ALLOC_MARS)
        o.render_iteration(p)
        if i >= 1:
            L.append(o.sample_radiance()[:, 0].copy())
        o.update(p)
    L = np.concatenate(L)
    assert abs(_zscore(L, (1 - 0.5 ** 4) / 0.5)) < 4.0
