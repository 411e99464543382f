"""Pins of the learned cache's render-side arithmetic in oracle/mlp_cache.py:
the training targets and weights, and the pooled count of learned-cache
iterations.  Expected values come from closed forms (grey factors, where the
resolved count is |T / I~| times the square root of the factor), from the C
oracle's own count rule (itself pinned by the two-technique toy's fixed
point and bit-exact GPU parity), and from the definition of the geometric
mean."""
import math

import numpy as np

import scenegen
from oracle import mlp_cache as MC
from oracle import oracle as orc

F = np.float32


def _rand_T_It(rng, n):
    T = rng.uniform(0.01, 3.0, (n, 3)).astype(F)
    It = rng.uniform(0.01, 2.0, (n, 3)).astype(F)
    return T, It


# ---------------------------------------------------------------------------
# Grey factors a (RR) and s (splitting) in every channel: beta^RR = |T/I~|
# sqrt(a) and beta^S = |T/I~| sqrt(s), so the target is 0.5 log a when
# beta^RR < 1, 0.5 log s when beta^S > 1, and -log|T/I~| when the count
# resolves to 1.  Catches: the target taken relative to T alone or to I~
# alone, the channel norm without its 1/3, the resolve cases swapped.
# ---------------------------------------------------------------------------
def test_targets_closed_form_grey_factors():
    rng = np.random.default_rng(1)
    n = 3000
    T, It = _rand_T_It(rng, n)
    a = rng.uniform(0.001, 5.0, n)
    s = a * rng.uniform(0.0, 1.0, n)            # variance <= second moment
    fac = np.zeros((n, 2, 3, 3), F)
    for t in range(3):
        fac[:, 0, t, :] = a[:, None]
        fac[:, 1, t, :] = s[:, None]
    counts = np.full((n, 3), 10.0)
    y, w = MC.targets(np.arange(n), T, It, fac, counts, [True, True, True])
    sm = np.sqrt(np.mean((T.astype(np.float64) / It) ** 2, 1))
    brr, bs = sm * np.sqrt(a), sm * np.sqrt(s)
    expect = np.where(brr < 1, 0.5 * np.log(a), np.where(bs > 1, 0.5 * np.log(s), -np.log(sm)))
    # near a case boundary binary32 may resolve differently: compare away from it
    far = (np.abs(brr - 1) > 1e-5) & (np.abs(bs - 1) > 1e-5) & (s > 0)
    assert far.sum() > 2500
    for t in range(3):
        np.testing.assert_allclose(y[far, t], expect[far], rtol=0, atol=2e-6)
    assert np.all(w[far] == F(10.0 / 64.0))


def test_target_weights():
    rng = np.random.default_rng(2)
    T, It = _rand_T_It(rng, 8)
    fac = np.full((8, 2, 3, 3), 0.5, F)
    fac[7, 0, 1, 0] = -1.0                          # technique 1 of cell 7: no data
    counts = np.array([[0, 3, 4], [5, 63, 64], [65, 1000, 2], [4, 4, 4],
                       [3.9, 64.5, 7], [0, 0, 0], [1e9, 1, 1], [10, 10, 10]], np.float64)
    y, w = MC.targets(np.arange(8), T, It, fac, counts, [True, True, False])
    exp = np.where(counts >= 4, np.minimum(counts, 64) / 64.0, 0.0)
    exp[:, 2] = 0.0                                 # disabled technique
    exp[7, 1] = 0.0
    np.testing.assert_array_equal(w, exp.astype(F))
    assert np.all(y[w == 0] == 0.0)


# ---------------------------------------------------------------------------
# The target's count equals the C oracle's own count rule: with the clamp
# opened to (0, inf), |T/I~| exp(y*) must give back the count the oracle's
# renderer draws with for that cell, T and I~.  Catches: targets built from
# a different resolve, colour rule or factor slot than the counts.
# ---------------------------------------------------------------------------
def test_target_count_matches_oracle_count_rule():
    rng = np.random.default_rng(3)
    sc = scenegen.make_cornell(8, 8)
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=3)
    for i in range(3):
        p = orc.Oracle.params(iteration=i, spp=16)
        o.render_iteration(p)
        o.update(p)
    nc = o.ncells
    fac = np.abs(rng.lognormal(-1.0, 1.5, (nc, 2, 3, 3))).astype(F)
    fac[:, 1] = fac[:, 0] * rng.uniform(0, 1, (nc, 3, 3)).astype(F)
    o.write_cells(factors=fac)
    p = orc.Oracle.params(alloc=orc.ALLOC_MARS, clamp_lo=0.0, clamp_hi=3.0e38)
    cells = rng.integers(0, nc, 400)
    T, It = _rand_T_It(rng, 400)
    y, w = MC.targets(cells, T, It, o.cells()["factors"], np.full((nc, 3), 100.0),
                      [True, True, True])
    sm, _ = MC.t_over_i(T, It)
    for k in range(400):
        b = o.cell_beta(p, int(cells[k]), T[k], It[k])
        np.testing.assert_allclose(sm[k] * np.exp(y[k]), b.astype(np.float64), rtol=2e-6)


# ---------------------------------------------------------------------------
# Pooled count.  Its fixed point: a network that outputs the target gives
# back the octree's count (inside the clamp).  In general it is the
# geometric mean of the two counts, clamped; the octree's count stays where
# the network's is not finite; a technique without samples stays off.
# ---------------------------------------------------------------------------
def test_pooled_count_fixed_point_and_geometric_mean():
    rng = np.random.default_rng(4)
    n = 2000
    T, It = _rand_T_It(rng, n)
    fac = rng.lognormal(-1.0, 1.0, (n, 2, 3, 3)).astype(F)
    fac[:, 1] = fac[:, 0] * F(0.5)
    y, w = MC.targets(np.arange(n), T, It, fac, np.full((n, 3), 64.0), [True, True, True])
    sm, z = MC.t_over_i(T, It)
    bh = np.stack([MC.octree_count_unclamped(fac[:, :, t, :], z) for t in range(3)], 1)
    lo, hi = 0.05, 20.0
    inside = (bh > lo) & (bh < hi)
    boct = np.clip(bh, lo, hi).astype(np.float64)
    pooled = MC.pooled_count(boct, y, T, It, lo, hi)
    np.testing.assert_allclose(pooled[inside], boct[inside], rtol=2e-6)
    # the geometric mean with an arbitrary network count
    y2 = rng.normal(0, 2, (n, 3))
    net = sm.astype(np.float64)[:, None] * np.exp(y2)
    pooled = MC.pooled_count(boct, y2, T, It, lo, hi)
    np.testing.assert_allclose(pooled, np.clip(np.sqrt(boct * net), lo, hi), rtol=1e-12)
    # non-finite network output: the octree's count; -inf: the clamp's floor
    yb = np.array([[np.inf, np.nan, -np.inf]])
    out = MC.pooled_count(np.array([[2.0, 3.0, 4.0]]), yb, T[:1], It[:1], lo, hi)
    assert out[0, 0] == 2.0 and out[0, 1] == 3.0 and out[0, 2] == lo
    out = MC.pooled_count(np.array([[0.0, 1.0, 0.0]]), np.zeros((1, 3)), T[:1], It[:1], lo, hi)
    assert out[0, 0] == 0.0 and out[0, 2] == 0.0 and out[0, 1] > 0


def test_inputs_normalise_to_the_octree_cube():
    sc = scenegen.make_cornell(8, 8)
    lo, inv = MC.octree_box(sc["V"])
    V = sc["V"].reshape(-1, 3).astype(np.float64)
    side = (V.max(0) - V.min(0)).max() * (1 + 2e-4)
    assert abs(1.0 / float(inv) - side) < 1e-6 * side
    P = np.array([[0, 0, 0], [1, 1, 1], [0.5, 0.5, 0.5], [-5, 7, 0.25]], F)
    x = MC.inputs(P, np.tile(np.array([[0, 1, 0]], F), (4, 1)), lo, inv)
    assert np.all(x[:, :3] >= 0) and np.all(x[:, :3] < 1)
    assert np.allclose(x[2, :3], 0.5, atol=1e-6)
    assert x[3, 0] == 0.0 and x[3, 1] == F(1.0) - F(2.0 ** -24)
    assert np.all(x[:, 3:] == [0, 1, 0])
    assert math.isclose(float(x[0, 0]), float((F(0) - lo[0]) * inv), rel_tol=0, abs_tol=0)
