"""EARS allocation in the oracle (the comparison method of Sec. 5: one count
shared by every technique of a vertex, beta_t = r_t lambda).  The shared
factor is pinned against a numerical optimum of the efficiency model of
Sec. 3.1 along that line, against the per-technique fixed point where the two
must agree, and by unbiasedness in the white furnace."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import scenegen
from oracle import oracle as orc

RATIOS = {orc.MODE_PT: (1.0, 1.0, 0.0), orc.MODE_PT_GUIDED: (0.5, 1.0, 0.5),
          orc.MODE_BDPT: (1.0, 1.0, 1.0)}


def _acc(stats):
    """stats: per technique (n, E1[3], E2[3], mean cost) -> accumulators [1, 3, 8]."""
    acc = np.zeros((1, 3, 8))
    for t, (n, e1, e2, c) in enumerate(stats):
        acc[0, t, 0:3] = n * np.asarray(e1)
        acc[0, t, 3:6] = n * np.asarray(e2)
        acc[0, t, 6] = n
        acc[0, t, 7] = n * c
    return acc


def _oracle(mode):
    o = orc.Oracle(scenegen.make_furnace(8, 8), mode=mode, max_depth=3)
    assert o.ncells == 1
    return o


def _factors_after(o, acc, V_I, C_I, ears):
    o.write_cells(factors=-np.ones((1, 2, 3, 3), np.float32), acc=acc)
    o.update_cells_only(V_I, C_I, ears=ears)
    return o.cells()["factors"][0]


STATS = [(120, (0.21, 0.35, 0.12), (0.52, 0.41, 0.23), 3.1),
         (64, (0.40, 0.10, 0.33), (0.95, 0.30, 0.61), 1.4),
         (90, (0.05, 0.18, 0.27), (0.31, 0.72, 0.44), 2.2)]


@pytest.mark.parametrize("mode", [orc.MODE_PT_GUIDED, orc.MODE_BDPT])
def test_ears_factor_is_the_model_optimum_on_the_line(mode):
    # efficiency model of one vertex's choice (Sec. 3.1): image variance
    # V_I + eps sum_t M_t / beta_t times cost C_I + eps sum_t beta_t C_t; with
    # beta_t = r_t lambda its minimiser, as eps -> 0, is the shared factor
    V_I, C_I, eps = 0.7, 4.0, 1e-9
    r = RATIOS[mode]
    fac = _factors_after(_oracle(mode), _acc(STATS), V_I, C_I, ears=True)
    for regime in (0, 1):  # 0: RR (second moment), 1: splitting (variance)
        for ch in range(3):
            M = [e2[ch] if regime == 0 else e2[ch] - e1[ch] ** 2 for (_, e1, e2, _) in STATS]
            C = [c for (*_, c) in STATS]

            def cost(lam):
                v = V_I + eps * sum(M[t] / (r[t] * lam) for t in range(3) if r[t] > 0)
                k = C_I + eps * sum(r[t] * C[t] * lam for t in range(3) if r[t] > 0)
                return v * k

            best = minimize_scalar(cost, bounds=(1e-3, 1e3), method="bounded",
                                   options={"xatol": 1e-10})
            assert fac[regime, 0, ch] == pytest.approx(best.x ** 2, rel=2e-3)


def test_ears_equals_mars_for_a_single_technique():
    # plain PT with data for the BSDF technique only: the line is that
    # technique's own axis, so the shared factor is its MARS factor
    stats = [STATS[0], (0, (0, 0, 0), (0, 0, 0), 0.0), (0, (0, 0, 0), (0, 0, 0), 0.0)]
    fe = _factors_after(_oracle(orc.MODE_PT), _acc(stats), 0.4, 2.5, ears=True)
    fm = _factors_after(_oracle(orc.MODE_PT), _acc(stats), 0.4, 2.5, ears=False)
    np.testing.assert_allclose(fe[:, 0], fm[:, 0], rtol=1e-6)


def test_ears_equals_mars_for_identical_techniques():
    # equal ratios and identical statistics for the three techniques: the
    # per-technique optimum already lies on the line
    stats = [STATS[1]] * 3
    fe = _factors_after(_oracle(orc.MODE_BDPT), _acc(stats), 0.9, 3.0, ears=True)
    fm = _factors_after(_oracle(orc.MODE_BDPT), _acc(stats), 0.9, 3.0, ears=False)
    for t in range(3):
        np.testing.assert_allclose(fe[:, 0], fm[:, t], rtol=1e-6)


def test_ears_counts_share_one_factor():
    o = _oracle(orc.MODE_PT_GUIDED)
    T, It = np.array([0.8, 0.5, 0.3], np.float32), np.array([0.4, 0.4, 0.2], np.float32)
    pe = orc.Oracle.params(alloc=orc.ALLOC_EARS)
    pc = orc.Oracle.params(alloc=orc.ALLOC_CLASSIC)
    # no data yet: the classic counts
    assert np.array_equal(o.cell_beta(pe, 0, T, It), o.cell_beta(pc, 0, T, It))
    _factors_after(o, _acc(STATS), 0.7, 4.0, ears=True)
    b = o.cell_beta(pe, 0, T, It)
    # beta_t = r_t lambda, lambda the count the slot-0 factors give (as MARS
    # would give the BSDF technique from the same factors)
    lam = o.cell_beta(orc.Oracle.params(alloc=orc.ALLOC_MARS), 0, T, It)[0]
    assert b[1] == lam and b[0] == np.float32(0.5) * lam and b[2] == np.float32(0.5) * lam


def test_furnace_ears_iterations_unbiased():
    sc = scenegen.make_furnace(32, 32)
    o = orc.Oracle(sc, max_depth=5)
    Ls = []
    for i in range(6):
        p = orc.Oracle.params(iteration=i, spp=4,
                              alloc=orc.ALLOC_CLASSIC if i < 1 else orc.ALLOC_EARS)
        o.render_iteration(p)
        if i >= 1:
            Ls.append(o.sample_radiance()[:, 1].copy())
        o.update(p)
    L = np.concatenate(Ls)
    z = (L.mean() - 1.9375) / (L.std() / math.sqrt(len(L)))
    assert abs(z) < 4.0
    assert o.ncells > 1
