"""Pins of the oracle's building blocks against what the paper and the
mathematics fix (closed forms, invariants, brute force, quadrature)."""
import math

import numpy as np
import pytest

from oracle import mis_math as mm
from oracle import oracle as orc

# ---------------------------------------------------------------------------
# Alg. 1 (supplement B.1): enumerating every u on a uniform grid gives
# E[gamma_t] = beta_t exactly up to the grid resolution, the total count is
# floor(sum beta) or one more, and the running remainder stays in [0, 1).
# ---------------------------------------------------------------------------
BETAS = [(0.3, 1.0, 0.0), (0.05, 20.0, 0.05), (2.7, 0.45, 7.25), (1.0, 1.0, 1.0), (0.5, 1.0, 0.5),
         (13.33, 0.999, 3.0001)]


@pytest.mark.parametrize("beta", BETAS)
def test_alg1_expectation_exhaustive(beta):
    n = 1 << 20
    mean, tot, r = orc.alg1_enumerate(beta, n)
    b = np.asarray(beta, np.float32).astype(np.float64)
    assert np.all(np.abs(mean - b) <= 4.0 / n + 1e-6), (mean, b)
    s = math.floor(float(np.sum(b)))
    assert tot[0] >= s and tot[1] <= s + 1
    assert r[0] >= 0.0 and r[1] < 1.0


def test_alg1_single_uniform_decides_all():
    # with beta = (0.5, 1, 0.5) exactly one of the two fractional techniques is taken
    for u in np.linspace(0, 1, 1001, endpoint=False):
        g = orc.alg1([0.5, 1.0, 0.5], u)
        assert g[1] == 1 and g[0] + g[2] == 1


# ---------------------------------------------------------------------------
# Variance of the secondary estimator with stochastic rounding
# (Sec. 3 "Variance model"): V/beta + rho(beta) mu^2, checked by Monte Carlo
# with an Exponential(1) primary estimator (mu = V = 1).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta", [0.3, 1.0, 1.5, 2.7, 7.25])
def test_rho_variance_model(beta):
    rng = np.random.default_rng(12345)
    n = 4_000_000
    fl = math.floor(beta)
    k = fl + (rng.random(n) < beta - fl)
    sums = np.where(k > 0, rng.gamma(np.maximum(k, 1), 1.0), 0.0)
    est = sums / beta
    v_mc = est.var()
    v_model = mm.secondary_variance(beta, 1.0, 1.0)
    assert abs(est.mean() - 1.0) < 5 * math.sqrt(v_model / n)
    assert abs(v_mc / v_model - 1.0) < 0.01, (v_mc, v_model)


def test_simplified_rho_only_changes_splitting():
    # max(1, 1/beta) - 1 equals rho for beta <= 1 and drops it for beta > 1
    mu, e2 = 0.7, 1.3
    for b in [0.1, 0.5, 1.0]:
        exact = mm.secondary_variance(b, mu, e2 - mu * mu)
        assert abs(mm.simplified_variance(b, mu, e2) - exact) < 1e-12
    for b in [1.5, 3.7]:
        assert abs(mm.simplified_variance(b, mu, e2) - (e2 - mu * mu) / b) < 1e-12


# ---------------------------------------------------------------------------
# Two-technique toy (Fig. 1DSketch, supplement A.4/C.1): the fixed point of
# the update equals the closed-form minimiser on the lambda line, which also
# equals a brute-force grid minimum; the oracle's own cell update + count
# resolution (C code) reproduces the iteration.
# ---------------------------------------------------------------------------
TOY_CASES = [
    # cost, C_delta, V_delta, regimes, expected optimum
    ((1.0, 30.0), 1.0, 1.0, ("RR", "RR"), (0.7382496, 0.1699712)),
    ((1.0, 30.0), 100.0, 0.01, ("S", "S"), (30.713837, 4.971772)),
]


def test_toy_moments_exact():
    mu, e2 = mm.toy_moments()
    assert abs(mu.sum() - 1.0) < 1e-12          # sum_t E<I_t> = I (partition of unity)
    np.testing.assert_allclose(mu, [0.4119796, 0.5880204], rtol=1e-6)
    np.testing.assert_allclose(e2, [0.2640612, 0.4199235], rtol=1e-6)


@pytest.mark.parametrize("cost,cd,vd,regimes,expected", TOY_CASES)
def test_toy_closed_form_and_brute_force(cost, cd, vd, regimes, expected):
    mu, e2 = mm.toy_moments()
    opt = mm.lambda_line_optimum(mu, e2, cost, vd, cd, regimes)
    np.testing.assert_allclose(opt, expected, rtol=1e-6)
    # brute force over a log grid
    g1 = np.exp(np.linspace(np.log(1e-3), np.log(50.0), 2001))
    g2 = np.exp(np.linspace(np.log(1e-3), np.log(50.0), 501))
    B = np.stack(np.meshgrid(g1, g2, indexing="ij"), -1)
    ie = mm.model_inverse_efficiency(B, mu, e2, cost, vd, cd)
    i, j = np.unravel_index(np.argmin(ie), ie.shape)
    ie_opt = mm.model_inverse_efficiency(np.asarray(opt), mu, e2, cost, vd, cd)
    assert ie.min() >= ie_opt * (1 - 1e-9)
    assert abs(g1[i] / opt[0] - 1) < 0.01 and abs(g2[j] / opt[1] - 1) < 0.03


def _toy_oracle():
    import scenegen
    return orc.Oracle(scenegen.make_cornell(8, 8), max_depth=2)


@pytest.mark.parametrize("cost,cd,vd,regimes,expected", TOY_CASES)
def test_toy_fixed_point_through_oracle_update(cost, cd, vd, regimes, expected):
    """Runs the fixed-point iteration with exact moments through the oracle's
    C update (orc_update_cells_only) and count resolution (orc_cell_beta)."""
    mu, e2 = mm.toy_moments()
    o = _toy_oracle()
    p = orc.Oracle.params(alloc=orc.ALLOC_MARS, clamp_lo=1e-6, clamp_hi=1e6)
    beta = np.array([1.0, 1.0])
    ie_opt = mm.model_inverse_efficiency(np.asarray(expected), mu, e2, cost, vd, cd)
    hist = []
    for it in range(200):
        V = sum(mm.simplified_variance(beta[t], mu[t], e2[t]) for t in range(2)) + vd
        Cc = float(np.dot(beta, cost)) + cd
        acc = np.zeros((o.ncells, 3, 8))
        for t in range(2):
            acc[0, t, 0:3] = mu[t]
            acc[0, t, 3:6] = e2[t]
            acc[0, t, 6] = 1.0
            acc[0, t, 7] = cost[t]
        o.write_cells(acc=acc)
        assert o.update_cells_only(V, Cc) == 1
        b = o.cell_beta(p, 0, [1, 1, 1], [1, 1, 1])
        beta = b[:2].astype(np.float64)
        hist.append(mm.model_inverse_efficiency(beta, mu, e2, cost, vd, cd))
    np.testing.assert_allclose(beta, expected, rtol=1e-5)
    # "close to the optimum after about five iterations" (Fig. 1DConvergence)
    assert hist[5] / ie_opt < 1.02


# ---------------------------------------------------------------------------
# MIS partition of unity (supplement A.1): sum_t w_it = 1 for the direct
# subintegrand over {B,N,G} and the indirect one over {B,G}.
# ---------------------------------------------------------------------------
def test_mis_partition_of_unity():
    rng = np.random.default_rng(7)
    for aware in (0, 1):
        for _ in range(2000):
            beta = rng.uniform(0.05, 20, 3).astype(np.float32)
            beta[rng.random(3) < 0.2] = 0.0
            beta[0] = max(beta[0], 0.05)
            p = np.exp(rng.uniform(-8, 8, 3)).astype(np.float32)
            wd, wi = orc.mis(aware, beta, p)
            assert abs(wd.sum() - 1) < 1e-6
            assert abs(wi[0] + wi[2] - 1) < 1e-6
            assert np.all(wd[beta == 0] == 0)


# ---------------------------------------------------------------------------
# sin/cos of 2 pi u, Philox statistics
# ---------------------------------------------------------------------------
def test_sincos2pi_accuracy():
    us = np.concatenate([np.arange(0, 1 << 24, 4099), [0, 1 << 22, 1 << 23, 3 << 22,
                                                       (1 << 24) - 1]]) / float(1 << 24)
    err = 0.0
    for u in us:
        s, c = orc.sincos2pi(u)
        err = max(err, abs(s - math.sin(2 * math.pi * u)), abs(c - math.cos(2 * math.pi * u)))
    assert err < 3e-7
    assert orc.sincos2pi(0.0) == (0.0, 1.0)
    assert orc.sincos2pi(0.25) == (1.0, -0.0) or orc.sincos2pi(0.25) == (1.0, 0.0)


def test_philox_uniformity_and_avalanche():
    rng = np.random.default_rng(3)
    outs = np.array([orc.philox((1, 0), (i, 7, 3, 0x44000000)) for i in range(20000)])
    u = (outs >> 8).astype(np.float64) / (1 << 24)
    hist, _ = np.histogram(u.ravel(), bins=64, range=(0, 1))
    exp = u.size / 64
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof, p ~ 1e-5
    # one flipped counter bit changes about half of the 128 output bits
    flips = []
    for _ in range(300):
        c = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        a = orc.philox((5, 9), c)
        c2 = c.copy()
        c2[rng.integers(0, 4)] ^= np.uint32(1 << int(rng.integers(0, 32)))
        b = orc.philox((5, 9), c2)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert 60 < np.mean(flips) < 68


# ---------------------------------------------------------------------------
# BSDF pins: pdf normalisation, sampling density, and E[f cos / p] = integral
# of f cos by quadrature (Lambert: albedo exactly).
# ---------------------------------------------------------------------------
def _hemisphere_grid(n_th=180, n_ph=360):
    th = (np.arange(n_th) + 0.5) * (math.pi / 2) / n_th
    ph = (np.arange(n_ph) + 0.5) * 2 * math.pi / n_ph
    T, P = np.meshgrid(th, ph, indexing="ij")
    dw = np.sin(T) * (math.pi / 2 / n_th) * (2 * math.pi / n_ph)
    d = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    return d.reshape(-1, 3), dw.ravel()


MATS = [
    [0, 0.7, 0.5, 0.3, 0.0, 0, 0, 0],
    [1, 0.9, 0.6, 0.3, 0.5, 0, 0, 0],
    [1, 0.4, 0.4, 0.4, 0.2, 0, 0, 0],
]


@pytest.mark.parametrize("mat", MATS)
def test_bsdf_pdf_and_albedo_quadrature(mat):
    n = np.array([0.0, 0.0, 1.0], np.float32)
    wo = np.array([0.3, -0.2, 0.9], np.float32)
    wo /= np.linalg.norm(wo)
    dirs, dw = _hemisphere_grid(120, 240)
    pdf_int = 0.0
    fint = np.zeros(3)
    for d, w in zip(dirs, dw):
        f, pdf = orc.bsdf_eval(mat, n, wo, d.astype(np.float32))
        pdf_int += pdf * w
        fint += f * w
    rng = np.random.default_rng(11)
    est = np.zeros(3)
    m = 40000
    lost = 0
    for _ in range(m):
        ok, wi = orc.bsdf_sample(mat, n, wo, *rng.random(2))
        if not ok:
            lost += 1
            continue
        f, pdf = orc.bsdf_eval(mat, n, wo, wi)
        est += f / pdf
    est /= m
    if mat[0] == 0:
        assert abs(pdf_int - 1) < 2e-3
        np.testing.assert_allclose(fint, mat[1:4], rtol=2e-3)
        np.testing.assert_allclose(est, mat[1:4], rtol=1e-5)
    else:
        # sampled reflections that leave the hemisphere carry the missing pdf mass
        assert abs(pdf_int - (1 - lost / m)) < 0.02
        np.testing.assert_allclose(est, fint, rtol=0.03)


def test_bsdf_sampling_matches_pdf_histogram():
    mat = MATS[1]
    n = np.array([0.0, 0.0, 1.0], np.float32)
    wo = np.array([0.0, 0.6, 0.8], np.float32)
    rng = np.random.default_rng(5)
    zs = []
    for _ in range(30000):
        ok, wi = orc.bsdf_sample(mat, n, wo, *rng.random(2))
        if ok:
            zs.append(wi[2])
    hist, edges = np.histogram(zs, bins=10, range=(0, 1))
    dirs, dw = _hemisphere_grid(200, 200)
    pdfs = np.array([orc.bsdf_eval(mat, n, wo, d.astype(np.float32))[1] for d in dirs])
    expct = np.array([np.sum((pdfs * dw)[(dirs[:, 2] >= a) & (dirs[:, 2] < b)])
                      for a, b in zip(edges[:-1], edges[1:])]) * 30000
    mask = expct > 50
    chi = ((hist[mask] - expct[mask]) ** 2 / expct[mask]).sum()
    assert chi < 3 * mask.sum() + 30, (hist, expct)


def test_guided_histogram_pdf_and_sampling():
    rng = np.random.default_rng(2)
    w = rng.random(64) ** 3
    pm = (0.9 * w / w.sum() + 0.1 / 64).astype(np.float32)
    cdf = np.cumsum(pm.astype(np.float64)).astype(np.float32)
    cdf[-1] = 1.0
    # pdf integrates to one over the sphere
    n_t, n_p = 400, 800
    z = -1 + (np.arange(n_t) + 0.5) * 2 / n_t
    ph = (np.arange(n_p) + 0.5) * 2 * math.pi / n_p
    Z, P = np.meshgrid(z, ph, indexing="ij")
    s = np.sqrt(1 - Z * Z)
    D = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3).astype(np.float32)
    tot = sum(orc.guided_pdf(pm, d) for d in D[::7]) * (4 * math.pi / (n_t * n_p)) * 7
    assert abs(tot - 1.0) < 0.01
    # sampled bins follow pm, and every sample's pdf is its bin's pm * 16/pi
    counts = np.zeros(64)
    m = 40000
    for _ in range(m):
        d = orc.guided_sample(pm, cdf, *rng.random(3))
        zz = min(7, int((d[2] + 1) * 4))
        phi = math.atan2(d[1], d[0]) % (2 * math.pi)
        counts[zz * 8 + min(7, int(phi / (2 * math.pi) * 8))] += 1
    exp = pm * m
    chi = ((counts - exp) ** 2 / exp).sum()
    assert chi < 140
