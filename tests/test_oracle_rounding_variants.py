"""The rounding variants of the supplement ("Rounding", Fig. rounding): the
secondary estimator's variance under stochastic rounding normalised by the
real or by the rounded count, under nearest rounding, and the simplified
model, each pinned by Monte Carlo on an exponential primary estimator
(mean 1, variance 1) or a scaled one; then the figure caption's statements,
checked on the efficiency of one technique beside a fixed rest of the
estimator (cost 1, variance V_delta)."""
import numpy as np
import pytest

from oracle import mis_math as mm


@pytest.mark.parametrize("variant", ["stochastic", "rounded", "nearest"])
@pytest.mark.parametrize("beta", [0.35, 1.0, 1.4, 2.5, 3.7])
def test_variant_variance_matches_monte_carlo(variant, beta):
    rng = np.random.default_rng(int(beta * 100) + len(variant))
    mu, var = 1.0, 1.0
    m, v, c = mm.rounding_variant_mc(beta, lambda r, k: r.exponential(1.0, k), variant,
                                     1_000_000, rng)
    vf, cf = mm.rounding_variant_var_cost(beta, mu, var, variant)
    assert abs(m - mu) < 5 * np.sqrt(vf / 1_000_000)          # unbiased
    assert abs(v / vf - 1) < 0.02, (v, vf)
    assert abs(c - cf) < 0.01


def test_all_variants_agree_for_rr_and_integer_counts():
    mu, var = 1.0, 0.7
    for beta in (0.2, 0.5, 0.9, 1.0, 2.0, 3.0, 5.0):
        vals = [mm.rounding_variant_efficiency(beta, mu, var, v, 0.3)
                for v in ("stochastic", "rounded", "nearest", "simplified")]
        assert max(vals) - min(vals) < 1e-9 * max(vals), (beta, vals)


def _best(variant, mu, var, vd):
    b = np.exp(np.linspace(np.log(0.05), np.log(20.0), 20001))
    e = mm.rounding_variant_efficiency(b, mu, var, variant, vd)
    return float(e.max()), float(b[np.argmax(e)])


def test_caption_low_variance_stochastic_worse_than_nearest():
    """(a) low variance: stochastic rounding adds more noise than nearest
    rounding at every non-integer count, and its best efficiency is below
    nearest rounding's."""
    mu, var, vd = 1.0, 0.01, 0.002
    b = np.linspace(1.05, 4.95, 200)
    b = b[np.abs(b - np.round(b)) > 0.05]
    vs, _ = mm.rounding_variant_var_cost(b, mu, var, "stochastic")
    vn, _ = mm.rounding_variant_var_cost(b, mu, var, "nearest")
    assert np.all(vs > vn)
    assert _best("stochastic", mu, var, vd)[0] < _best("nearest", mu, var, vd)[0]


def test_caption_rounding_noise_fades_with_variance():
    """(b) the figure's middle panel is not in the text; what the model gives:
    stochastic rounding's efficiency relative to nearest rounding, averaged
    over non-integer counts in (1, 5), rises with the primary estimator's
    variance and passes nearest rounding once the variance is several times
    the squared mean.  Normalising by the rounded count removes the rounding
    noise of the mean (far better at low variance) and costs a Jensen gap
    E[1/n] > 1/beta (about 2% worse at high variance)."""
    b = np.linspace(1.0, 5.0, 4001)
    b = b[np.abs(b - np.round(b)) > 1e-6]
    ratios, rounded = [], []
    for var in (0.01, 0.1, 1.0, 10.0, 100.0):
        vd = 0.2 * var
        es = mm.rounding_variant_efficiency(b, 1.0, var, "stochastic", vd)
        en = mm.rounding_variant_efficiency(b, 1.0, var, "nearest", vd)
        er = mm.rounding_variant_efficiency(b, 1.0, var, "rounded", vd)
        ratios.append(float(np.mean(es / en)))
        rounded.append(float(np.mean(es / er)))
    assert all(x < y for x, y in zip(ratios, ratios[1:])), ratios
    assert ratios[0] < 0.5 and ratios[-1] > 1.0, ratios
    assert rounded[0] < 0.5 and 1.0 < rounded[-1] < 1.03, rounded


def test_caption_high_variance_stochastic_matches_simplified():
    """(c) high variance: stochastic rounding and the simplified model agree
    (the rounding term rho mu^2 is small against V / beta)."""
    mu, var, vd = 1.0, 100.0, 20.0
    b = np.exp(np.linspace(np.log(1.0), np.log(20.0), 500))
    es = mm.rounding_variant_efficiency(b, mu, var, "stochastic", vd)
    e0 = mm.rounding_variant_efficiency(b, mu, var, "simplified", vd)
    assert np.max(np.abs(es / e0 - 1)) < 0.01
    # and the two unbiased normalisations perform alike at their optima
    assert abs(_best("rounded", mu, var, vd)[0] / _best("stochastic", mu, var, vd)[0] - 1) < 0.02
