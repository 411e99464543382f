"""The 1D studies behind the proxy model (Fig. 1DSketch; supplement C.1 and
the rounding section): a single integrand estimated by two techniques, the
better-matching one 30 times as expensive, with C_delta = V_delta = 1.
Optimal mixture sampling (OS), optimal RR and splitting of a fixed mixture
(RRS), the two combined (O+R) and the proxy fixed point ("ours") are compared
on the model's true inverse efficiency, for budget-unaware and budget-aware
balance heuristics, and Alg. 1's single-uniform rounding against independent
rounding."""
import numpy as np
import pytest

from oracle import mis_math as mm


def _eff(beta, aware):
    return 1.0 / mm.study_inverse_efficiency(beta, aware)


def test_proxy_is_exact_for_budget_unaware_weights():
    # weights independent of the counts: the proxy drops nothing, so its
    # fixed point is the true optimum and its gradient the true gradient
    ours = mm.study_fixed_point(aware=False)
    best = mm.study_brute_force_optimum(aware=False)
    np.testing.assert_allclose(ours, best, rtol=1e-4)
    assert _eff(ours, False) == pytest.approx(_eff(best, False), rel=1e-8)
    for b in ([0.1, 0.1], [0.5, 3.0], [4.0, 0.2], [12.0, 7.0]):
        gt, gp = mm.study_true_gradient(b, False), mm.study_proxy_gradient(b, False)
        np.testing.assert_allclose(gp, gt, rtol=1e-5, atol=1e-9)


def test_ours_beats_os_rrs_and_their_combination():
    aware = False
    ours = _eff(mm.study_fixed_point(aware), aware)
    a = mm.study_os_ratio(aware)
    e_os = _eff(a, aware)
    e_rrs = _eff(mm.study_line_optimum([0.5, 0.5], aware), aware)
    e_or = _eff(mm.study_line_optimum(a, aware), aware)
    # OS then RRS improves on OS alone (OS is one point of O+R's line) but,
    # optimising ratio and total apart, stays clearly below the joint optimum
    assert e_or >= e_os
    assert ours > 1.2 * max(e_os, e_rrs, e_or)


def test_budget_aware_proxy_near_the_true_optimum():
    aware = True
    ours = mm.study_fixed_point(aware)
    best = mm.study_brute_force_optimum(aware)
    assert _eff(ours, aware) >= 0.99 * _eff(best, aware)
    # budget-aware weights do better than the best budget-unaware allocation
    assert _eff(best, aware) > _eff(mm.study_brute_force_optimum(False), False)
    # the proxy gradient points like the true one almost everywhere
    g = np.exp(np.linspace(np.log(0.05), np.log(20.0), 24))
    cos = []
    for b1 in g:
        for b2 in g:
            gt = mm.study_true_gradient([b1, b2], aware)
            gp = mm.study_proxy_gradient([b1, b2], aware)
            cos.append(gt @ gp / (np.linalg.norm(gt) * np.linalg.norm(gp)))
    cos = np.array(cos)
    assert np.median(cos) > 0.99 and (cos > 0.9).mean() > 0.85 and (cos > 0).mean() > 0.95
    assert cos.min() < 0.5  # but not everywhere: the proxy is not exact here


def test_low_discrepancy_rounding():
    rng = np.random.default_rng(3)
    for _ in range(200):
        b = rng.uniform(0.0, 4.0, 3)
        # the total count only takes floor or ceil of sum beta: the least
        # variance an integer count with that mean can have
        fr = b.sum() - np.floor(b.sum())
        v_ld = mm.rounding_noise_variance(b, np.ones(3), independent=False)
        v_in = mm.rounding_noise_variance(b, np.ones(3), independent=True)
        assert v_ld == pytest.approx(fr * (1 - fr), abs=1e-3)
        assert v_ld <= v_in + 1e-3
    # in the 1D example at the unaware optimum, the secondary estimator's
    # variance drops with Alg. 1 (rounding noise sum_t c_t gamma_t with
    # c_t = mu_t / beta_t, the rest of the variance unchanged)
    b = mm.study_fixed_point(aware=False)
    mu, e2 = mm.study_moments(b, False)
    c = mu / b
    rest = float(np.sum((e2 - mu * mu) / b)) + mm.STUDY_VD
    v_ld = rest + mm.rounding_noise_variance(b, c, independent=False)
    v_in = rest + mm.rounding_noise_variance(b, c, independent=True)
    assert v_ld < 0.95 * v_in
