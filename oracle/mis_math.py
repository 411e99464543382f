"""Plain math of the multi-sample allocation model (test infrastructure).

Each function cites the passage of the paper it restates:
  rho / secondary_variance     -- Sec. 3 "Variance model"; supplement A.1 "Variance"
  simplified_variance          -- Sec. 3 "Optimization" (rho ~ max(1, 1/beta) - 1)
  fixed_point_step             -- Sec. 3 "Fixed point" (Eq. optimalBeta), supplement A.3
  lambda_line_optimum          -- supplement A.4 (optimality for budget-unaware weights)
  toy_*                        -- the two-technique 1D example of Fig. 1DSketch / supplement C.1
  study_*                      -- the 1D comparisons of Fig. 1DSketch and supplement C.1 (OS,
                                  RRS, O+R, the proxy fixed point; budget-unaware and -aware
                                  balance heuristic; proxy gradients) and the low-discrepancy
                                  rounding of Alg. 1 against independent rounding
"""
from __future__ import annotations

import numpy as np


def rho(beta):
    """Extra relative variance from stochastic rounding:
    (beta - floor beta)(ceil beta - beta) / beta^2."""
    b = np.asarray(beta, np.float64)
    return (b - np.floor(b)) * (np.ceil(b) - b) / (b * b)


def secondary_variance(beta, mu, var):
    """V[<I; beta>] = V[<I>]/beta + rho(beta) E[<I>]^2."""
    return var / beta + rho(beta) * mu * mu


def simplified_variance(beta, mu, e2):
    """E2/beta - mu^2 if beta <= 1, else (E2 - mu^2)/beta."""
    beta = np.asarray(beta, np.float64)
    return np.where(beta <= 1.0, e2 / beta - mu * mu, (e2 - mu * mu) / beta)


def model_inverse_efficiency(beta, mu, e2, cost, v_delta, c_delta):
    """Inverse efficiency of the proxy model: (sum_t V_t(beta_t) + V_delta) *
    (sum_t beta_t C_t + C_delta)."""
    beta = np.asarray(beta, np.float64)
    V = sum(simplified_variance(beta[..., t], mu[t], e2[t]) for t in range(len(mu))) + v_delta
    Cc = sum(beta[..., t] * cost[t] for t in range(len(mu))) + c_delta
    return V * Cc


def fixed_point_step(beta, mu, e2, cost, v_delta, c_delta):
    """One update beta_t <- sqrt(C/C_t * M_t / V) with M_t = E2_t (RR case,
    result < 1), V_t (splitting case, result > 1), else 1."""
    beta = np.asarray(beta, np.float64)
    V = sum(simplified_variance(beta[t], mu[t], e2[t]) for t in range(len(mu))) + v_delta
    Cc = sum(beta[t] * cost[t] for t in range(len(mu))) + c_delta
    out = np.empty_like(beta)
    for t in range(len(mu)):
        brr = np.sqrt(Cc / cost[t] * e2[t] / V)
        bs = np.sqrt(Cc / cost[t] * (e2[t] - mu[t] ** 2) / V)
        out[t] = brr if brr < 1 else (bs if bs > 1 else 1.0)
    return out


def lambda_line_optimum(mu, e2, cost, v_delta, c_delta, regimes):
    """Closed-form minimiser of the proxy once the regime of every technique
    is fixed ('RR' or 'S'): V = sum M_t/beta_t + V', C = sum beta_t C_t + C_delta
    with M_t = E2_t (RR) or V_t (S) and V' = V_delta - sum_{RR} mu_t^2.  Its
    minimiser is beta_t = lam sqrt(M_t / C_t) with lam = sqrt(C_delta / V')."""
    M = np.array([e2[t] if r == "RR" else e2[t] - mu[t] ** 2 for t, r in enumerate(regimes)])
    vp = v_delta - sum(mu[t] ** 2 for t, r in enumerate(regimes) if r == "RR")
    lam = np.sqrt(c_delta / vp)
    return lam * np.sqrt(M / np.asarray(cost, np.float64))


# ---- the two-technique 1D toy: f(x) = 3x^2 on [0,1] (I = 1), p1 = 1, p2 = 2x,
#      budget-unaware balance heuristic, so <I_t> = f / (p1 + p2) ----
def toy_moments(npts=200):
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    f = 3 * x * x
    p = [np.ones_like(x), 2 * x]
    est = f / (p[0] + p[1])
    mu = np.array([np.sum(w * est * p[t]) for t in range(2)])
    e2 = np.array([np.sum(w * est * est * p[t]) for t in range(2)])
    return mu, e2


# ---- 1D studies (Fig. 1DSketch, supplement C.1): f = 3x^2 on [0, 1], p1 = 1,
#      p2 = 2x (the better match) at 30 times p1's cost; C_delta = V_delta = 1 ----
STUDY_COST = np.array([1.0, 30.0])
STUDY_CD, STUDY_VD = 1.0, 1.0


def _study_quadrature(npts=400):
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    return x, 0.5 * w


_SX, _SW = _study_quadrature()


def study_moments(beta, aware):
    """Mean and second moment of each technique's primary estimate
    w_t f / p_t under x ~ p_t, with the balance heuristic: budget-unaware
    w_t = p_t / sum_k p_k, budget-aware w_t = beta_t p_t / sum_k beta_k p_k."""
    b = np.asarray(beta, np.float64)
    f = 3 * _SX * _SX
    p = [np.ones_like(_SX), 2 * _SX]
    den = b[0] * p[0] + b[1] * p[1] if aware else p[0] + p[1]
    mu, e2 = np.zeros(2), np.zeros(2)
    for t in range(2):
        wt = (b[t] if aware else 1.0) * p[t] / den
        est = wt * f / p[t]
        mu[t] = np.sum(_SW * est * p[t])
        e2[t] = np.sum(_SW * est * est * p[t])
    return mu, e2


def study_inverse_efficiency(beta, aware):
    """The model's inverse efficiency with the MIS weights' dependence on
    beta kept (the true model of the comparison)."""
    mu, e2 = study_moments(beta, aware)
    return float(model_inverse_efficiency(np.asarray(beta, np.float64), mu, e2, STUDY_COST,
                                          STUDY_VD, STUDY_CD))


def study_proxy_gradient(beta, aware, h=1e-6):
    """d(inverse efficiency)/d beta with the moments frozen at beta (the
    proxy: the MIS weights' dependence dropped), by central differences."""
    b = np.asarray(beta, np.float64)
    mu, e2 = study_moments(b, aware)
    g = np.zeros(2)
    for t in range(2):
        d = np.zeros(2)
        d[t] = h * b[t]
        g[t] = (model_inverse_efficiency(b + d, mu, e2, STUDY_COST, STUDY_VD, STUDY_CD) -
                model_inverse_efficiency(b - d, mu, e2, STUDY_COST, STUDY_VD, STUDY_CD)) / (2 * d[t])
    return g


def study_true_gradient(beta, aware, h=1e-6):
    b = np.asarray(beta, np.float64)
    g = np.zeros(2)
    for t in range(2):
        d = np.zeros(2)
        d[t] = h * b[t]
        g[t] = (study_inverse_efficiency(b + d, aware) -
                study_inverse_efficiency(b - d, aware)) / (2 * d[t])
    return g


def study_fixed_point(aware, iters=400):
    """The proxy's fixed point (Eq. optimalBeta iterated), moments re-evaluated
    at every step; a technique whose count reaches 0 stays off."""
    b = np.array([1.0, 1.0])
    for _ in range(iters):
        mu, e2 = study_moments(b, aware)
        with np.errstate(invalid="ignore", divide="ignore"):
            nb = fixed_point_step(b, mu, e2, STUDY_COST, STUDY_VD, STUDY_CD)
        b = np.where(np.isfinite(nb), nb, 0.0)
        b = np.maximum(b, 1e-300)
    return b


def study_line_optimum(ratio, aware):
    """Counts lam * ratio with lam minimising the inverse efficiency (optimal
    RR and splitting of a fixed mixture, as RRS does)."""
    from scipy.optimize import minimize_scalar
    r = np.asarray(ratio, np.float64)
    res = minimize_scalar(lambda ll: study_inverse_efficiency(np.exp(ll) * r, aware),
                          bounds=(-12.0, 12.0), method="bounded", options={"xatol": 1e-10})
    return np.exp(res.x) * r


def study_os_ratio(aware):
    """Optimal mixture sampling (OS): the split (a, 1 - a) of one sample that
    minimises the variance alone."""
    from scipy.optimize import minimize_scalar

    def var(a):
        b = np.array([a, 1.0 - a])
        mu, e2 = study_moments(b, aware)
        return float(sum(simplified_variance(b[t], mu[t], e2[t]) for t in range(2)))
    a = minimize_scalar(var, bounds=(1e-4, 1.0 - 1e-4), method="bounded").x
    return np.array([a, 1.0 - a])


def study_brute_force_optimum(aware, n=120):
    """The true model's minimiser: a log grid, then Nelder-Mead from its best point."""
    from scipy.optimize import minimize
    g = np.exp(np.linspace(np.log(1e-3), np.log(1e2), n))
    best = min((study_inverse_efficiency([b1, b2], aware), b1, b2) for b1 in g for b2 in g)
    r = minimize(lambda lb: study_inverse_efficiency(np.exp(lb), aware),
                 np.log([best[1], best[2]]), method="Nelder-Mead",
                 options={"xatol": 1e-10, "fatol": 1e-15, "maxiter": 5000})
    return np.exp(r.x)


def rounding_noise_variance(beta, c, independent, n_u=20000):
    """Var[sum_t c_t gamma_t] of the rounded counts gamma (each with mean
    beta_t): independent stochastic rounding per technique, or Alg. 1 (one
    uniform u for all techniques, its fractional carry passed on), the
    latter integrated over u on a midpoint grid."""
    b = np.asarray(beta, np.float64)
    c = np.asarray(c, np.float64)
    if independent:
        fr = b - np.floor(b)
        return float(np.sum(c * c * fr * (1.0 - fr)))
    u = (np.arange(n_u) + 0.5) / n_u
    r = u.copy()
    s = np.zeros_like(u)
    for t in range(len(b)):
        g = np.floor(b[t] + r)
        s += c[t] * g
        r = r + b[t] - g
    return float(s.var())


# ---- rounding variants (supplement "Rounding": Fig. rounding) ----
# A secondary estimator of one technique, built from a primary estimator with
# mean mu and variance V, realises a real count beta by an integer number n
# of samples.  Variants:
#   stochastic, real count:    n = floor(beta) + [u < beta - floor(beta)],
#                              estimate (1/beta) sum_n <I>          (the paper's)
#   stochastic, rounded count: the same n, estimate (1/n) sum_n <I> when
#                              beta > 1; (1/beta) sum for RR (beta < 1)
#   nearest:                   n = floor(beta + 1/2) for beta >= 1, estimate
#                              (1/n) sum_n <I>; RR as above for beta < 1
#   simplified model:          the variance the fixed point optimises:
#                              E2/beta - mu^2 for beta <= 1, V/beta above
# Every variant's expected number of samples is its cost in units of one
# sample; n is deterministic for nearest rounding.
def rounding_variant_var_cost(beta, mu, var, variant):
    b = np.asarray(beta, np.float64)
    e2 = var + mu * mu
    rr = e2 / b - mu * mu                      # Russian roulette, any variant
    lo, hi = np.floor(b), np.ceil(b)
    p_hi = b - lo
    if variant == "stochastic":
        v = var / b + rho(b) * mu * mu
        c = b
    elif variant == "rounded":
        inv_n = np.where(hi > lo, p_hi / np.maximum(hi, 1) + (1 - p_hi) / np.maximum(lo, 1), 1 / b)
        v = np.where(b < 1, rr, var * inv_n)
        c = b
    elif variant == "nearest":
        n = np.maximum(np.floor(b + 0.5), 1.0)
        v = np.where(b < 1, rr, var / n)
        c = np.where(b < 1, b, n)
    elif variant == "simplified":
        v = simplified_variance(b, mu, e2)
        c = b
    else:
        raise ValueError(variant)
    return v, c


def rounding_variant_efficiency(beta, mu, var, variant, v_delta=0.0, c_delta=1.0):
    """1 / ((V_delta + V(beta)) (C_delta + cost(beta))): the efficiency of one
    technique's secondary estimator beside a fixed rest of the estimator."""
    v, c = rounding_variant_var_cost(beta, mu, var, variant)
    return 1.0 / ((v_delta + v) * (c_delta + c))


def rounding_variant_mc(beta, sampler, variant, n_trials, rng):
    """Monte Carlo mean and variance of the variant's secondary estimate
    (`sampler(rng, k)` draws k primary estimates) and its mean cost."""
    lo = int(np.floor(beta))
    fr = beta - lo
    if variant == "nearest" and beta >= 1:
        n = np.full(n_trials, int(np.floor(beta + 0.5)))
    else:
        n = lo + (rng.random(n_trials) < fr).astype(np.int64)
    tot = np.zeros(n_trials)
    mx = int(n.max()) if n_trials else 0
    for k in range(mx):
        tot += np.where(n > k, sampler(rng, n_trials), 0.0)
    if variant in ("rounded", "nearest") and beta >= 1:
        est = tot / np.maximum(n, 1)
    else:
        est = tot / beta
    return float(est.mean()), float(est.var()), float(n.mean())
