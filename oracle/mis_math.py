"""Plain math of the multi-sample allocation model (test infrastructure).

Each function cites the passage of the paper it restates:
  rho / secondary_variance     -- Sec. 3 "Variance model"; supplement A.1 "Variance"
  simplified_variance          -- Sec. 3 "Optimization" (rho ~ max(1, 1/beta) - 1)
  fixed_point_step             -- Sec. 3 "Fixed point" (Eq. optimalBeta), supplement A.3
  lambda_line_optimum          -- supplement A.4 (optimality for budget-unaware weights)
  toy_*                        -- the two-technique 1D example of Fig. 1DSketch / supplement C.1
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
