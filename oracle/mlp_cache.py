"""Render-side arithmetic of the learned cache -- TEST INFRASTRUCTURE ONLY.

The learned cache (a network in place of the octree's per-cell counts) is
not in the paper; its Sec. 6 ("Discontinuity artefacts") asks for sample
counts that vary smoothly in space, which a network fitted to the octree's
estimates provides.  This module states, plainly and per vertex, what the
renderer computes around the network:

  inputs    q = clamp((x - lo) * inv, 0, 1 - 2^-24) (the octree's cube
            normalisation of the vertex position) and the stored geometric
            normal n; the network then sees sin / cos(2^k pi .) of these
            (oracle/mlp_ref.py);
  target    y*_t = log(beta^_t) - log|T / I~| for every technique t the
            scene has, where beta^_t is the octree's resolved, unclamped count
            of the vertex from its cell's factors after the update (the
            fixed point of Sec. 3.1 with the colour rule of Sec. 4.1), and
            |T / I~| = sqrt((1/3) sum_ch (T_ch / I~_ch)^2); weight
            min(n_t, 64) / 64 if the cell drew at least 4 samples of t in the
            iteration, else 0 (target 0);
  count     the network's count |T / I~| exp(y_t) pooled with the octree's
            count beta_t as their geometric mean sqrt(beta_t |T/I~| exp(y_t)),
            clamped to [lo, hi]; the octree's count where that is not finite;
            a technique the octree gives no samples keeps none.

Decisions (which resolve case, whether a weight is zero) are taken in
binary32 with the renderer's operation order, as the renderer takes them;
values (logarithms, the geometric mean) are computed in binary64.
"""
from __future__ import annotations

import numpy as np

F = np.float32
ONE_MINUS = F(1.0) - F(2.0 ** -24)


def octree_box(V):
    """The octree's root cube: the scene's bounding box widened to a cube of
    its largest extent, padded by 2e-4 relative, computed in binary64 and
    stored as binary32 (corner, reciprocal side)."""
    V = np.asarray(V, np.float64).reshape(-1, 3)
    lo, hi = V.min(0), V.max(0)
    side = (hi - lo).max() * (1 + 2e-4)
    return ((lo + hi) * 0.5 - 0.5 * side).astype(F), F(1.0 / side)


def inputs(P, n, oct_lo, oct_inv):
    """P [N,3], n [N,3] (binary32) -> x6 [N,6]: the network's inputs."""
    P = np.asarray(P, F)
    q = (P - np.asarray(oct_lo, F)) * F(oct_inv)
    q = np.minimum(np.maximum(q, F(0.0)), ONE_MINUS)
    return np.concatenate([q, np.asarray(n, F)], 1).astype(F)


def t_over_i(T, It):
    """|T / I~|: the colour rule's norm of the relative throughput, binary32."""
    z = np.asarray(T, F) / np.asarray(It, F)
    s = (z[:, 0] * z[:, 0] + z[:, 1] * z[:, 1]) + z[:, 2] * z[:, 2]
    return np.sqrt(s * F(1.0 / 3.0)).astype(F), z


def octree_count_unclamped(fac, z):
    """Resolved count of the Sec. 3.1 fixed point for one technique:
    fac [N,2,3] (RR / S factor per channel), z [N,3] = T / I~ -> beta^ [N]
    (binary32, no clamp); NaN where the cell has no factors (fac < 0)."""
    fac = np.asarray(fac, F)
    zz = z * z
    with np.errstate(invalid="ignore"):
        return _resolve(fac, zz)


def _resolve(fac, zz):
    sr = (zz[:, 0] * fac[:, 0, 0] + zz[:, 1] * fac[:, 0, 1]) + zz[:, 2] * fac[:, 0, 2]
    ss = (zz[:, 0] * fac[:, 1, 0] + zz[:, 1] * fac[:, 1, 1]) + zz[:, 2] * fac[:, 1, 2]
    b_rr = np.sqrt(sr * F(1.0 / 3.0))
    b_s = np.sqrt(ss * F(1.0 / 3.0))
    b = np.where(b_rr < F(1.0), b_rr, np.where(b_s > F(1.0), b_s, F(1.0))).astype(F)
    return np.where(fac[:, 0, 0] < F(0.0), F(np.nan), b)


def targets(cell, T, It, factors, counts, enabled):
    """Training targets and weights of recorded vertices.

    cell [N] leaf of each vertex; T [N,3] prefix throughput; It [N,3] the
    pixel estimate; factors [cells,2,3,3] (RR / S, technique, channel);
    counts [cells,3] samples per technique in the iteration; enabled [3].
    Returns y [N,3] (binary64) and w [N,3] (binary32)."""
    cell = np.asarray(cell, np.int64)
    sm, z = t_over_i(T, It)
    y = np.zeros((len(cell), 3))
    w = np.zeros((len(cell), 3), F)
    for t in range(3):
        if not enabled[t]:
            continue
        fac = np.asarray(factors, F)[cell][:, :, t, :]        # [N,2,3]
        bh = octree_count_unclamped(fac, z)
        n = np.asarray(counts, np.float64)[cell, t]
        ok = (n >= 4.0) & (sm > F(0.0)) & np.isfinite(bh) & (bh > F(0.0))
        with np.errstate(divide="ignore", invalid="ignore"):
            yt = np.log(bh.astype(np.float64)) - np.log(sm.astype(np.float64))
        ok &= np.isfinite(yt)
        y[ok, t] = yt[ok]
        w[ok, t] = (np.minimum(n[ok], 64.0) / 64.0).astype(F)
    return y, w


def pooled_count(beta_oct, y, T, It, clamp_lo, clamp_hi):
    """Counts of a learned-cache iteration: beta_oct [N,3] the octree's
    clamped counts of the vertices, y [N,3] the network's outputs."""
    sm, _ = t_over_i(T, It)
    b_oct = np.asarray(beta_oct, np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        g = np.sqrt(b_oct * sm.astype(np.float64)[:, None] * np.exp(np.asarray(y, np.float64)))
    out = b_oct.copy()
    ok = (b_oct > 0.0) & np.isfinite(g)
    out[ok] = np.minimum(np.maximum(g[ok], clamp_lo), clamp_hi)
    return out
