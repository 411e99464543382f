"""Per-iteration log as JSON lines: one object per render iteration with its
update, for convergence and throughput tracking (Sec. 4.1, image estimates:
the image's cost is the number of rays traced, C_I, and the allocation's
quality is read as 1/(V_I C_I)).

Fields: iteration, alloc, spp, seconds (render + update, host wall clock),
rays by kind and in total, Mrays/s and Mpaths/s over those seconds, V_I, C_I
and 1/(V_I C_I) of the update, the tiles and overflow re-runs of the render,
and, when a count map is given, the mean count per technique at the first
hit over the image (BSDF, NEE, third technique)."""
from __future__ import annotations

import json
import math

RAY_KINDS = ("rays_camera", "rays_ext", "rays_shadow", "rays_light", "rays_conn")


def record(iteration, params, it_stats, up_stats, seconds, width, height, count_map=None):
    """One log object.  it_stats / up_stats: the render's and the update's
    statistics (attributes as in mars_iter_stats / mars_update_stats);
    count_map: the per-pixel first-hit counts [H][W][3] or None."""
    rays = {k: int(getattr(it_stats, k)) for k in RAY_KINDS}
    total = sum(rays.values())
    spp = int(params.spp)
    paths = width * height * spp
    v, c = float(up_stats.V_I), float(up_stats.C_I)
    out = {"iteration": int(iteration), "alloc": int(params.alloc), "spp": spp,
           "seconds": float(seconds), **rays, "rays": total,
           "mrays_per_s": total / seconds / 1e6 if seconds > 0 else None,
           "mpaths_per_s": paths / seconds / 1e6 if seconds > 0 else None,
           "V_I": v, "C_I": c,
           "proxy_efficiency": 1.0 / (v * c) if v > 0 and c > 0 and math.isfinite(v * c) else None,
           "tiles": int(it_stats.tiles), "overflow_retries": int(it_stats.overflow_retries)}
    if count_map is not None:
        flat = count_map.reshape(-1, count_map.shape[-1])
        out["mean_first_hit_counts"] = [float(x) for x in flat.mean(axis=0)]
    return out


class IterationLog:
    """Appends one JSON line per iteration to `path`."""

    def __init__(self, path):
        self.f = open(path, "a")

    def write(self, obj):
        self.f.write(json.dumps(obj) + "\n")
        self.f.flush()

    def close(self):
        if self.f:
            self.f.close()
            self.f = None
