#!/usr/bin/env python
"""Benchmark of the MARS hot path on one MI355X.

Default workload (the metric's configuration): the learned cache against the
plain octree, bidirectional MARS at 1920 x 1080 on a seeded procedural
interior of 2.08M triangles (4500 instanced furniture pieces, one small
emitter hidden behind an occluder), max path length 12.  One step = one
learned-cache MARS iteration at 2 samples per pixel: light subpaths, camera
paths with per-vertex counts from the network pooled with the octree, all
connections and shadow rays, back-propagation, cell statistics, the update
(image estimates, fixed point, targets, refinement) and 32 Adam steps of
the network.  The schedule: 3 classic-RR iterations, 2 octree MARS
iterations (the network trains from the first of them), then learned-cache
iterations; the default warm-up (10) ends after 5 of those, so that the
timed steps see a network past its first updates.  Beside the
throughput: the efficiency 1/(relMSE s) of both methods at equal relMSE
over the paper's growing-iteration schedule, the traversal kernel's
roofline, and the CPU oracle's throughput on the same scene.

Other workloads (--workload): guided (512 x 512 guided PT), bdpt
(1280 x 720 bidirectional), batch (32 scenes), ears (MARS vs EARS vs
classic RR), convergence, rounding (Alg. 1 against independent rounding)
and lp_lengths (separate light-path budgets per light-vertex index against
one budget).  Prints one JSON line.  --gpus above 1 is not supported (one
GPU per box).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2410_20429_amd import iterlog  # noqa: E402  (host-side JSON lines, no GPU)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "guided_pt_512x512_heightfield132k_d10"
BYTES_RAY_IO = 48.0      # ray 32 B in (origin, direction) + hit 16 B out
BYTES_SHADOW_IO = 36.0   # shadow ray 32 B in (origin + tmax, direction) + 4 B visibility out
BYTES_NODE = 128.0       # one 4-wide BVH node (four child boxes + references)
BYTES_TRI = 48.0         # one triangle record (v0, e1, e2)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_math.hpp", "mars_internal.h"):
        with open(os.path.join(ROOT, "paper_2410_20429_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name, window):
    """Measured HBM bytes per launch of the traversal kernel from the
    committed rocprofv3 counter summary profiles/<name>, if it was taken on
    the current kernel source and over the same window (workload, warm-up and
    timed steps) as this run; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash() or t.get("window") != window:
        return None
    return t


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def roofline(api, ctx, prof, step_counted, rays_closest, rays_shadow, traffic_name, window):
    """The traversal kernel against the HBM roofline.  achieved = algorithmic
    bytes per launch (per ray: I/O plus one 128 B node per visited node and
    48 B per tested triangle, node and triangle counts from one instrumented
    iteration) / the average launch time of the timed steps (HIP events the
    dispatch stamps).  traffic = measured HBM bytes per launch (rocprofv3
    FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy) over the same
    window, when a summary of it is committed; measured_hbm_frac follows
    from it."""
    ctx.trace_counting(True)
    step_counted()
    tc = ctx.trace_counts()
    ctx.trace_counting(False)
    bpr_c = BYTES_RAY_IO + (BYTES_NODE * tc[1] + BYTES_TRI * tc[2]) / max(tc[0], 1)
    bpr_s = BYTES_SHADOW_IO + (BYTES_NODE * tc[4] + BYTES_TRI * tc[5]) / max(tc[3], 1)
    ms_tr, n_tr = prof["trace"]
    avg_ms = ms_tr / max(n_tr, 1)
    bytes_per_launch = (bpr_c * rays_closest + bpr_s * rays_shadow) / max(n_tr, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    t = load_traffic(traffic_name, window)
    traffic = t["hbm_bytes_per_launch"] if t else None
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "trace",
           "achieved_is": "algorithmic bytes (every visited node and tested triangle counted "
                          "as fetched) / average launch time",
           "avg_launch_ms": avg_ms, "launches_timed": n_tr,
           "algorithmic_bytes_per_launch": bytes_per_launch,
           "bytes_per_closest_ray": bpr_c, "bytes_per_shadow_ray": bpr_s,
           "nodes_per_closest_ray": tc[1] / max(tc[0], 1),
           "tris_per_closest_ray": tc[2] / max(tc[0], 1),
           "nodes_per_shadow_ray": tc[4] / max(tc[3], 1),
           "max_nodes_closest_ray": tc[6], "max_nodes_shadow_ray": tc[7],
           "rays_over_64_nodes": [tc[8], tc[9]]}
    if t:
        out["measured_hbm_gbs"] = traffic / (avg_ms * 1e-3) / 1e9
        out["measured_hbm_frac"] = out["measured_hbm_gbs"] / HBM_PEAK_GBS
        out["traffic_source"] = "profiles/" + traffic_name
        for k in ("occupancy_waves_per_simd", "occupancy_waves_per_simd_time_weighted", "vgprs",
                  "scratch_bytes"):
            if k in t:
                out[k] = t[k]
    return out


def relmse(img, ref, eps=1e-2, drop=1e-4):
    """relMSE: mean over pixels of the channel-mean (I - R)^2 / (R^2 + eps),
    the largest fraction `drop` of the per-pixel terms discarded."""
    import numpy as np
    d = img.astype(np.float64) - ref
    e = np.sort(np.mean(d * d / (ref * ref + eps), axis=-1).ravel())
    keep = e.size - int(np.floor(drop * e.size))
    return float(np.mean(e[:keep]))


def reference_image(api, ctx, sc, spp=16, iters=256, seed_iter=100000, mode=None, depth=10):
    """Classic-RR rendering at spp x iters samples per pixel (the same
    integrand; independent random streams via the iteration index)."""
    import numpy as np
    mode = api.MODE_PT_GUIDED if mode is None else mode
    r = api.Scene(ctx, sc, mode=mode, max_depth=depth, max_cells=cells_budget())
    acc = np.zeros((sc["height"], sc["width"], 3))
    for i in range(iters):
        r.render_iteration(api.iter_params(iteration=seed_iter + i, spp=spp,
                                           stat_clamp=0.0 if mode == api.MODE_BDPT else 50.0))
        acc += r.image(api.IMAGE_LAST)
    r.release()
    return acc / iters


# queue memory of each method's scene in the efficiency protocols
EFFICIENCY_QUEUE_GIB = 96


def efficiency_leg(api, ctx, sc, torch, n_iter=9, mode=None, depth=10, ref_spp=(16, 256),
                   ears=False, unaware=False, lp_lengths=False):
    """Efficiency 1/(relMSE * seconds) of MARS and of classic RR, as in the
    paper's evaluation: n_iter iterations of 1, 2, 4, ... spp, the first
    three with classic RR, then MARS (render + update each); the MARS image
    is the inverse-variance weighted combination of all iterations; classic
    RR renders the same sample counts (mean image).  Each method's queue and
    tile sizes come from the autotuner before its 4th iteration (outside the
    timed region).  relMSE against a classic reference of ref_spp[0] x
    ref_spp[1] spp, 0.01% brightest outliers discarded.  With ears, EARS (one shared count per vertex, the
    paper's comparison method) runs the same schedule as MARS; with unaware,
    so does MARS with the budget-unaware balance heuristic; with lp_lengths,
    MARS with separate light-path budgets per light-vertex index (y_1, y_2,
    y_3+; bidirectional scenes), with both MIS forms."""
    import numpy as np
    mode = api.MODE_PT_GUIDED if mode is None else mode
    kc = 0.0 if mode == api.MODE_BDPT else 50.0
    ref = reference_image(api, ctx, sc, spp=ref_spp[0], iters=ref_spp[1], mode=mode, depth=depth)

    def run(alloc_after, aware=True, per_length=False):
        s = api.Scene(ctx, sc, mode=mode, max_depth=depth, max_cells=cells_budget(),
                      lp_lengths=per_length)
        acc = np.zeros_like(ref)
        spp_tot = rays = 0
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(n_iter):
            alloc = api.ALLOC_CLASSIC if i < 3 else alloc_after
            p = api.iter_params(iteration=i, spp=1 << i, alloc=alloc, stat_clamp=kc,
                                budget_aware=aware)
            if i == 3:
                # queue and tile sizes for this method's own queue peaks (a
                # MARS iteration draws many more connections than a classic
                # one), outside the timed region
                torch.cuda.synchronize()
                t_pause = time.perf_counter()
                api.autotune([s], p, mem_budget=EFFICIENCY_QUEUE_GIB << 30)
                torch.cuda.empty_cache()
                torch.cuda.synchronize()
                t += time.perf_counter() - t_pause
            rays += s.render_iteration(p).total_rays()
            if alloc_after != api.ALLOC_CLASSIC:
                s.update(p)
            else:
                torch.cuda.synchronize()
                t_pause = time.perf_counter()
                acc += s.image(api.IMAGE_LAST) * (1 << i)
                t += time.perf_counter() - t_pause  # read-back excluded
            spp_tot += 1 << i
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        img = s.image(api.IMAGE_IVW) if alloc_after != api.ALLOC_CLASSIC else acc / spp_tot
        s.release()
        return relmse(img, ref), dt, spp_tot, rays

    e_m, t_m, spp, r_m = run(api.ALLOC_MARS)
    e_c, t_c, _, r_c = run(api.ALLOC_CLASSIC)
    rs = ref_spp[0] * ref_spp[1]
    out = {"definition": "1/(relMSE*s); relMSE = mean (I-R)^2/(R^2+0.01), 0.01% outliers "
                         f"discarded, vs a {rs} spp classic reference; iterations of 1,2,4.. spp",
           "mars": 1.0 / (e_m * t_m), "classic": 1.0 / (e_c * t_c),
           "gain_vs_classic": (e_c * t_c) / (e_m * t_m),
           "relmse_mars": e_m, "relmse_classic": e_c, "seconds_mars": t_m,
           "seconds_classic": t_c, "spp": spp, "iterations": n_iter, "reference_spp": rs,
           "rays_mars": r_m, "rays_classic": r_c,
           "ray_efficiency_gain_vs_classic": (e_c * r_c) / (e_m * r_m)}
    if ears:
        e_e, t_e, _, r_e = run(api.ALLOC_EARS)
        out.update({"ears": 1.0 / (e_e * t_e), "gain_vs_ears": (e_e * t_e) / (e_m * t_m),
                    "relmse_ears": e_e, "seconds_ears": t_e, "rays_ears": r_e,
                    "rays_mars_vs_ears": r_m / r_e - 1.0,
                    "ray_efficiency_gain_vs_ears": (e_e * r_e) / (e_m * r_m)})
    if lp_lengths:
        for aw, tag in ((True, "per_length"), (False, "per_length_budget_unaware")):
            e_l, t_l, _, r_l = run(api.ALLOC_MARS, aware=aw, per_length=True)
            out.update({tag: 1.0 / (e_l * t_l), f"relmse_{tag}": e_l, f"seconds_{tag}": t_l,
                        f"rays_{tag}": r_l})
        out["gain_per_length_vs_one_budget"] = (e_m * t_m) / (out["relmse_per_length"] *
                                                             out["seconds_per_length"])
    if unaware:
        e_u, t_u, _, r_u = run(api.ALLOC_MARS, aware=False)
        out.update({"mars_budget_unaware": 1.0 / (e_u * t_u),
                    "gain_vs_budget_unaware": (e_u * t_u) / (e_m * t_m),
                    "relmse_budget_unaware": e_u, "seconds_budget_unaware": t_u,
                    "rays_budget_unaware": r_u})
    return out


def run_ears(args, api, torch):
    """MARS against EARS (one count shared by every technique of a vertex,
    the paper's comparison method), MARS with budget-unaware MIS weights,
    and classic RR, by the efficiency
    protocol above: the guided 512x512 heightfield (9 iterations of 1..256
    spp, 4096 spp reference) and the bidirectional 1280x720 interior (7
    iterations of 1..64 spp, 1024 spp reference).  value = MARS's efficiency
    gain over EARS on the guided scene."""
    import scenegen
    ctx = api.Context(0)
    sc = scenegen.make_heightfield_scene(seed=1)
    print("[bench] ears: guided", file=sys.stderr, flush=True)
    g = efficiency_leg(api, ctx, sc, torch, ears=True, unaware=True)
    print("[bench] ears: bdpt", file=sys.stderr, flush=True)
    scb = scenegen.make_interior(seed=1)
    b = efficiency_leg(api, ctx, scb, torch, n_iter=7, mode=api.MODE_BDPT, depth=12,
                       ref_spp=(16, 64), ears=True, unaware=True)
    return {"metric": "efficiency 1/(relMSE*s): MARS vs EARS (classic RR beside them)",
            "value": g["gain_vs_ears"], "unit": "ratio", "n_gpus": 1, "steps": g["iterations"],
            "warmup": 3, "ms_per_step": g["seconds_mars"] * 1e3 / g["iterations"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "ears_vs_mars_guided512_bdpt720",
                       "guided": {"width": sc["width"], "height": sc["height"],
                                  "triangles": int(sc["V"].shape[0]), "max_depth": 10},
                       "bdpt": {"width": scb["width"], "height": scb["height"],
                                "triangles": int(scb["V"].shape[0]), "max_depth": 12}},
            "guided": g, "bdpt": b,
            "paper_context": {"guided_mars_vs_ears_plus_mixture_gd": 1.32,
                              "guided_rays_vs_ears": -0.17, "bdpt_mars_vs_ears": 1.6,
                              "bdpt_rays_vs_ears": -0.13,
                              "note": "10 production scenes, 5 min equal time, CPU (Mitsuba); "
                                      "the guided comparison there also differs in the guiding "
                                      "method (gradient-descent mixtures)"}}


def run_lp_lengths(args, api, torch):
    """Separate light-path budgets per light-vertex index (y_1, y_2, y_3+;
    the variant Sec. 5 leaves to future work) against one light-path budget,
    classic RR beside them, by the efficiency protocol on the bidirectional
    1280x720 interior (7 iterations of 1..64 spp against 1024 spp), with
    the budget-aware and the budget-unaware balance heuristic.  value =
    per-length MARS's 1/(relMSE s) over one-budget MARS's."""
    import scenegen
    ctx = api.Context(0)
    scb = scenegen.make_interior(seed=1)
    print("[bench] lp_lengths: bdpt", file=sys.stderr, flush=True)
    b = efficiency_leg(api, ctx, scb, torch, n_iter=7, mode=api.MODE_BDPT, depth=12,
                       ref_spp=(16, 64), unaware=True, lp_lengths=True)
    return {"metric": "efficiency 1/(relMSE*s): per-length light-path budgets vs one budget "
                      "(MARS, bidirectional)",
            "value": b["gain_per_length_vs_one_budget"], "unit": "ratio", "n_gpus": 1,
            "steps": b["iterations"], "warmup": 3,
            "ms_per_step": b["seconds_per_length"] * 1e3 / b["iterations"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "lp_lengths_bdpt720", "width": scb["width"],
                       "height": scb["height"], "triangles": int(scb["V"].shape[0]),
                       "max_depth": 12, "classes": ["y_1", "y_2", "y_3+"]},
            "bdpt": b}


# queue memory of the bidirectional workload (of the 288 GB of HBM): half
# the frame's camera samples per tile
BDPT_QUEUE_GIB = 160


def run_bdpt(args, api, torch):
    """Bidirectional workload: 1280x720 interior, 1,040,714 triangles, max
    path length 12.  One step = one MARS iteration at 1 spp (render + update)
    after classic warm-up iterations; efficiency of MARS vs classic-RR BDPT
    with the doubling schedule (1..64 spp) against a 1024 spp reference."""
    import scenegen
    sc = scenegen.make_interior(seed=1)
    ctx = api.Context(0)
    s = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12, max_cells=cells_budget())
    warm = max(4, args.warmup)

    def step(i):
        alloc = api.ALLOC_CLASSIC if i < 3 else api.ALLOC_MARS
        p = api.iter_params(iteration=i, spp=1, alloc=alloc, stat_clamp=0.0)
        st = s.render_iteration(p)
        s.update(p)
        return st
    for i in range(warm):
        step(i)
    # queue and tile sizes from the autotuner on a MARS iteration (connections
    # multiply the shadow queues), then one untimed iteration at those sizes
    tuned = api.autotune([s], api.iter_params(iteration=warm, spp=1, alloc=api.ALLOC_MARS,
                                              stat_clamp=0.0), mem_budget=BDPT_QUEUE_GIB << 30)
    torch.cuda.empty_cache()
    step(warm)
    warm += 1
    print(f"[bench] bdpt: warm, tuned {tuned}", file=sys.stderr, flush=True)
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rays = 0
    for k in range(args.steps):
        rays += step(warm + k).total_rays()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    s.release()
    px = sc["width"] * sc["height"]
    out = {"metric": "Mpaths/s (bidirectional MARS iterations)", "value": px * args.steps / dt / 1e6,
           "unit": "Mpaths/s", "n_gpus": 1, "steps": args.steps, "warmup": warm,
           "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "bdpt_1280x720_interior1m_d12", "width": sc["width"],
                      "height": sc["height"], "triangles": int(sc["V"].shape[0]), "max_depth": 12,
                      "spp_per_step": 1, "techniques": ["bsdf", "nee", "light_path"],
                      "queue_capacity": tuned[0][0], "shadow_queue_capacity": tuned[0][3],
                      "tile_roots": tuned[0][1]},
           "mrays_per_s": rays / dt / 1e6,
           "kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]}}
    if not args.no_efficiency:
        print("[bench] bdpt: efficiency", file=sys.stderr, flush=True)
        out["efficiency"] = efficiency_leg(api, ctx, sc, torch, n_iter=7, mode=api.MODE_BDPT,
                                           depth=12, ref_spp=(16, 64))
    return out


LEARNED_WORKLOAD = "learned_vs_octree_bdpt_1920x1080_interior2m_d12"
LEARNED_SPP = 2            # camera samples per pixel of a timed step
LEARNED_TRAIN_STEPS = 32   # Adam steps of 8192 samples after every update
LEARNED_FIRST = 5          # the first learned-cache iteration (after 3 classic, 2 octree MARS)


def learned_scene():
    import scenegen
    return scenegen.make_interior(seed=3, width=1920, height=1080, n_pieces=4500)


def relmse_pair(img, r1, r2, eps=1e-2, drop=1e-4):
    """relMSE against the mean of two independent half references, with the
    reference's own noise removed: E[(I - (R1+R2)/2)^2] exceeds the error to
    the expectation by Var(R)/2 per half, estimated per pixel as
    (R1 - R2)^2 / 4.  Same outlier rule and epsilon as relmse()."""
    import numpy as np
    ref = 0.5 * (r1 + r2)
    d = img.astype(np.float64) - ref
    noise = 0.25 * (r1 - r2) ** 2
    e = np.sort(np.mean((d * d - noise) / (ref * ref + eps), axis=-1).ravel())
    keep = e.size - int(np.floor(drop * e.size))
    return float(np.mean(e[:keep]))


def time_to_relmse(curve, target):
    """Seconds a (seconds, relMSE) curve needs to reach `target`,
    interpolated log-log between the iterations around it; None if never."""
    import math
    prev = None
    for t, e in curve:
        if e <= target:
            if prev is None or prev[1] <= e:
                return t
            a = (math.log(target) - math.log(prev[1])) / (math.log(e) - math.log(prev[1]))
            return math.exp(math.log(prev[0]) + a * (math.log(t) - math.log(prev[0])))
        prev = (t, e)
    return None


def learned_efficiency(api, ctx, sc, torch, seeds=(1, 2, 3, 4, 5), n_iter=11, ref_half_spp=512):
    """Octree MARS and learned-cache MARS over the growing-iteration schedule
    (spp_i = min(2^max(0, i - 3), 16): 3 classic-RR iterations, octree MARS
    from the 4th, the network's counts from the 6th; the network trains 32
    Adam steps after every update from the 4th; queue and tile sizes from the
    autotuner before the 4th), each iteration's inverse-variance weighted
    image scored against a reference of 2 x ref_half_spp spp of classic-RR
    BDPT with its own noise removed.  Efficiency at equal relMSE: the target
    is the larger of the two methods' final relMSE, each method's time to
    reach it is interpolated on its curve, and efficiency = 1 / (target x
    time).  Five random-stream seeds; the value is the geometric mean of
    the per-seed ratios."""
    import math

    import numpy as np

    def half(base):
        r = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12, max_cells=cells_budget())
        acc = np.zeros((sc["height"], sc["width"], 3))
        n = ref_half_spp // 16
        for i in range(n):
            r.render_iteration(api.iter_params(iteration=base + i, spp=16, stat_clamp=0.0))
            acc += r.image(api.IMAGE_LAST)
        r.release()
        return acc / n
    t0 = time.perf_counter()
    r1, r2 = half(100000), half(200000)
    t_ref = time.perf_counter() - t0
    print(f"[bench] learned: reference {2 * ref_half_spp} spp in {t_ref:.1f} s", file=sys.stderr,
          flush=True)
    runs = []
    for seed in seeds:
        res = {"seed": seed}
        for kind in ("octree", "learned"):
            s = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12, max_cells=cells_budget(),
                          mlp=(kind == "learned"), seed=seed)
            curve, t_cum, rays, spp_tot, t_train = [], 0.0, 0, 0, 0.0
            for i in range(n_iter):
                spp = min(1 << max(0, i - 3), 16)
                alloc = api.ALLOC_CLASSIC if i < 3 else api.ALLOC_MARS
                if kind == "learned" and i >= 5:
                    alloc = api.ALLOC_MLP
                p = api.iter_params(iteration=i, spp=spp, alloc=alloc, stat_clamp=0.0)
                if i == 3:
                    api.autotune([s], p, mem_budget=96 << 30)
                    torch.cuda.empty_cache()
                torch.cuda.synchronize()
                ta = time.perf_counter()
                rays += s.render_iteration(p).total_rays()
                s.update(p)
                if kind == "learned" and i >= 3:
                    torch.cuda.synchronize()
                    tt = time.perf_counter()
                    s.mlp_train(steps=LEARNED_TRAIN_STEPS, batch=8192, lr=2e-3)
                    torch.cuda.synchronize()
                    t_train += time.perf_counter() - tt
                torch.cuda.synchronize()
                t_cum += time.perf_counter() - ta
                spp_tot += spp
                curve.append((t_cum, relmse_pair(s.image(api.IMAGE_IVW), r1, r2)))
            s.release()
            res[kind] = {"curve": [[round(t, 4), e] for t, e in curve], "seconds": t_cum,
                         "relmse": curve[-1][1], "rays": rays, "spp": spp_tot,
                         "train_seconds": t_train,
                         "efficiency_equal_iterations": 1.0 / (curve[-1][1] * t_cum)}
        target = max(res["octree"]["relmse"], res["learned"]["relmse"])
        for kind in ("octree", "learned"):
            tk = time_to_relmse([tuple(c) for c in res[kind]["curve"]], target)
            res[kind]["seconds_to_target"] = tk
            res[kind]["efficiency"] = 1.0 / (target * tk)
        res["target_relmse"] = target
        res["ratio"] = res["learned"]["efficiency"] / res["octree"]["efficiency"]
        print(f"[bench] learned: seed {seed} ratio {res['ratio']:.3f}", file=sys.stderr, flush=True)
        runs.append(res)
    ratios = [r["ratio"] for r in runs]
    return {"definition": "1/(relMSE*s) at equal relMSE: the larger final relMSE of the two "
                          "methods is the target, each method's time to reach it interpolated "
                          "log-log on its per-iteration curve; relMSE = mean (I-R)^2/(R^2+0.01) "
                          "minus the reference's own noise, 0.01% largest terms discarded",
            "ratio_learned_vs_octree": float(math.exp(np.mean(np.log(ratios)))),
            "ratio_per_seed": ratios,
            "octree": float(np.mean([r["octree"]["efficiency"] for r in runs])),
            "learned": float(np.mean([r["learned"]["efficiency"] for r in runs])),
            "schedule_spp": [min(1 << max(0, i - 3), 16) for i in range(n_iter)],
            "reference_spp": 2 * ref_half_spp, "reference_seconds": t_ref, "per_seed": runs}


def cpu_baseline_learned(sc, warm, spp=LEARNED_SPP, frac=0.25, seed=7):
    """The oracle as it stands (octree MARS: it has no learned cache) on the
    same scene at 1/16 of the pixels (480 x 270), a random quarter of them
    rendered: `warm` warm-up iterations (3 classic), then timed MARS
    iterations of `spp` samples per pixel (render + update) on all host
    threads, then one of 1 spp on a single thread."""
    import numpy as np

    import scenegen
    from oracle import oracle as orc
    small = scenegen.scaled(sc, 480, 270)
    threads = orc.set_threads(0)
    o = orc.Oracle(small, mode=orc.MODE_BDPT, max_depth=12, max_cells=cells_budget())
    rng = np.random.default_rng(seed)
    npx = small["width"] * small["height"]
    sub = rng.choice(npx, int(frac * npx), replace=False)
    o.set_pixel_subset(sub)
    for i in range(warm):
        alloc = orc.ALLOC_CLASSIC if i < 3 else orc.ALLOC_MARS
        p = orc.Oracle.params(iteration=i, spp=1 if i < 3 else spp, alloc=alloc, stat_clamp=0.0)
        o.render_iteration(p)
        o.update(p)
    t0 = time.perf_counter()
    n_iter, rays = 0, 0
    while True:
        p = orc.Oracle.params(iteration=warm + n_iter, spp=spp, alloc=orc.ALLOC_MARS,
                              stat_clamp=0.0)
        rays += o.render_iteration(p).total_rays()
        o.update(p)
        n_iter += 1
        if time.perf_counter() - t0 > 12.0 or n_iter >= 3:
            break
    dt = time.perf_counter() - t0
    # one core: one more iteration of 1 spp on the same pixels (the light
    # subpaths of every pixel are traced whatever the subset, so a smaller
    # subset would not scale)
    orc.set_threads(1)
    p = orc.Oracle.params(iteration=warm + n_iter, spp=1, alloc=orc.ALLOC_MARS, stat_clamp=0.0)
    t1 = time.perf_counter()
    o.render_iteration(p)
    o.update(p)
    dt1 = time.perf_counter() - t1
    orc.set_threads(0)
    paths = len(sub) * spp * n_iter
    return {"value": paths / dt / 1e6, "unit": "Mpaths/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_info(), "mrays_per_s": rays / dt / 1e6,
            "one_core_mpaths_per_s": len(sub) / dt1 / 1e6,
            "sample": f"the oracle's octree MARS (no learned cache) on the same scene at "
                      f"480x270, {len(sub)} random pixels, {warm} warm-up iterations, "
                      f"{n_iter} timed iterations of {spp} spp in {dt:.1f} s on {threads} "
                      f"threads; the one-core figure from one more iteration of 1 spp on the "
                      f"same pixels ({dt1:.1f} s)"}


def run_learned(args, api, torch):
    """The default workload: learned-cache MARS iterations on the 1920x1080
    bidirectional interior (see the module docstring)."""
    sc = learned_scene()
    ctx = api.Context(0)
    s = api.Scene(ctx, sc, mode=api.MODE_BDPT, max_depth=12, max_cells=cells_budget(), mlp=True,
                  seed=1)
    # 3 classic, 2 octree MARS (updates to train on), then learned-cache
    # iterations; the timed steps are learned-cache iterations only
    n_warm = max(args.warmup, LEARNED_FIRST)

    def alloc_of(i):
        if i < 3:
            return api.ALLOC_CLASSIC
        return api.ALLOC_MARS if i < LEARNED_FIRST else api.ALLOC_MLP

    log = iterlog_open(args)

    def step(i):
        p = api.iter_params(iteration=i, spp=LEARNED_SPP, alloc=alloc_of(i), stat_clamp=0.0)
        if i == 3:
            api.autotune([s], p, mem_budget=96 << 30)
            torch.cuda.empty_cache()
        t = time.perf_counter()
        st = s.render_iteration(p)
        us = s.update(p)
        if i >= 3:
            s.mlp_train(steps=LEARNED_TRAIN_STEPS, batch=8192, lr=2e-3)
        if log:
            log.write(iterlog.record(i, p, st, us, time.perf_counter() - t, sc["width"],
                                     sc["height"], s.count_map()))
        return st, us

    for i in range(n_warm):
        step(i)
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile(True, kernels=["trace"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rays = rays_closest = rays_shadow = retries = 0
    t_steps = []  # host time at the end of each step (each step ends with host waits)
    for k in range(args.steps):
        st, _ = step(n_warm + k)
        t_steps.append(time.perf_counter())
        rays += st.total_rays()
        retries += st.overflow_retries
        rays_closest += st.rays_camera + st.rays_ext + st.rays_light
        rays_shadow += st.rays_shadow + st.rays_conn
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    qq = s.query_queues()
    window = {"workload": LEARNED_WORKLOAD, "warmup": n_warm, "steps": args.steps}
    paths = args.steps * sc["width"] * sc["height"] * LEARNED_SPP
    out = {
        "metric": "Mpaths/s of learned-cache MARS iterations; efficiency 1/(relMSE*s) of the "
                  "learned cache vs octree MARS at equal relMSE beside it",
        "value": paths / dt / 1e6, "unit": "Mpaths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 radiance, bf16 network",
        "data": "synthetic",
        "config": {"workload": LEARNED_WORKLOAD, "width": sc["width"], "height": sc["height"],
                   "triangles": int(sc["V"].shape[0]), "max_depth": 12,
                   "spp_per_step": LEARNED_SPP, "techniques": ["bsdf", "nee", "light_path"],
                   "network": "6 inputs, 72 sin/cos features, 3 x 64 ReLU, 3 log counts",
                   "train_steps_per_update": LEARNED_TRAIN_STEPS, "max_cells": cells_budget(),
                   "warmup_iterations": n_warm, "queue_capacity": qq[0],
                   "shadow_queue_capacity": qq[1], "tile_roots": s.query()[1],
                   "overflow_reruns_timed": retries},
        "mrays_per_s": rays / dt / 1e6,
        "trace_launches_timed": prof["trace"][1],
        "step_ms": [round((b - a) * 1e3, 2) for a, b in zip([t0] + t_steps[:-1], t_steps)],
    }
    if args.profile_steps >= 0:
        print(json.dumps(out), flush=True)
        return None
    n_brk = 2
    ctx.profile(True)
    for k in range(n_brk):
        step(n_warm + args.steps + k)
    brk = ctx.profile_read()
    ctx.profile(False)
    out["kernels_ms_per_step"] = {k: round(v[0] / n_brk, 3) for k, v in brk.items() if v[1]}
    out["roofline"] = roofline(api, ctx, prof, lambda: step(n_warm + args.steps + n_brk),
                               rays_closest, rays_shadow, "trace_learned1080_traffic.json",
                               window)
    s.release()
    if not args.no_efficiency:
        print("[bench] learned: efficiency", file=sys.stderr, flush=True)
        out["efficiency"] = learned_efficiency(api, ctx, sc, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_learned(sc, LEARNED_FIRST)
    return out


def run_convergence(args, api, torch, seeds=(1, 2, 3), n_iter=9):
    """Convergence of the fixed point on the guided 512x512 heightfield:
    for MARS and EARS, per iteration of the doubling schedule (1..256 spp,
    the first three classic RR), the mean count per technique at the first
    hit, the method's own 1/(V_I C_I), rays per camera sample and the
    running efficiency 1/(relMSE s) of the inverse-variance weighted image
    against a 4096 spp classic reference; each with several random-stream
    seeds, whose spread is the stability check.  value = the mean over seeds
    of MARS's final efficiency divided by classic RR's at the same spp."""
    import numpy as np
    import scenegen
    ctx = api.Context(0)
    sc = scenegen.make_heightfield_scene(seed=1)
    ref = reference_image(api, ctx, sc, spp=16, iters=256)
    print("[bench] convergence: reference done", file=sys.stderr, flush=True)

    def run(alloc_after, seed):
        s = api.Scene(ctx, sc, mode=api.MODE_PT_GUIDED, max_depth=10, max_cells=cells_budget(),
                      seed=seed)
        rows, t, spp_tot, acc = [], 0.0, 0, np.zeros_like(ref)
        for i in range(n_iter):
            alloc = api.ALLOC_CLASSIC if i < 3 else alloc_after
            p = api.iter_params(iteration=i, spp=1 << i, alloc=alloc, stat_clamp=50.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.render_iteration(p)
            us = s.update(p) if alloc_after != api.ALLOC_CLASSIC else None
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            spp_tot += 1 << i
            cm = s.count_map().reshape(-1, 3)
            if alloc_after == api.ALLOC_CLASSIC:
                acc += s.image(api.IMAGE_LAST) * (1 << i)
                img = acc / spp_tot
            else:
                img = s.image(api.IMAGE_IVW)
            e = relmse(img, ref)
            rows.append({"iteration": i, "spp": 1 << i, "alloc": int(alloc),
                         "mean_count_first_hit": [float(v) for v in cm.mean(0)],
                         "inv_vi_ci": (1.0 / (us.V_I * us.C_I)) if us and us.V_I > 0 else None,
                         "rays_per_sample": st.total_rays() / float(sc["width"] * sc["height"]
                                                                    * (1 << i)),
                         "relmse": e, "seconds": t, "efficiency": 1.0 / (e * t)})
        s.release()
        return rows

    out_runs = {"mars": [], "ears": [], "classic": []}
    for seed in seeds:
        for name, alloc in (("mars", api.ALLOC_MARS), ("ears", api.ALLOC_EARS),
                            ("classic", api.ALLOC_CLASSIC)):
            out_runs[name].append({"seed": seed, "rows": run(alloc, seed)})
        print(f"[bench] convergence: seed {seed} done", file=sys.stderr, flush=True)

    def final(name):
        return np.array([r["rows"][-1]["efficiency"] for r in out_runs[name]])
    fm, fe, fc = final("mars"), final("ears"), final("classic")
    stab = {n: {"final_efficiency_mean": float(f.mean()),
                "final_efficiency_cv": float(f.std() / f.mean()),
                "final_mean_counts": [[round(v, 4) for v in r["rows"][-1]["mean_count_first_hit"]]
                                      for r in out_runs[n]]}
            for n, f in (("mars", fm), ("ears", fe), ("classic", fc))}
    return {"metric": "convergence: per-iteration counts and efficiency (MARS, EARS, classic RR)",
            "value": float(np.mean(fm / fc)), "unit": "ratio", "n_gpus": 1, "steps": n_iter,
            "warmup": 3, "ms_per_step": float(np.mean([r["rows"][-1]["seconds"]
                                                       for r in out_runs["mars"]])) * 1e3 / n_iter,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "convergence_guided_512x512_heightfield132k_d10",
                       "seeds": list(seeds), "iterations": n_iter, "reference_spp": 4096},
            "mars_vs_ears_final": float(np.mean(fm / fe)), "stability": stab, "runs": out_runs}


def run_rounding(args, api, torch, n_alloc=9, n_rep=24, seed=1):
    """Low-discrepancy rounding (supplement Alg. 1) against rounding each
    count with its own uniform, in renders: the guided 512x512 heightfield
    after a MARS schedule (the doubling schedule of 9 iterations), then the
    allocation frozen (no further update) and n_rep render iterations of
    4 spp with each rounding, alternating; the per-pixel variance of the
    iteration images over the repetitions, relative to the squared mean
    image (channel mean, pixels with a mean above 1e-3 of the image's), for
    each scheme.  value = 1 - V(Alg. 1) / V(independent): the variance the
    low-discrepancy rounding saves.  The same for the bidirectional 1280x720
    interior beside it."""
    import numpy as np
    import scenegen
    ctx = api.Context(0)
    out = {}
    for name, sc, mode, depth, kc in (
            ("guided512", scenegen.make_heightfield_scene(seed=1), api.MODE_PT_GUIDED, 10, 50.0),
            ("bdpt720", scenegen.make_interior(seed=1), api.MODE_BDPT, 12, 0.0)):
        s = api.Scene(ctx, sc, mode=mode, max_depth=depth, max_cells=cells_budget(), seed=seed)
        for i in range(n_alloc):
            p = api.iter_params(iteration=i, spp=min(1 << max(0, i - 3), 16), stat_clamp=kc,
                                alloc=api.ALLOC_CLASSIC if i < 3 else api.ALLOC_MARS)
            s.render_iteration(p)
            s.update(p)
        imgs = {0: [], 1: []}
        rays = {0: 0, 1: 0}
        for r in range(n_rep):
            for rounding in (0, 1):
                p = api.iter_params(iteration=1000 + r, spp=4, stat_clamp=kc,
                                    alloc=api.ALLOC_MARS, rounding=rounding)
                rays[rounding] += s.render_iteration(p).total_rays()
                imgs[rounding].append(s.image(api.IMAGE_LAST).astype(np.float64))
        s.release()
        mean = 0.5 * (np.mean(imgs[0], 0) + np.mean(imgs[1], 0))
        m = mean.mean(-1)
        keep = m > 1e-3 * m.mean()
        rel = {k: float(np.mean(np.var(np.array(v), 0, ddof=1).mean(-1)[keep] / m[keep] ** 2))
               for k, v in imgs.items()}
        # the spread of that ratio from halves of the repetitions
        half = []
        for a, b in ((slice(0, n_rep // 2), slice(n_rep // 2, n_rep)),):
            for sl in (a, b):
                r0 = np.mean(np.var(np.array(imgs[0][sl]), 0, ddof=1).mean(-1)[keep] / m[keep] ** 2)
                r1 = np.mean(np.var(np.array(imgs[1][sl]), 0, ddof=1).mean(-1)[keep] / m[keep] ** 2)
                half.append(1.0 - r0 / r1)
        out[name] = {"rel_var_alg1": rel[0], "rel_var_independent": rel[1],
                     "saving": 1.0 - rel[0] / rel[1], "saving_halves": half,
                     "rays_alg1": rays[0], "rays_independent": rays[1],
                     "pixels": int(keep.sum()), "repetitions": n_rep}
        print(f"[bench] rounding {name}: saving {out[name]['saving']:.4f}", file=sys.stderr,
              flush=True)
    return {"metric": "variance saved by low-discrepancy rounding (Alg. 1) against rounding "
                      "each count independently, frozen MARS allocation",
            "value": out["guided512"]["saving"], "unit": "fraction", "n_gpus": 1,
            "steps": n_rep, "warmup": n_alloc, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "rounding_guided512_bdpt720", "spp_per_repetition": 4},
            "per_scene": out, "paper_context": {"saving": 0.02}}


def iterlog_open(args):
    """The per-iteration JSON-lines log of --log-jsonl, or None.  Logging
    reads the count map back after every step (a few ms at 1920x1080), so a
    logged run's timing is not the benchmark's."""
    return iterlog.IterationLog(args.log_jsonl) if args.log_jsonl else None


def cells_budget(mbytes=72.0):
    # bytes per cell: factors 72, accumulators 192, visits/leaf data 12,
    # directional pmf+cdf 512, training sums 512, octree node words 32
    return int(mbytes * 1e6 / (72 + 192 + 12 + 512 + 512 + 32))


BATCH_WORKLOAD = "batch32_mixed_guided_bdpt"


def queue_bytes(scene, cap, scap):
    """The library's queue memory model: per level 168 B per ray-queue entry
    (+32 B for BDPT) and 16 B per shadow value, the 32 B shadow rays in one
    level (no learned cache or per-length budgets in the batch)."""
    per = 168 + (32 if scene.mode == 2 else 0)
    return (scene.max_depth + 2) * (cap * per + scap * 16) + scap * 32


def run_batch(args, api, torch, seed=1, budget=64 << 30):
    """The batched workload: 32 independent scenes (resolution uniform over
    64^2 .. 1024^2, 1k-500k triangles log-uniform, half guided PT and half
    BDPT, depth 6-12, counts clamped to 8), one step = one iteration of every
    scene (render at 1 spp + update) as one replay of the captured graph.
    Queue and tile sizes come from the autotuner under a 64 GiB queue budget.
    Beside it: the same iterations through the per-scene calls."""
    import scenegen
    t0 = time.perf_counter()
    scenes = scenegen.make_batch(seed=seed)
    ctx = api.Context(0)
    modes = {"guided": api.MODE_PT_GUIDED, "bdpt": api.MODE_BDPT}
    S, E = [], []
    for sc in scenes:
        roots = sc["width"] * sc["height"]
        kw = dict(mode=modes[sc["mode"]], max_depth=sc["max_depth"], max_cells=cells_budget(),
                  queue_capacity=min(4 * roots, 1 << 19), tile_roots=min(roots, 1 << 17))
        S.append(api.Scene(ctx, sc, **kw))
        E.append(api.Scene(ctx, sc, **kw))
    print(f"[bench] batch: {len(S)} scenes uploaded twice in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    def params(i):
        alloc = api.ALLOC_CLASSIC if i < 2 else api.ALLOC_MARS
        return api.iter_params(iteration=i, spp=1, alloc=alloc, stat_clamp=50.0, clamp_hi=8.0)

    warm = max(3, args.warmup)
    for i in range(warm):
        api.iterate_batch(S, params(i))
        for e in E:
            e.render_iteration(params(i))
            e.update(params(i))
    torch.cuda.synchronize()
    # tuned on a MARS iteration: splitting sets the queue peaks
    t1 = time.perf_counter()
    tuned = api.autotune(S, params(warm), mem_budget=budget)
    for e, (cap, tile, _, scap, _) in zip(E, tuned):
        e.configure(queue_capacity=cap, tile_roots=tile, shadow_capacity=scap)
    torch.cuda.empty_cache()  # queue buffers replaced while tuning
    print(f"[bench] batch: autotuned in {time.perf_counter() - t1:.1f} s", file=sys.stderr,
          flush=True)
    # first use of the tuned sizes (graph capture) outside the timed region
    api.iterate_batch(S, params(warm))
    for e in E:
        e.render_iteration(params(warm))
        e.update(params(warm))
    torch.cuda.synchronize()
    print("[bench] batch: warm", file=sys.stderr, flush=True)
    warm += 1
    reruns = []

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    step_ms = {"graph": [], "pool": []}
    reruns_pool = []

    def graph_steps(i0):
        for k in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            its, _ = api.iterate_batch(S, params(i0 + k))
            step_ms["graph"].append(round((time.perf_counter() - t) * 1e3, 1))
            reruns.append(sum(1 for s in its if s.overflow_retries > 0))

    def eager_steps(i0):
        for k in range(args.steps):
            for e in E:
                e.render_iteration(params(i0 + k))
                e.update(params(i0 + k))

    def pool_steps(i0):
        for k in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            its, _ = api.iterate_batch(E, params(i0 + k), graph=False)
            step_ms["pool"].append(round((time.perf_counter() - t) * 1e3, 1))
            reruns_pool.append(sum(1 for s in its if s.overflow_retries > 0))

    dt = timed(lambda: graph_steps(warm))
    ctx.profile(True)
    dt_eager = timed(lambda: eager_steps(warm))
    prof = ctx.profile_read()
    ctx.profile(False)
    dt_pool = timed(lambda: pool_steps(warm + args.steps))
    px = sum(sc["width"] * sc["height"] for sc in scenes)
    tris = sum(int(sc["V"].shape[0]) for sc in scenes)
    ctx_out = {
        "metric": "Mpaths/s (batched iterations of 32 scenes)",
        "value": px * args.steps / dt / 1e6,
        "unit": "Mpaths/s",
        "n_gpus": 1, "steps": args.steps, "warmup": warm,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "scenes": len(scenes), "pixels_per_step": px,
                   "triangles": tris, "spp_per_step": 1, "clamp_hi": 8.0,
                   "guided": sum(sc["mode"] == "guided" for sc in scenes),
                   "bdpt": sum(sc["mode"] == "bdpt" for sc in scenes),
                   "queue_bytes": sum(queue_bytes(s, c, sc_) for s, (c, _, _, sc_, _) in zip(S, tuned))},
        "eager_ms_per_step": dt_eager * 1e3 / args.steps,
        "stream_pool_ms_per_step": dt_pool * 1e3 / args.steps,
        "graph_speedup_vs_eager": dt_eager / dt,
        "overflow_reruns_per_step": reruns,
        "step_ms": step_ms, "overflow_reruns_per_step_pool": reruns_pool,
        "eager_kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]},
    }
    return ctx_out


def cpu_baseline_guided(sc, warm, n_pix=65536, seed=7):
    """The oracle as it stands on the guided workload: n_pix random pixels of
    the same 512 x 512 frame, the same `warm` warm-up iterations as the GPU
    (the first three classic), then the MARS iterations the GPU times (render
    + update, 1 spp) on all host threads, and one more on a single thread
    over a sixteenth of the pixels."""
    import numpy as np

    from oracle import oracle as orc
    threads = orc.set_threads(0)
    o = orc.Oracle(sc, mode=orc.MODE_PT_GUIDED, max_depth=10, max_cells=cells_budget())
    rng = np.random.default_rng(seed)
    sub = rng.choice(sc["width"] * sc["height"], n_pix, replace=False)
    o.set_pixel_subset(sub)
    for i in range(warm):
        p = orc.Oracle.params(iteration=i, spp=1,
                              alloc=orc.ALLOC_CLASSIC if i < min(3, warm) else orc.ALLOC_MARS)
        o.render_iteration(p)
        o.update(p)
    t0 = time.perf_counter()
    n_iter = rays = 0
    while True:
        p = orc.Oracle.params(iteration=warm + n_iter, spp=1, alloc=orc.ALLOC_MARS)
        rays += o.render_iteration(p).total_rays()
        o.update(p)
        n_iter += 1
        if time.perf_counter() - t0 > 10.0 or n_iter >= 8:
            break
    dt = time.perf_counter() - t0
    orc.set_threads(1)
    o.set_pixel_subset(sub[: n_pix // 16])
    p = orc.Oracle.params(iteration=warm + n_iter, spp=1, alloc=orc.ALLOC_MARS)
    t1 = time.perf_counter()
    o.render_iteration(p)
    o.update(p)
    dt1 = time.perf_counter() - t1
    orc.set_threads(0)
    return {"value": n_pix * n_iter / dt / 1e6, "unit": "Mpaths/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_info(), "mrays_per_s": rays / dt / 1e6,
            "one_core_mpaths_per_s": (n_pix // 16) / dt1 / 1e6,
            "sample": f"{n_pix} random pixels of the 512x512 frame, the GPU's {warm} warm-up "
                      f"iterations, then {n_iter} MARS iterations (render+update, the GPU's "
                      f"timed iterations {warm}..{warm + n_iter - 1}) in {dt:.1f} s on "
                      f"{threads} threads; one core: one iteration on {n_pix // 16} pixels"}


def run_guided(args, api, torch):
    """Guided path tracing at 512 x 512 on the 132k-triangle heightfield:
    one step = one MARS iteration at 1 spp (render + update) after classic
    warm-up iterations; efficiency of MARS vs classic RR beside it."""
    import scenegen
    sc = scenegen.make_heightfield_scene(seed=1)
    ctx = api.Context(0)
    s = api.Scene(ctx, sc, mode=api.MODE_PT_GUIDED, max_depth=10, max_cells=cells_budget())
    n_classic = min(3, args.warmup)

    log = iterlog_open(args)

    def step(i):
        alloc = api.ALLOC_CLASSIC if i < n_classic else api.ALLOC_MARS
        p = api.iter_params(iteration=i, spp=1, alloc=alloc, stat_clamp=50.0)
        t = time.perf_counter()
        st = s.render_iteration(p)
        us = s.update(p)
        if log:
            log.write(iterlog.record(i, p, st, us, time.perf_counter() - t, sc["width"],
                                     sc["height"], s.count_map()))
        return st, us

    for i in range(args.warmup):
        step(i)
        print(f"[bench] warmup {i}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # HIP events around the launches of the roofline's kernel only, so that
    # the timed steps carry no events for the others
    ctx.profile(True, kernels=["trace"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rays = rays_closest = rays_shadow = 0
    for k in range(args.steps):
        st, us = step(args.warmup + k)
        rays += st.total_rays()
        rays_closest += st.rays_camera + st.rays_ext
        rays_shadow += st.rays_shadow
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    print(f"[bench] timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    paths = args.steps * sc["width"] * sc["height"]
    out = {
        "metric": "Mpaths/s (guided MARS iterations; efficiency 1/(relMSE*s) beside it)",
        "value": paths / dt / 1e6, "unit": "Mpaths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "width": sc["width"], "height": sc["height"],
                   "triangles": int(sc["V"].shape[0]), "max_depth": 10, "spp_per_step": 1,
                   "techniques": ["bsdf", "nee", "guided"], "max_cells": cells_budget()},
        "mrays_per_s": rays / dt / 1e6,
        "trace_launches_timed": prof["trace"][1],
    }
    if args.profile_steps >= 0:
        print(json.dumps(out), flush=True)
        return None
    n_brk = 2
    ctx.profile(True)
    for k in range(n_brk):
        step(args.warmup + args.steps + k)
    brk = ctx.profile_read()
    ctx.profile(False)
    out["kernels_ms_per_step"] = {k: round(v[0] / n_brk, 3) for k, v in brk.items() if v[1]}
    window = {"workload": WORKLOAD, "warmup": args.warmup, "steps": args.steps}
    out["roofline"] = roofline(api, ctx, prof, lambda: step(args.warmup + args.steps + n_brk),
                               rays_closest, rays_shadow, "trace_guided512_traffic.json", window)
    if not args.no_efficiency:
        print("[bench] efficiency", file=sys.stderr, flush=True)
        out["efficiency"] = efficiency_leg(api, ctx, sc, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_guided(sc, args.warmup)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default: 10 for the learned workload, else 5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=-1,
                    help="(profiling runs) stop after the timed steps: no breakdown, "
                         "roofline, efficiency or CPU leg")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--workload", default="learned",
                    choices=["learned", "mlp", "guided", "batch", "bdpt", "ears", "convergence",
                             "lp_lengths",
                             "rounding"],
                    help="learned (default; mlp is the same): 1920x1080 bidirectional, learned "
                         "cache vs octree; guided: the 512x512 guided-PT workload; batch: 32 "
                         "mixed scenes; bdpt: 1280x720 bidirectional; ears: MARS vs EARS vs "
                         "classic RR efficiency (guided and bidirectional); convergence: "
                         "per-iteration counts and efficiency over several seeds; rounding: "
                         "low-discrepancy against independent rounding in renders")
    ap.add_argument("--no-efficiency", action="store_true")
    ap.add_argument("--log-jsonl", default=None,
                    help="(learned and guided workloads) append one JSON line per iteration "
                         "(rays, Mrays/s, Mpaths/s, V_I, C_I, 1/(V_I C_I), mean first-hit "
                         "counts) to this file")
    args = ap.parse_args()
    if args.warmup is None:
        args.warmup = 10 if args.workload == "learned" else 5
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per box: this benchmark runs on a single MI355X; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2410_20429_amd import api

    if args.copy_calib:
        # plain copy of known size: 1 GiB read + 1 GiB written
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        bcopy = torch.empty_like(a)
        torch.cuda.synchronize()
        bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy
    run = {"learned": run_learned, "mlp": run_learned, "guided": run_guided, "batch": run_batch,
           "lp_lengths": run_lp_lengths,
           "bdpt": run_bdpt, "ears": run_ears, "convergence": run_convergence,
           "rounding": run_rounding}[args.workload]
    out = run(args, api, torch)
    if out is not None:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
