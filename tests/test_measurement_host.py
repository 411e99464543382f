"""Host-side measurement logic of bench.py and the rocprofv3 summaries
(no GPU): the relMSE estimators, the equal-relMSE time interpolation, the
counter calibration and occupancy averages, and the tie between the
committed traffic summaries and the kernel source."""
import csv
import importlib.util
import json
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_relmse_closed_forms(bench):
    rng = np.random.default_rng(3)
    ref = rng.uniform(0.1, 2.0, (40, 50, 3))
    assert bench.relmse(ref.copy(), ref) == 0.0
    # a relative error c in every channel: c^2 R^2 / (R^2 + eps) per channel
    c, eps = 0.1, 1e-2
    want = np.mean(np.mean((c * ref) ** 2 / (ref * ref + eps), axis=-1))
    assert bench.relmse(ref * (1 + c), ref, eps=eps, drop=0.0) == pytest.approx(want, rel=1e-12)
    # the largest fraction `drop` of the per-pixel terms is discarded: one
    # outlier among 2000 pixels with drop = 5e-4 (one term) leaves the
    # others' mean
    img = ref * (1 + c)
    img[7, 9] += 1e3
    assert bench.relmse(img, ref, eps=eps, drop=5e-4) == pytest.approx(
        np.mean(np.delete(np.mean((c * ref) ** 2 / (ref * ref + eps), axis=-1).ravel(), 7 * 50 + 9)),
        rel=1e-12)


def test_relmse_pair_removes_reference_noise(bench):
    rng = np.random.default_rng(4)
    ref = rng.uniform(0.5, 1.5, (64, 64, 3))
    # identical halves: no noise term, the plain estimator
    img = ref * 1.05
    assert bench.relmse_pair(img, ref, ref, drop=0.0) == pytest.approx(
        bench.relmse(img, ref, drop=0.0), rel=1e-12)
    # noisy halves around the truth: the noise-corrected error of the truth
    # itself is near zero, while the plain estimator against the averaged
    # reference sees the reference's variance
    sigma = 0.05
    r1 = ref + rng.normal(0.0, sigma, ref.shape)
    r2 = ref + rng.normal(0.0, sigma, ref.shape)
    plain = bench.relmse(ref, 0.5 * (r1 + r2), drop=0.0)
    fixed = bench.relmse_pair(ref, r1, r2, drop=0.0)
    assert plain > 1e-3 and abs(fixed) < 0.1 * plain


def test_time_to_relmse_log_log(bench):
    curve = [(1.0, 1e-2), (4.0, 1e-3), (8.0, 5e-4)]
    # halfway in log relMSE between 1 s and 4 s: the geometric mean, 2 s
    assert bench.time_to_relmse(curve, 10 ** -2.5) == pytest.approx(2.0, rel=1e-12)
    assert bench.time_to_relmse(curve, 2e-2) == 1.0  # reached at the first point
    assert bench.time_to_relmse(curve, 5e-4) == pytest.approx(8.0)
    assert bench.time_to_relmse(curve, 1e-4) is None
    # a curve that rises before it falls below the target takes the point
    # where it first does so
    assert bench.time_to_relmse([(1.0, 1e-3), (2.0, 2e-3), (3.0, 5e-4)], 1e-3) == 1.0


def _write_counters(path, rows):
    keys = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
            "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))


def test_profiling_calibration_and_occupancy(tmp_path):
    from paper_2410_20429_amd import profiling as P
    copy = "__amd_rocclr_copyBuffer(void*, void*)"
    kern = "mars::trace_quad_kernel(mars::SceneDev, mars::QueuesDev)"
    gib_kib = (1 << 30) / 1024.0
    # the 1 GiB copy reads as half its bytes in FETCH_SIZE (scale 2) and as
    # its bytes in WRITE_SIZE (scale 1); three kernel dispatches, the first
    # outside the window (last_n = 2)
    _write_counters(tmp_path / "f.csv", [
        (1, copy, "FETCH_SIZE", gib_kib / 2, 0, 10), (2, kern, "FETCH_SIZE", 999.0, 10, 20),
        (3, kern, "FETCH_SIZE", 100.0, 20, 30), (4, kern, "FETCH_SIZE", 300.0, 30, 40)])
    _write_counters(tmp_path / "w.csv", [
        (1, copy, "WRITE_SIZE", gib_kib, 0, 10), (2, kern, "WRITE_SIZE", 999.0, 10, 20),
        (3, kern, "WRITE_SIZE", 10.0, 20, 30), (4, kern, "WRITE_SIZE", 30.0, 30, 40)])
    # occupancy per CU 8 (2 waves per SIMD) for 3000 ns, 24 (6 per SIMD) for 1000 ns
    _write_counters(tmp_path / "o.csv", [
        (2, kern, "MeanOccupancyPerCU", 99.0, 0, 5), (3, kern, "MeanOccupancyPerCU", 8.0, 0, 3000),
        (4, kern, "MeanOccupancyPerCU", 24.0, 5000, 6000)])
    win = {"workload": "w", "warmup": 1, "steps": 2}
    t = P.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "trace_quad_kernel", 2, win,
                  str(tmp_path / "o.csv"))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["launches"] == 2 and t["window"] == win
    assert t["hbm_fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert t["hbm_write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert t["occupancy_waves_per_simd"] == pytest.approx((2.0 + 6.0) / 2)
    assert t["occupancy_waves_per_simd_time_weighted"] == pytest.approx((2.0 * 3 + 6.0 * 1) / 4)


@pytest.mark.parametrize("name", ["trace_learned1080_traffic.json", "trace_guided512_traffic.json"])
def test_committed_traffic_summaries_match_kernel_source(bench, name):
    """bench.py uses a committed counter summary only when it was taken on the
    current kernel source over the bench's own window; the committed ones
    must pass that check (re-profile after a kernel change)."""
    with open(os.path.join(ROOT, "profiles", name)) as f:
        t = json.load(f)
    assert bench.load_traffic(name, t["window"]) is not None
    other = dict(t["window"], steps=t["window"]["steps"] + 1)
    assert bench.load_traffic(name, other) is None
    assert t["hbm_bytes_per_launch"] == pytest.approx(
        t["hbm_fetch_bytes_per_launch"] + t["hbm_write_bytes_per_launch"])
    assert math.isfinite(t["occupancy_waves_per_simd_time_weighted"])


def test_iteration_log_lines(tmp_path):
    """One JSON object per iteration with the rays, rates, V_I, C_I, the
    proxy 1/(V_I C_I) and the mean first-hit counts."""
    from types import SimpleNamespace as NS

    from paper_2410_20429_amd import iterlog
    p = NS(spp=2, alloc=1)
    st = NS(rays_camera=100, rays_ext=50, rays_shadow=30, rays_light=20, rays_conn=0, tiles=3,
            overflow_retries=1)
    us = NS(V_I=0.5, C_I=4.0)
    cm = np.zeros((2, 5, 3), np.float32)
    cm[..., 0], cm[..., 1], cm[..., 2] = 1.0, 2.0, 0.5
    cm[0, 0, 0] = 11.0  # mean over 10 pixels: 2.0
    path = tmp_path / "log.jsonl"
    log = iterlog.IterationLog(path)
    log.write(iterlog.record(7, p, st, us, 0.5, 5, 2, cm))
    log.write(iterlog.record(8, p, st, NS(V_I=0.0, C_I=4.0), 0.5, 5, 2))
    log.close()
    a, b = [json.loads(x) for x in open(path).read().splitlines()]
    assert a["iteration"] == 7 and a["rays"] == 200 and a["tiles"] == 3
    assert a["mrays_per_s"] == pytest.approx(200 / 0.5 / 1e6)
    assert a["mpaths_per_s"] == pytest.approx(5 * 2 * 2 / 0.5 / 1e6)
    assert a["proxy_efficiency"] == pytest.approx(0.5)
    assert a["mean_first_hit_counts"] == pytest.approx([2.0, 2.0, 0.5])
    assert b["proxy_efficiency"] is None and "mean_first_hit_counts" not in b
