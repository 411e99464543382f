"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
oracle.c and a stand-alone driver (oracle/sanitize_driver.c) are built with
gcc's sanitizers, every report fatal, and run a short MARS schedule on small
scenes of each mode.  The run must end cleanly (no memory error, undefined
behaviour or leak) and reproduce, bit for bit, the per-sample radiance of the
oracle library (one thread) on the same schedule."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import scenegen
from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "sanitize_driver")
    cmd = ["gcc", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-Wno-unknown-pragmas", "-o", exe, os.path.join(ORACLE, "oracle.c"),
           os.path.join(ORACLE, "sanitize_driver.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("gcc sanitizer runtimes not installed")
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _write_scene(path, sc):
    V = np.ascontiguousarray(sc["V"], np.float32)
    tm = np.ascontiguousarray(sc["tri_mat"], np.uint32)
    mats = np.ascontiguousarray(sc["mats"], np.float32)
    cam = np.ascontiguousarray(sc["camera"], np.float32)
    with open(path, "wb") as f:
        np.array([V.shape[0], mats.shape[0], cam.size, sc["width"], sc["height"]],
                 np.int32).tofile(f)
        V.tofile(f)
        tm.tofile(f)
        mats.tofile(f)
        cam.tofile(f)


CASES = {
    "pt_cornell": (lambda: scenegen.make_cornell(16, 16), orc.MODE_PT, 5, 1, 50.0),
    "guided_heightfield": (lambda: scenegen.make_heightfield_scene(seed=2, width=16, height=16,
                                                                   grid=12, n_boxes=6),
                           orc.MODE_PT_GUIDED, 6, 1, 50.0),
    "bdpt_interior": (lambda: scenegen.make_interior(seed=3, n_pieces=12, tess=1, width=24,
                                                     height=16), orc.MODE_BDPT, 6, 1, 0.0),
    "bdpt_lp_lengths": (lambda: scenegen.make_interior(seed=3, n_pieces=12, tess=1, width=24,
                                                       height=16), orc.MODE_BDPT, 6, 3, 0.0),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_oracle_clean_under_sanitizers(driver, tmp_path, case):
    make, mode, depth, lp_classes, stat_clamp = CASES[case]
    sc = make()
    iters, spp = 4, 2
    scene_file, out_file = str(tmp_path / "scene.bin"), str(tmp_path / "radiance.bin")
    _write_scene(scene_file, sc)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=66",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=67")
    r = subprocess.run([driver, scene_file, str(mode), str(depth), str(lp_classes), str(iters),
                        str(spp), repr(stat_clamp), out_file], capture_output=True, text=True,
                       env=env, timeout=600)
    if r.returncode != 0 and "LeakSanitizer does not work under ptrace" in r.stderr:
        pytest.skip("LeakSanitizer unavailable here")
    assert r.returncode == 0, r.stderr[-4000:]
    got = np.fromfile(out_file, np.float32).reshape(iters, -1, 3)
    # the same schedule on the oracle library, one thread (its reductions then
    # sum in the driver's order)
    old = orc.set_threads(0)  # 0: query only
    orc.set_threads(1)
    try:
        o = orc.Oracle(sc, mode=mode, max_depth=depth, lp_classes=lp_classes)
        for it in range(iters):
            p = orc.Oracle.params(iteration=it, spp=spp, stat_clamp=stat_clamp,
                                  alloc=orc.ALLOC_CLASSIC if it == 0 else orc.ALLOC_MARS)
            o.render_iteration(p)
            want = o.sample_radiance()
            assert np.array_equal(got[it].view(np.uint32), want.view(np.uint32)), (case, it)
            o.update(p)
        o.close()
    finally:
        orc.set_threads(old)
