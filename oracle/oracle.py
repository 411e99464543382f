"""ctypes wrapper of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

MODE_PT, MODE_PT_GUIDED, MODE_BDPT = 0, 1, 2
ALLOC_CLASSIC, ALLOC_MARS, ALLOC_FIXED, ALLOC_EARS = 0, 1, 2, 4


class Config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("max_depth", C.c_int32), ("max_cells", C.c_int32),
                ("max_tree_depth", C.c_int32), ("split_visits", C.c_int32),
                ("nee_enabled", C.c_int32), ("seed", C.c_uint64), ("lp_classes", C.c_int32)]


class IterParams(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("spp", C.c_int32), ("alloc", C.c_int32),
                ("budget_aware", C.c_int32), ("rr_start", C.c_int32), ("fixed_scale", C.c_int32),
                ("clamp_lo", C.c_float), ("clamp_hi", C.c_float), ("stat_clamp", C.c_float),
                ("center_jitter", C.c_int32), ("debug_depth", C.c_int32), ("lp_stride", C.c_int32),
                ("rounding", C.c_int32)]


class IterStats(C.Structure):
    _fields_ = [("rays_camera", C.c_uint64), ("rays_ext", C.c_uint64), ("rays_shadow", C.c_uint64),
                ("rays_light", C.c_uint64), ("rays_conn", C.c_uint64), ("vertices", C.c_uint64),
                ("samples", C.c_uint64)]

    def total_rays(self):
        return self.rays_camera + self.rays_ext + self.rays_shadow + self.rays_light + self.rays_conn

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class UpdateStats(C.Structure):
    _fields_ = [("V_I", C.c_double), ("C_I", C.c_double), ("n_cells_before", C.c_int32),
                ("n_cells_after", C.c_int32), ("n_excluded", C.c_int32)]


class VertexRec(C.Structure):
    _fields_ = [("root", C.c_uint32), ("depth", C.c_uint32), ("stream_lo", C.c_uint32),
                ("stream_hi", C.c_uint32), ("cell", C.c_uint32), ("beta", C.c_float * 3),
                ("gamma", C.c_uint32 * 3), ("T", C.c_float * 3), ("beta_x", C.c_float * 2),
                ("gamma_x", C.c_uint32 * 2)]


VERTEX_DTYPE = np.dtype([("root", "<u4"), ("depth", "<u4"), ("stream_lo", "<u4"),
                         ("stream_hi", "<u4"), ("cell", "<u4"), ("beta", "<f4", 3),
                         ("gamma", "<u4", 3), ("T", "<f4", 3), ("beta_x", "<f4", 2),
                         ("gamma_x", "<u4", 2)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        fp = C.POINTER(C.c_float)
        L.orc_create.restype = P
        L.orc_create.argtypes = [P, P, C.c_int32, P, C.c_int32, P, C.c_int32, C.c_int32,
                                 C.POINTER(Config)]
        L.orc_destroy.argtypes = [P]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_set_threads.restype = C.c_int32
        L.orc_render_iteration.argtypes = [P, C.POINTER(IterParams), C.POINTER(IterStats)]
        L.orc_update.argtypes = [P, C.POINTER(IterParams), C.POINTER(UpdateStats)]
        for n in ["orc_num_cells", "orc_num_nodes"]:
            getattr(L, n).argtypes = [P]
            getattr(L, n).restype = C.c_int32
        L.orc_read_nodes.argtypes = [P, P]
        L.orc_read_sample_radiance.argtypes = [P, P]
        L.orc_read_image.argtypes = [P, C.c_int32, P]
        L.orc_read_Itilde.argtypes = [P, P]
        L.orc_read_count_map.argtypes = [P, P]
        L.orc_read_cells.argtypes = [P, P, P, P, P]
        L.orc_read_hist.argtypes = [P, P, P]
        L.orc_read_debug.argtypes = [P, P, C.c_int32]
        L.orc_read_debug.restype = C.c_int32
        L.orc_write_cells.argtypes = [P, C.c_int32, P, P, P]
        L.orc_lp_classes.argtypes = [P]
        L.orc_lp_classes.restype = C.c_int32
        L.orc_read_cells_x.argtypes = [P, P, P]
        L.orc_write_cells_x.argtypes = [P, C.c_int32, P, P]
        L.orc_set_Itilde.argtypes = [P, P]
        L.orc_set_pixel_subset.argtypes = [P, P, C.c_int32]
        L.orc_set_fixed_beta.argtypes = [P, P, C.c_int32]
        L.orc_set_record_depth.argtypes = [P, C.c_int32]
        L.orc_set_hist.argtypes = [P, C.c_int32, P, P]
        L.orc_update_cells_only.argtypes = [P, C.c_double, C.c_double]
        L.orc_update_cells_only.restype = C.c_int32
        L.orc_update_cells_ears.argtypes = [P, C.c_double, C.c_double]
        L.orc_update_cells_ears.restype = C.c_int32
        L.orc_refine_only.argtypes = [P]
        L.orc_refine_only.restype = C.c_int32
        L.orc_philox.argtypes = [C.c_uint32, C.c_uint32, P, P]
        L.orc_sincos2pi.argtypes = [C.c_float, fp, fp]
        L.orc_alg1.argtypes = [P, C.c_float, P]
        L.orc_alg1_enumerate.argtypes = [P, C.c_uint32, P, P, P]
        L.orc_cell_beta.argtypes = [P, C.POINTER(IterParams), C.c_uint32, P, P, C.c_int32, P]
        L.orc_bsdf_sample.argtypes = [P, P, P, C.c_float, C.c_float, P]
        L.orc_bsdf_sample.restype = C.c_int32
        L.orc_bsdf_eval.argtypes = [P, P, P, P, P, fp]
        L.orc_guided_sample.argtypes = [P, P, C.c_float, C.c_float, C.c_float, P]
        L.orc_guided_pdf.argtypes = [P, P]
        L.orc_guided_pdf.restype = C.c_float
        L.orc_mis.argtypes = [C.c_int32, P, P, P, P]
        L.orc_octree_lookup.argtypes = [P, P, C.POINTER(C.c_uint32)]
        L.orc_octree_lookup.restype = C.c_uint32
        L.orc_intersect.argtypes = [P, P, P, C.c_float, fp, C.POINTER(C.c_uint32)]
        L.orc_intersect.restype = C.c_int32
        L.orc_bdpt_weights.argtypes = [P, C.POINTER(IterParams), P, P, C.c_int32, P, P]
        L.orc_camera_ray.argtypes = [P, C.c_int32, C.c_int32, C.c_float, C.c_float, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n):
    return lib().orc_set_threads(int(n))


class Oracle:
    """Plain CPU implementation of the hot path, one scene per instance."""

    def __init__(self, scene, mode=MODE_PT, max_depth=5, max_cells=65536, max_tree_depth=8,
                 split_visits=32, nee=True, seed=1, lp_classes=1):
        L = lib()
        self.scene = scene
        self.V = np.ascontiguousarray(scene["V"], np.float32)
        self.tm = np.ascontiguousarray(scene["tri_mat"], np.uint32)
        self.mats = np.ascontiguousarray(scene["mats"], np.float32)
        self.cam = np.ascontiguousarray(scene["camera"], np.float32)
        self.W, self.H = int(scene["width"]), int(scene["height"])
        self.cfg = Config(mode, max_depth, max_cells, max_tree_depth, split_visits, int(bool(nee)),
                          seed, int(lp_classes))
        self.h = L.orc_create(_p(self.V), _p(self.tm), self.V.shape[0], _p(self.mats),
                              self.mats.shape[0], _p(self.cam), self.W, self.H, C.byref(self.cfg))
        if not self.h:
            raise ValueError("oracle: invalid scene")
        self.spp = 0

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def params(iteration=0, spp=1, alloc=ALLOC_CLASSIC, budget_aware=True, rr_start=5,
               fixed_scale=False, clamp_lo=0.05, clamp_hi=20.0, stat_clamp=50.0,
               center_jitter=False, debug_depth=0, lp_stride=7919, rounding=0):
        return IterParams(iteration, spp, alloc, int(budget_aware), rr_start, int(fixed_scale),
                          clamp_lo, clamp_hi, stat_clamp, int(center_jitter), debug_depth, lp_stride,
                          int(rounding))

    def render_iteration(self, p):
        st = IterStats()
        rc = lib().orc_render_iteration(self.h, C.byref(p), C.byref(st))
        if rc != 0:
            raise RuntimeError(f"oracle render failed: {rc}")
        self.spp = p.spp
        self._last_params = p
        return st

    def update(self, p=None):
        p = p or self._last_params
        us = UpdateStats()
        rc = lib().orc_update(self.h, C.byref(p), C.byref(us))
        if rc != 0:
            raise RuntimeError(f"oracle update failed: {rc}")
        return us

    # ---- read-back ----
    @property
    def ncells(self):
        return lib().orc_num_cells(self.h)

    def nodes(self):
        n = lib().orc_num_nodes(self.h)
        a = np.zeros(n, np.uint32)
        lib().orc_read_nodes(self.h, _p(a))
        return a

    def sample_radiance(self):
        a = np.zeros((self.H * self.W * self.spp, 3), np.float32)
        lib().orc_read_sample_radiance(self.h, _p(a))
        return a

    def image(self, which=0):
        a = np.zeros((self.H, self.W, 3), np.float32)
        lib().orc_read_image(self.h, int(which), _p(a))
        return a

    def itilde(self):
        a = np.zeros((self.H, self.W, 3), np.float32)
        lib().orc_read_Itilde(self.h, _p(a))
        return a

    def count_map(self):
        a = np.zeros((self.H, self.W, 3), np.float32)
        lib().orc_read_count_map(self.h, _p(a))
        return a

    def cells(self):
        n = self.ncells
        fac = np.zeros((n, 2, 3, 3), np.float32)
        acc = np.zeros((n, 3, 8), np.float64)
        vis = np.zeros(n, np.uint32)
        dep = np.zeros(n, np.uint32)
        lib().orc_read_cells(self.h, _p(fac), _p(acc), _p(vis), _p(dep))
        return {"factors": fac, "acc": acc, "visits": vis, "depth": dep}

    @property
    def lp_classes(self):
        return lib().orc_lp_classes(self.h)

    def cells_x(self):
        """Per-length light-path budgets: factors [n][2][2][3] and
        accumulators [n][2][8] of techniques 3 (y_2) and 4 (y_3+)."""
        n = self.ncells
        fac = np.zeros((n, 2, 2, 3), np.float32)
        acc = np.zeros((n, 2, 8), np.float64)
        lib().orc_read_cells_x(self.h, _p(fac), _p(acc))
        return {"factors": fac, "acc": acc}

    def write_cells_x(self, factors=None, acc=None):
        f = None if factors is None else np.ascontiguousarray(factors, np.float32)
        a = None if acc is None else np.ascontiguousarray(acc, np.float64)
        lib().orc_write_cells_x(self.h, self.ncells, None if f is None else _p(f),
                                None if a is None else _p(a))

    def hist(self):
        n = self.ncells
        pm = np.zeros((n, 64), np.float32)
        cdf = np.zeros((n, 64), np.float32)
        lib().orc_read_hist(self.h, _p(pm), _p(cdf))
        return pm, cdf

    def debug_vertices(self):
        n = lib().orc_read_debug(self.h, None, 0)
        a = np.zeros(n, VERTEX_DTYPE)
        if n:
            lib().orc_read_debug(self.h, _p(a), n)
        return a

    # ---- write-in ----
    def write_cells(self, factors=None, acc=None, visits=None):
        n = self.ncells
        f = None if factors is None else np.ascontiguousarray(factors, np.float32)
        a = None if acc is None else np.ascontiguousarray(acc, np.float64)
        v = None if visits is None else np.ascontiguousarray(visits, np.uint32)
        lib().orc_write_cells(self.h, n, None if f is None else _p(f), None if a is None else _p(a),
                              None if v is None else _p(v))

    def set_itilde(self, it):
        it = np.ascontiguousarray(it, np.float32).reshape(self.H, self.W, 3)
        lib().orc_set_Itilde(self.h, _p(it))

    def set_pixel_subset(self, pix):
        if pix is None:
            lib().orc_set_pixel_subset(self.h, None, 0)
            return
        a = np.ascontiguousarray(pix, np.int32)
        lib().orc_set_pixel_subset(self.h, _p(a), a.shape[0])

    def set_fixed_beta(self, beta):
        b = np.ascontiguousarray(beta, np.float32).reshape(-1, 3)
        lib().orc_set_fixed_beta(self.h, _p(b), b.shape[0])

    def set_record_depth(self, depth):
        """(tests) sample statistics only from vertices up to `depth`; 0: all"""
        lib().orc_set_record_depth(self.h, int(depth))

    def set_hist(self, pm, cdf):
        pm = np.ascontiguousarray(pm, np.float32)
        cdf = np.ascontiguousarray(cdf, np.float32)
        lib().orc_set_hist(self.h, pm.shape[0], _p(pm), _p(cdf))

    def update_cells_only(self, V_I, C_I, ears=False):
        f = lib().orc_update_cells_ears if ears else lib().orc_update_cells_only
        return f(self.h, float(V_I), float(C_I))

    def refine_only(self):
        return lib().orc_refine_only(self.h)

    def cell_beta(self, p, cell, T, It, depth=1):
        T = np.ascontiguousarray(T, np.float32)
        It = np.ascontiguousarray(It, np.float32)
        b = np.zeros(3, np.float32)
        lib().orc_cell_beta(self.h, C.byref(p), int(cell), _p(T), _p(It), int(depth), _p(b))
        return b

    # ---- geometry probes ----
    def octree_lookup(self, p):
        p = np.ascontiguousarray(p, np.float32)
        d = C.c_uint32()
        c = lib().orc_octree_lookup(self.h, _p(p), C.byref(d))
        return c, d.value

    def intersect(self, o, d, tmax=np.inf):
        o = np.ascontiguousarray(o, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        t = C.c_float()
        pr = C.c_uint32()
        hit = lib().orc_intersect(self.h, _p(o), _p(d), float(tmax), C.byref(t), C.byref(pr))
        return (t.value, pr.value) if hit else (None, None)

    def bdpt_weights(self, p, P, prims, It):
        P = np.ascontiguousarray(P, np.float32)
        prims = np.ascontiguousarray(prims, np.uint32)
        It = np.ascontiguousarray(It, np.float32)
        k = P.shape[0] - 1
        out = np.zeros(k, np.float32)
        lib().orc_bdpt_weights(self.h, C.byref(p), _p(P), _p(prims), k, _p(It), _p(out))
        return out

    def camera_ray(self, px, py, jx=0.5, jy=0.5):
        o = np.zeros(3, np.float32)
        d = np.zeros(3, np.float32)
        lib().orc_camera_ray(self.h, px, py, jx, jy, _p(o), _p(d))
        return o, d


# ---- building blocks ----
def philox(key, ctr):
    c = np.ascontiguousarray(ctr, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(int(key[0]), int(key[1]), _p(c), _p(out))
    return out


def sincos2pi(u):
    s, c = C.c_float(), C.c_float()
    lib().orc_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def alg1(beta, u):
    b = np.ascontiguousarray(beta, np.float32)
    g = np.zeros(3, np.uint32)
    lib().orc_alg1(_p(b), float(u), _p(g))
    return g


def alg1_enumerate(beta, n):
    b = np.ascontiguousarray(beta, np.float32)
    mean = np.zeros(3, np.float64)
    tot = np.zeros(2, np.uint32)
    r = np.zeros(2, np.float32)
    lib().orc_alg1_enumerate(_p(b), int(n), _p(mean), _p(tot), _p(r))
    return mean, tot, r


def bsdf_sample(mat, n, wo, u0, u1):
    m = np.ascontiguousarray(mat, np.float32)
    n = np.ascontiguousarray(n, np.float32)
    wo = np.ascontiguousarray(wo, np.float32)
    wi = np.zeros(3, np.float32)
    ok = lib().orc_bsdf_sample(_p(m), _p(n), _p(wo), float(u0), float(u1), _p(wi))
    return bool(ok), wi


def bsdf_eval(mat, n, wo, wi):
    m = np.ascontiguousarray(mat, np.float32)
    arrs = [np.ascontiguousarray(x, np.float32) for x in (n, wo, wi)]
    f = np.zeros(3, np.float32)
    pdf = C.c_float()
    lib().orc_bsdf_eval(_p(m), _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(f), C.byref(pdf))
    return f, pdf.value


def guided_sample(pm, cdf, u0, u1, u2):
    pm = np.ascontiguousarray(pm, np.float32)
    cdf = np.ascontiguousarray(cdf, np.float32)
    wi = np.zeros(3, np.float32)
    lib().orc_guided_sample(_p(pm), _p(cdf), float(u0), float(u1), float(u2), _p(wi))
    return wi


def guided_pdf(pm, wi):
    pm = np.ascontiguousarray(pm, np.float32)
    wi = np.ascontiguousarray(wi, np.float32)
    return lib().orc_guided_pdf(_p(pm), _p(wi))


def mis(aware, beta, p):
    b = np.ascontiguousarray(beta, np.float32)
    pp = np.ascontiguousarray(p, np.float32)
    wd = np.zeros(3, np.float32)
    wi = np.zeros(3, np.float32)
    lib().orc_mis(int(aware), _p(b), _p(pp), _p(wd), _p(wi))
    return wd, wi


def run_schedule(orc, n_iter, warmup=1, spp=1, budget_aware=True, stat_clamp=None, rr_start=5,
                 clamp_hi=20.0, spp_schedule=None, on_iter=None):
    """Iterative rendering: `warmup` classic-RR iterations, then MARS
    iterations; each followed by the update step."""
    if stat_clamp is None:
        stat_clamp = 0.0 if orc.cfg.mode == MODE_BDPT else 50.0
    hist = []
    for i in range(n_iter):
        s = spp_schedule(i) if spp_schedule else spp
        p = Oracle.params(iteration=i, spp=s, alloc=ALLOC_CLASSIC if i < warmup else ALLOC_MARS,
                          budget_aware=budget_aware, rr_start=rr_start, stat_clamp=stat_clamp,
                          clamp_hi=clamp_hi)
        st = orc.render_iteration(p)
        us = orc.update(p)
        hist.append((st.as_dict(), us.V_I, us.C_I, us.n_cells_after))
        if on_iter:
            on_iter(i, st, us)
    return hist
