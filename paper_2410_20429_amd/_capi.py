"""ctypes binding of the C ABI in include/mars.h: argument marshalling only.

Every function here has the name of the C entry point it calls.  Work runs
in the HIP library; a missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmars.so")

MARS_OK, MARS_E_ARG, MARS_E_OOM, MARS_E_HIP, MARS_E_STATE, MARS_E_OVERFLOW, MARS_E_NONFINITE, \
    MARS_E_IO = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "MARS_OK", -1: "MARS_E_ARG", -2: "MARS_E_OOM", -3: "MARS_E_HIP",
                -4: "MARS_E_STATE", -5: "MARS_E_OVERFLOW", -6: "MARS_E_NONFINITE", -7: "MARS_E_IO"}
MODE_PT, MODE_PT_GUIDED, MODE_BDPT = 0, 1, 2
ALLOC_CLASSIC, ALLOC_MARS, ALLOC_FIXED, ALLOC_MLP, ALLOC_EARS = 0, 1, 2, 3, 4
IMAGE_MEAN, IMAGE_IVW, IMAGE_LAST = 0, 1, 2
SCENE_MLP = 1
SCENE_LP_LENGTHS = 2
BATCH_UPDATE, BATCH_NO_GRAPH = 1, 2

alloc_fn = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
free_fn = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class mars_ctx_desc(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", alloc_fn),
                ("free", free_fn), ("user", C.c_void_p)]


class mars_scene_desc(C.Structure):
    _fields_ = [("V", C.c_void_p), ("tri_mat", C.c_void_p), ("mats", C.c_void_p),
                ("camera", C.c_void_p), ("n_tris", C.c_int32), ("n_mats", C.c_int32),
                ("width", C.c_int32), ("height", C.c_int32), ("mode", C.c_int32),
                ("max_depth", C.c_int32), ("max_cells", C.c_int32), ("max_tree_depth", C.c_int32),
                ("split_visits", C.c_int32), ("nee_enabled", C.c_int32), ("seed", C.c_uint64),
                ("queue_capacity", C.c_int64), ("tile_roots", C.c_int32), ("flags", C.c_int32)]


class mars_iter_params(C.Structure):
    _fields_ = [("iteration", C.c_int32), ("spp", C.c_int32), ("alloc", C.c_int32),
                ("budget_aware", C.c_int32), ("rr_start", C.c_int32), ("fixed_scale", C.c_int32),
                ("clamp_lo", C.c_float), ("clamp_hi", C.c_float), ("stat_clamp", C.c_float),
                ("center_jitter", C.c_int32), ("debug_depth", C.c_int32), ("lp_stride", C.c_int32),
                ("rounding", C.c_int32)]


class mars_iter_stats(C.Structure):
    _fields_ = [("rays_camera", C.c_uint64), ("rays_ext", C.c_uint64), ("rays_shadow", C.c_uint64),
                ("rays_light", C.c_uint64), ("rays_conn", C.c_uint64), ("vertices", C.c_uint64),
                ("samples", C.c_uint64), ("tiles", C.c_int32), ("overflow_retries", C.c_int32),
                ("ms", C.c_double)]

    def total_rays(self):
        return self.rays_camera + self.rays_ext + self.rays_shadow + self.rays_light + self.rays_conn

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mars_update_stats(C.Structure):
    _fields_ = [("V_I", C.c_double), ("C_I", C.c_double), ("n_cells_before", C.c_int32),
                ("n_cells_after", C.c_int32), ("n_excluded", C.c_int32), ("reserved", C.c_int32)]


class mars_vertex_rec(C.Structure):
    _fields_ = [("root", C.c_uint32), ("depth", C.c_uint32), ("stream_lo", C.c_uint32),
                ("stream_hi", C.c_uint32), ("cell", C.c_uint32), ("beta", C.c_float * 3),
                ("gamma", C.c_uint32 * 3), ("T", C.c_float * 3), ("beta_x", C.c_float * 2),
                ("gamma_x", C.c_uint32 * 2)]


P = C.c_void_p
I32 = C.c_int32
PI32 = C.POINTER(C.c_int32)
SIGNATURES = {
    "mars_create": [C.POINTER(mars_ctx_desc), C.POINTER(C.c_void_p)],
    "mars_destroy": [P],
    "mars_scene_upload": [P, C.POINTER(mars_scene_desc), PI32],
    "mars_scene_release": [P, I32],
    "mars_render_iteration": [P, I32, C.POINTER(mars_iter_params), C.POINTER(mars_iter_stats)],
    "mars_render_batch": [P, P, I32, C.POINTER(mars_iter_params), C.POINTER(mars_iter_stats)],
    "mars_iterate_batch": [P, P, I32, C.POINTER(mars_iter_params), I32, P, P],
    "mars_scene_configure": [P, I32, C.c_int64, I32],
    "mars_scene_configure_queues": [P, I32, C.c_int64, C.c_int64, I32],
    "mars_scene_query": [P, I32, C.POINTER(C.c_int64), PI32, C.POINTER(C.c_double)],
    "mars_scene_query_queues": [P, I32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "mars_autotune": [P, P, I32, C.POINTER(mars_iter_params), C.c_int64, C.c_char_p, P, P, P, P,
                      P],
    "mars_update_counts": [P, I32, C.POINTER(mars_iter_params), C.POINTER(mars_update_stats)],
    "mars_set_fixed_counts": [P, I32, P, I32],
    "mars_set_itilde": [P, I32, P],
    "mars_set_hist": [P, I32, I32, P, P],
    "mars_write_cells": [P, I32, I32, P, P, P],
    "mars_update_cells_only": [P, I32, C.c_double, C.c_double],
    "mars_refine_only": [P, I32, PI32],
    "mars_read_image": [P, I32, I32, P, I32],
    "mars_read_count_map": [P, I32, P, I32],
    "mars_read_sample_radiance": [P, I32, P, I32],
    "mars_read_itilde": [P, I32, P, I32],
    "mars_num_cells": [P, I32, PI32, PI32],
    "mars_read_cells": [P, I32, P, P, P, P],
    "mars_read_cells_x": [P, I32, P, P],
    "mars_write_cells_x": [P, I32, I32, P, P],
    "mars_read_nodes": [P, I32, P],
    "mars_read_hist": [P, I32, P, P],
    "mars_debug_vertices": [P, I32, P, I32, PI32],
    "mars_checkpoint_save": [P, I32, C.c_char_p],
    "mars_checkpoint_load": [P, I32, C.c_char_p],
    "mars_probe": [P, I32, I32, P, P],
    "mars_profile_enable": [P, I32],
    "mars_profile_enable_mask": [P, C.c_uint64],
    "mars_profile_read": [P, P, P, I32, PI32],
    "mars_trace_counting": [P, I32],
    "mars_read_trace_counts": [P, P],
    "mars_mlp_train": [P, I32, I32, I32, C.c_float, P, PI32],
    "mars_mlp_read_params": [P, I32, P],
    "mars_mlp_write_params": [P, I32, P],
    "mars_mlp_forward": [P, I32, P, I32, P],
    "mars_mlp_grad": [P, I32, P, P, P, I32, P, P],
    "mars_mlp_apply_grad": [P, I32, P, C.c_float],
    "mars_mlp_grad_noalloc": [P, I32, P, P, P, I32, P],
    "mars_mlp_write_records": [P, I32, P, P, P, P, I32],
    "mars_mlp_targets_only": [P, I32],
    "mars_mlp_read_train": [P, I32, P, P, P, I32, PI32],
}

_lib = None


def lib():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.mars_last_error.argtypes = [P]
        L.mars_last_error.restype = C.c_char_p
        L.mars_profile_kernel_name.argtypes = [I32]
        L.mars_profile_kernel_name.restype = C.c_char_p
        L.mars_mlp_num_params.argtypes = []
        L.mars_mlp_num_params.restype = C.c_int32
        L.mars_version.argtypes = []
        L.mars_version.restype = C.c_char_p
        _lib = L
    return _lib


class MarsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, ctx=None):
    if code != MARS_OK:
        msg = lib().mars_last_error(ctx).decode() if ctx else ""
        raise MarsError(code, msg)


def _call(name, ctx, *args):
    check(getattr(lib(), name)(ctx, *args), ctx)


# ---- thin wrappers with the C names -----------------------------------------
def mars_create(device=0, stream=None, alloc=None, free=None, user=None):
    d = mars_ctx_desc(device, stream, alloc or alloc_fn(), free or free_fn(), user)
    out = C.c_void_p()
    check(lib().mars_create(C.byref(d), C.byref(out)))
    return out


def mars_destroy(ctx):
    check(lib().mars_destroy(ctx))


def mars_scene_upload(ctx, desc):
    sid = C.c_int32()
    _call("mars_scene_upload", ctx, C.byref(desc), C.byref(sid))
    return sid.value


def mars_scene_release(ctx, sid):
    _call("mars_scene_release", ctx, sid)


def mars_render_iteration(ctx, sid, params):
    st = mars_iter_stats()
    _call("mars_render_iteration", ctx, sid, C.byref(params), C.byref(st))
    return st


def mars_render_batch(ctx, sids, params):
    arr = (C.c_int32 * len(sids))(*sids)
    st = mars_iter_stats()
    _call("mars_render_batch", ctx, C.cast(arr, C.c_void_p), len(sids), C.byref(params),
          C.byref(st))
    return st


def mars_iterate_batch(ctx, sids, params, flags):
    n = len(sids)
    arr = (C.c_int32 * n)(*sids)
    its = (mars_iter_stats * n)()
    ups = (mars_update_stats * n)()
    _call("mars_iterate_batch", ctx, C.cast(arr, C.c_void_p), n, C.byref(params), flags,
          C.cast(its, C.c_void_p), C.cast(ups, C.c_void_p))
    return list(its), list(ups)


def mars_scene_configure(ctx, sid, queue_capacity=0, tile_roots=0):
    _call("mars_scene_configure", ctx, sid, queue_capacity, tile_roots)


def mars_scene_configure_queues(ctx, sid, ray_capacity=0, shadow_capacity=0, tile_roots=0):
    _call("mars_scene_configure_queues", ctx, sid, ray_capacity, shadow_capacity, tile_roots)


def mars_scene_query(ctx, sid):
    cap, tile, peak = C.c_int64(), C.c_int32(), C.c_double()
    _call("mars_scene_query", ctx, sid, C.byref(cap), C.byref(tile), C.byref(peak))
    return cap.value, tile.value, peak.value


def mars_scene_query_queues(ctx, sid):
    cap, scap, pr, ps = C.c_int64(), C.c_int64(), C.c_double(), C.c_double()
    _call("mars_scene_query_queues", ctx, sid, C.byref(cap), C.byref(scap), C.byref(pr),
          C.byref(ps))
    return cap.value, scap.value, pr.value, ps.value


def mars_autotune(ctx, sids, params, mem_budget=0, cache_path=None):
    n = len(sids)
    arr = (C.c_int32 * n)(*sids)
    cap, tile, peak = (C.c_int64 * n)(), (C.c_int32 * n)(), (C.c_double * n)()
    scap, speak = (C.c_int64 * n)(), (C.c_double * n)()
    _call("mars_autotune", ctx, C.cast(arr, C.c_void_p), n, C.byref(params), mem_budget,
          cache_path.encode() if cache_path else None, C.cast(cap, C.c_void_p),
          C.cast(tile, C.c_void_p), C.cast(peak, C.c_void_p), C.cast(scap, C.c_void_p),
          C.cast(speak, C.c_void_p))
    return list(cap), list(tile), list(peak), list(scap), list(speak)


def mars_update_counts(ctx, sid, params):
    us = mars_update_stats()
    _call("mars_update_counts", ctx, sid, C.byref(params) if params is not None else None,
          C.byref(us))
    return us


def mars_set_fixed_counts(ctx, sid, beta_ptr, n):
    _call("mars_set_fixed_counts", ctx, sid, beta_ptr, n)


def mars_set_itilde(ctx, sid, ptr):
    _call("mars_set_itilde", ctx, sid, ptr)


def mars_set_hist(ctx, sid, n, pm_ptr, cdf_ptr):
    _call("mars_set_hist", ctx, sid, n, pm_ptr, cdf_ptr)


def mars_write_cells(ctx, sid, n, fac_ptr, acc_ptr, vis_ptr):
    _call("mars_write_cells", ctx, sid, n, fac_ptr, acc_ptr, vis_ptr)


def mars_update_cells_only(ctx, sid, V_I, C_I):
    _call("mars_update_cells_only", ctx, sid, float(V_I), float(C_I))


def mars_refine_only(ctx, sid):
    n = C.c_int32()
    _call("mars_refine_only", ctx, sid, C.byref(n))
    return n.value


def mars_read_image(ctx, sid, which, dst_ptr, dst_is_device=0):
    _call("mars_read_image", ctx, sid, which, dst_ptr, dst_is_device)


def mars_read_count_map(ctx, sid, dst_ptr, dst_is_device=0):
    _call("mars_read_count_map", ctx, sid, dst_ptr, dst_is_device)


def mars_read_sample_radiance(ctx, sid, dst_ptr, dst_is_device=0):
    _call("mars_read_sample_radiance", ctx, sid, dst_ptr, dst_is_device)


def mars_read_itilde(ctx, sid, dst_ptr, dst_is_device=0):
    _call("mars_read_itilde", ctx, sid, dst_ptr, dst_is_device)


def mars_num_cells(ctx, sid):
    a, b = C.c_int32(), C.c_int32()
    _call("mars_num_cells", ctx, sid, C.byref(a), C.byref(b))
    return a.value, b.value


def mars_read_cells(ctx, sid, fac_ptr, acc_ptr, vis_ptr, dep_ptr):
    _call("mars_read_cells", ctx, sid, fac_ptr, acc_ptr, vis_ptr, dep_ptr)


def mars_read_nodes(ctx, sid, ptr):
    _call("mars_read_nodes", ctx, sid, ptr)


def mars_read_cells_x(ctx, sid, fac_ptr, acc_ptr):
    _call("mars_read_cells_x", ctx, sid, fac_ptr, acc_ptr)


def mars_write_cells_x(ctx, sid, n, fac_ptr, acc_ptr):
    _call("mars_write_cells_x", ctx, sid, n, fac_ptr, acc_ptr)


def mars_read_hist(ctx, sid, pm_ptr, cdf_ptr):
    _call("mars_read_hist", ctx, sid, pm_ptr, cdf_ptr)


def mars_debug_vertices(ctx, sid, dst_ptr, cap):
    n = C.c_int32()
    _call("mars_debug_vertices", ctx, sid, dst_ptr, cap, C.byref(n))
    return n.value


def mars_checkpoint_save(ctx, sid, path):
    _call("mars_checkpoint_save", ctx, sid, path.encode())


def mars_checkpoint_load(ctx, sid, path):
    _call("mars_checkpoint_load", ctx, sid, path.encode())


def mars_probe(ctx, kind, n, in_ptr, out_ptr):
    _call("mars_probe", ctx, kind, n, in_ptr, out_ptr)


def mars_profile_enable(ctx, on):
    _call("mars_profile_enable", ctx, int(bool(on)))


def mars_profile_enable_mask(ctx, mask):
    _call("mars_profile_enable_mask", ctx, int(mask))


def mars_profile_read(ctx):
    import numpy as np
    nk = C.c_int32()
    ms = np.zeros(32, np.float64)
    cnt = np.zeros(32, np.uint64)
    _call("mars_profile_read", ctx, ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p),
          32, C.byref(nk))
    return {lib().mars_profile_kernel_name(k).decode(): (float(ms[k]), int(cnt[k]))
            for k in range(nk.value)}


def mars_profile_kernel_name(k):
    return lib().mars_profile_kernel_name(k).decode()


def mars_trace_counting(ctx, on):
    _call("mars_trace_counting", ctx, int(bool(on)))


def mars_read_trace_counts(ctx):
    out = (C.c_uint64 * 10)()
    _call("mars_read_trace_counts", ctx, C.cast(out, C.c_void_p))
    return list(out)


def mars_mlp_num_params():
    return lib().mars_mlp_num_params()


def mars_mlp_train(ctx, sid, steps, batch, lr):
    loss = C.c_float()
    n = C.c_int32()
    _call("mars_mlp_train", ctx, sid, steps, batch, float(lr), C.byref(loss), C.byref(n))
    return loss.value, n.value


def mars_mlp_read_params(ctx, sid, ptr):
    _call("mars_mlp_read_params", ctx, sid, ptr)


def mars_mlp_write_params(ctx, sid, ptr):
    _call("mars_mlp_write_params", ctx, sid, ptr)


def mars_mlp_forward(ctx, sid, x_ptr, n, y_ptr):
    _call("mars_mlp_forward", ctx, sid, x_ptr, n, y_ptr)


def mars_mlp_grad(ctx, sid, x_ptr, t_ptr, w_ptr, n, g_ptr):
    loss = C.c_float()
    _call("mars_mlp_grad", ctx, sid, x_ptr, t_ptr, w_ptr, n, g_ptr, C.byref(loss))
    return loss.value


def mars_mlp_apply_grad(ctx, sid, g_ptr, lr):
    _call("mars_mlp_apply_grad", ctx, sid, g_ptr, float(lr))


def mars_mlp_grad_noalloc(ctx, sid, x_ptr, t_ptr, w_ptr, n, g_ptr):
    """device pointers; enqueued on the context's stream, not waited for"""
    _call("mars_mlp_grad_noalloc", ctx, sid, x_ptr, t_ptr, w_ptr, n, g_ptr)


def mars_mlp_write_records(ctx, sid, pos_ptr, nrm_ptr, t_ptr, pix_ptr, n):
    _call("mars_mlp_write_records", ctx, sid, pos_ptr, nrm_ptr, t_ptr, pix_ptr, n)


def mars_mlp_targets_only(ctx, sid):
    _call("mars_mlp_targets_only", ctx, sid)


def mars_mlp_read_train(ctx, sid, x_ptr, t_ptr, w_ptr, cap):
    n = C.c_int32()
    _call("mars_mlp_read_train", ctx, sid, x_ptr, t_ptr, w_ptr, cap, C.byref(n))
    return n.value


def mars_version():
    return lib().mars_version().decode()
