"""Python front end of the MARS library: numpy in/out, PyTorch for device
memory (caching allocator) and the HIP stream.  All work runs in the HIP
library behind the C ABI."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from ._capi import (ALLOC_CLASSIC, ALLOC_EARS, ALLOC_FIXED, ALLOC_MARS, ALLOC_MLP, IMAGE_IVW,  # noqa: F401
                    IMAGE_LAST, IMAGE_MEAN, MODE_BDPT, MODE_PT, MODE_PT_GUIDED, SCENE_MLP, MarsError,
                    BATCH_NO_GRAPH, BATCH_UPDATE, SCENE_LP_LENGTHS)

VERTEX_DTYPE = np.dtype([("root", "<u4"), ("depth", "<u4"), ("stream_lo", "<u4"),
                         ("stream_hi", "<u4"), ("cell", "<u4"), ("beta", "<f4", 3),
                         ("gamma", "<u4", 3), ("T", "<f4", 3), ("beta_x", "<f4", 2),
                         ("gamma_x", "<u4", 2)])


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    """One HIP device + stream.  With torch_memory=True device buffers come
    from PyTorch's caching allocator on the current torch stream."""

    def __init__(self, device=0, torch_memory=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch")
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self._keep = []
        alloc = free = None
        if torch_memory:
            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device,
                                                              self.stream.cuda_stream)
                except Exception:  # out of memory is reported as NULL
                    return None

            def _free(ptr, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            alloc, free = capi.alloc_fn(_alloc), capi.free_fn(_free)
            self._keep += [alloc, free]
        self.h = capi.mars_create(device, C.c_void_p(self.stream.cuda_stream), alloc, free)

    def close(self):
        if getattr(self, "h", None):
            capi.mars_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on=True, kernels=None):
        """Per-kernel HIP-event timing; `kernels` (names) limits it to those."""
        if kernels is None or not on:
            capi.mars_profile_enable(self.h, on)
            return
        names = {capi.mars_profile_kernel_name(k): k for k in range(64)}
        mask = 0
        for name in kernels:
            if name not in names:
                raise ValueError(f"unknown kernel {name!r}")
            mask |= 1 << names[name]
        capi.mars_profile_enable_mask(self.h, mask)

    def profile_read(self):
        return capi.mars_profile_read(self.h)

    def trace_counting(self, on=True):
        capi.mars_trace_counting(self.h, on)

    def trace_counts(self):
        return capi.mars_read_trace_counts(self.h)

    def probe(self, kind, inp, out_shape, out_dtype):
        inp = np.ascontiguousarray(inp)
        out = np.zeros(out_shape, out_dtype)
        capi.mars_probe(self.h, kind, out.shape[0], _p(inp), _p(out))
        return out


def iter_params(iteration=0, spp=1, alloc=ALLOC_CLASSIC, budget_aware=True, rr_start=5,
                fixed_scale=False, clamp_lo=0.05, clamp_hi=20.0, stat_clamp=50.0,
                center_jitter=False, debug_depth=0, lp_stride=7919, rounding=0):
    return capi.mars_iter_params(iteration, spp, alloc, int(budget_aware), rr_start,
                                 int(fixed_scale), clamp_lo, clamp_hi, stat_clamp,
                                 int(center_jitter), debug_depth, lp_stride, int(rounding))


class Scene:
    """A scene uploaded to the GPU with its cache and image state."""

    def __init__(self, ctx: Context, scene: dict, mode=MODE_PT, max_depth=5, max_cells=65536,
                 max_tree_depth=8, split_visits=32, nee=True, seed=1, queue_capacity=0,
                 tile_roots=0, mlp=False, lp_lengths=False):
        self.ctx = ctx
        self.V = np.ascontiguousarray(scene["V"], np.float32)
        self.tm = np.ascontiguousarray(scene["tri_mat"], np.uint32)
        self.mats = np.ascontiguousarray(scene["mats"], np.float32)
        self.cam = np.ascontiguousarray(scene["camera"], np.float32)
        self.W, self.H = int(scene["width"]), int(scene["height"])
        self.mode = mode
        self.max_depth = int(max_depth)
        d = capi.mars_scene_desc(_p(self.V), _p(self.tm), _p(self.mats), _p(self.cam),
                                 self.V.shape[0], self.mats.shape[0], self.W, self.H, mode,
                                 max_depth, max_cells, max_tree_depth, split_visits, int(bool(nee)),
                                 seed, int(queue_capacity), int(tile_roots),
                                 (SCENE_MLP if mlp else 0) | (SCENE_LP_LENGTHS if lp_lengths else 0))
        self.id = capi.mars_scene_upload(ctx.h, d)
        self.spp = 0
        self._last = None

    def release(self):
        if self.id is not None and self.ctx.h:
            capi.mars_scene_release(self.ctx.h, self.id)
            self.id = None

    # ---- iteration ----
    def render_iteration(self, params):
        st = capi.mars_render_iteration(self.ctx.h, self.id, params)
        self.spp = params.spp
        self._last = params
        return st

    def update(self, params=None):
        return capi.mars_update_counts(self.ctx.h, self.id, params or self._last)

    # ---- inputs ----
    def set_fixed_counts(self, beta):
        b = np.ascontiguousarray(beta, np.float32).reshape(-1, 3)
        capi.mars_set_fixed_counts(self.ctx.h, self.id, _p(b), b.shape[0])

    def set_itilde(self, it):
        it = np.ascontiguousarray(it, np.float32).reshape(self.H, self.W, 3)
        capi.mars_set_itilde(self.ctx.h, self.id, _p(it))

    def set_hist(self, pm, cdf):
        pm = np.ascontiguousarray(pm, np.float32)
        cdf = np.ascontiguousarray(cdf, np.float32)
        capi.mars_set_hist(self.ctx.h, self.id, pm.shape[0], _p(pm), _p(cdf))

    def write_cells(self, factors=None, acc=None, visits=None):
        n = self.ncells
        arrs = [None if x is None else np.ascontiguousarray(x, dt)
                for x, dt in ((factors, np.float32), (acc, np.float64), (visits, np.uint32))]
        capi.mars_write_cells(self.ctx.h, self.id, n, *[None if a is None else _p(a) for a in arrs])

    def update_cells_only(self, V_I, C_I):
        capi.mars_update_cells_only(self.ctx.h, self.id, V_I, C_I)

    def refine_only(self):
        return capi.mars_refine_only(self.ctx.h, self.id)

    # ---- outputs ----
    @property
    def ncells(self):
        return capi.mars_num_cells(self.ctx.h, self.id)[0]

    def nodes(self):
        _, nn = capi.mars_num_cells(self.ctx.h, self.id)
        a = np.zeros(nn, np.uint32)
        capi.mars_read_nodes(self.ctx.h, self.id, _p(a))
        return a

    def image(self, which=IMAGE_MEAN):
        a = np.zeros((self.H, self.W, 3), np.float32)
        capi.mars_read_image(self.ctx.h, self.id, which, _p(a))
        return a

    def count_map(self):
        a = np.zeros((self.H, self.W, 3), np.float32)
        capi.mars_read_count_map(self.ctx.h, self.id, _p(a))
        return a

    def sample_radiance(self):
        a = np.zeros((self.H * self.W * self.spp, 3), np.float32)
        capi.mars_read_sample_radiance(self.ctx.h, self.id, _p(a))
        return a

    def itilde(self):
        a = np.zeros((self.H, self.W, 3), np.float32)
        capi.mars_read_itilde(self.ctx.h, self.id, _p(a))
        return a

    def cells(self):
        n = self.ncells
        fac = np.zeros((n, 2, 3, 3), np.float32)
        acc = np.zeros((n, 3, 8), np.float64)
        vis = np.zeros(n, np.uint32)
        dep = np.zeros(n, np.uint32)
        capi.mars_read_cells(self.ctx.h, self.id, _p(fac), _p(acc), _p(vis), _p(dep))
        return {"factors": fac, "acc": acc, "visits": vis, "depth": dep}

    def cells_x(self):
        """Per-length light-path budgets: factors [n][2][2][3] and
        accumulators [n][2][8] of techniques 3 (y_2) and 4 (y_3+)."""
        n = self.ncells
        fac = np.zeros((n, 2, 2, 3), np.float32)
        acc = np.zeros((n, 2, 8), np.float64)
        capi.mars_read_cells_x(self.ctx.h, self.id, _p(fac), _p(acc))
        return {"factors": fac, "acc": acc}

    def write_cells_x(self, factors=None, acc=None):
        arrs = [None if x is None else np.ascontiguousarray(x, dt)
                for x, dt in ((factors, np.float32), (acc, np.float64))]
        capi.mars_write_cells_x(self.ctx.h, self.id, self.ncells,
                                *[None if a is None else _p(a) for a in arrs])

    def hist(self):
        n = self.ncells
        pm = np.zeros((n, 64), np.float32)
        cdf = np.zeros((n, 64), np.float32)
        capi.mars_read_hist(self.ctx.h, self.id, _p(pm), _p(cdf))
        return pm, cdf

    def debug_vertices(self):
        n = capi.mars_debug_vertices(self.ctx.h, self.id, None, 0)
        a = np.zeros(n, VERTEX_DTYPE)
        if n:
            capi.mars_debug_vertices(self.ctx.h, self.id, _p(a), n)
        return a

    # ---- learned cache ----
    def mlp_train(self, steps=8, batch=32768, lr=1e-3):
        return capi.mars_mlp_train(self.ctx.h, self.id, steps, batch, lr)

    def mlp_params(self):
        a = np.zeros(capi.mars_mlp_num_params(), np.float32)
        capi.mars_mlp_read_params(self.ctx.h, self.id, _p(a))
        return a

    def set_mlp_params(self, params):
        a = np.ascontiguousarray(params, np.float32)
        assert a.shape[0] == capi.mars_mlp_num_params()
        capi.mars_mlp_write_params(self.ctx.h, self.id, _p(a))

    def mlp_forward(self, x6):
        x = np.ascontiguousarray(x6, np.float32).reshape(-1, 6)
        y = np.zeros((x.shape[0], 3), np.float32)
        capi.mars_mlp_forward(self.ctx.h, self.id, _p(x), x.shape[0], _p(y))
        return y

    def mlp_grad(self, x6, target, weight):
        x = np.ascontiguousarray(x6, np.float32).reshape(-1, 6)
        t = np.ascontiguousarray(target, np.float32).reshape(-1, 3)
        w = np.ascontiguousarray(weight, np.float32).reshape(-1, 3)
        g = np.zeros(capi.mars_mlp_num_params(), np.float32)
        loss = capi.mars_mlp_grad(self.ctx.h, self.id, _p(x), _p(t), _p(w), x.shape[0], _p(g))
        return loss, g

    def mlp_apply_grad(self, grad, lr=1e-3):
        g = np.ascontiguousarray(grad, np.float32)
        capi.mars_mlp_apply_grad(self.ctx.h, self.id, _p(g), lr)

    def mlp_write_records(self, pos, nrm, T, pix):
        """(tests) replaces the training vertices of the learned cache"""
        arrs = [np.ascontiguousarray(x, np.float32).reshape(-1, 3) for x in (pos, nrm, T)]
        px = np.ascontiguousarray(pix, np.uint32).ravel()
        capi.mars_mlp_write_records(self.ctx.h, self.id, *[_p(a) for a in arrs], _p(px),
                                    px.shape[0])

    def mlp_targets_only(self):
        capi.mars_mlp_targets_only(self.ctx.h, self.id)

    def mlp_train_set(self):
        """inputs [n][6], targets [n][3] and weights [n][3] of the training set"""
        n = capi.mars_mlp_read_train(self.ctx.h, self.id, None, None, None, 0)
        x = np.zeros((n, 6), np.float32)
        t = np.zeros((n, 3), np.float32)
        w = np.zeros((n, 3), np.float32)
        if n:
            capi.mars_mlp_read_train(self.ctx.h, self.id, _p(x), _p(t), _p(w), n)
        return x, t, w

    # ---- queue sizing ----
    def configure(self, queue_capacity=0, tile_roots=0, shadow_capacity=None):
        """Queue sizes: queue_capacity entries per level of the ray queues and
        shadow_capacity of the shadow queues (None: queue_capacity); 0 keeps."""
        if shadow_capacity is None:
            capi.mars_scene_configure(self.ctx.h, self.id, int(queue_capacity), int(tile_roots))
        else:
            capi.mars_scene_configure_queues(self.ctx.h, self.id, int(queue_capacity),
                                             int(shadow_capacity), int(tile_roots))

    def query(self):
        """(ray-queue capacity, tile size, peak queue level per camera sample
        of the last eager iteration)"""
        return capi.mars_scene_query(self.ctx.h, self.id)

    def query_queues(self):
        """(ray-queue capacity, shadow-queue capacity, peak ray and shadow
        entries per camera sample of the last eager iteration)"""
        return capi.mars_scene_query_queues(self.ctx.h, self.id)

    def checkpoint_save(self, path):
        capi.mars_checkpoint_save(self.ctx.h, self.id, str(path))

    def checkpoint_load(self, path):
        capi.mars_checkpoint_load(self.ctx.h, self.id, str(path))


def render_batch(scenes, params):
    """One render iteration of every scene as one batch; returns the totals."""
    st = capi.mars_render_batch(scenes[0].ctx.h, [s.id for s in scenes], params)
    for s in scenes:
        s.spp, s._last = params.spp, params
    return st


def iterate_batch(scenes, params, update=True, graph=True):
    """Render (and update) iteration of every scene in one captured launch
    graph; returns per-scene iteration and update statistics."""
    flags = (BATCH_UPDATE if update else 0) | (0 if graph else BATCH_NO_GRAPH)
    its, ups = capi.mars_iterate_batch(scenes[0].ctx.h, [s.id for s in scenes], params, flags)
    for s in scenes:
        s.spp, s._last = params.spp, params
    return its, ups


def autotune(scenes, params, mem_budget=0, cache_path=None):
    """Queue and tile sizes per scene: [(ray capacity, tile, peak rays per
    sample, shadow capacity, peak shadow entries per sample)]."""
    r = capi.mars_autotune(scenes[0].ctx.h, [s.id for s in scenes], params, int(mem_budget),
                           cache_path)
    return list(zip(*r))


def run_schedule(scene: Scene, n_iter, warmup=1, spp=1, budget_aware=True, stat_clamp=None,
                 rr_start=5, clamp_hi=20.0, spp_schedule=None, on_iter=None, iter0=0):
    """`warmup` classic-RR iterations then MARS iterations, each followed by
    the update step (Sec. 4.1 "Fixed-point iteration")."""
    if stat_clamp is None:
        stat_clamp = 0.0 if scene.mode == MODE_BDPT else 50.0
    hist = []
    for i in range(iter0, iter0 + n_iter):
        s = spp_schedule(i) if spp_schedule else spp
        p = iter_params(iteration=i, spp=s, alloc=ALLOC_CLASSIC if i < warmup else ALLOC_MARS,
                        budget_aware=budget_aware, rr_start=rr_start, stat_clamp=stat_clamp,
                        clamp_hi=clamp_hi)
        st = scene.render_iteration(p)
        us = scene.update(p)
        hist.append((st.as_dict(), us.V_I, us.C_I, us.n_cells_after))
        if on_iter:
            on_iter(i, st, us)
    return hist
