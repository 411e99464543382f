"""The allocation-free gradient pass (mars_mlp_grad_noalloc) against
mars_mlp_grad, through the C ABI: two calls in a row, the second with a
smaller batch, each equal to the allocating entry point's result bit for
bit; sizes beyond the fixed array are refused."""
import ctypes as C

import numpy as np
import pytest

import scenegen
from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)


def test_mlp_grad_noalloc_matches_grad():
    import torch

    from paper_2410_20429_amd import _capi, api
    ctx = api.Context(0)
    s = api.Scene(ctx, scenegen.make_cornell(8, 8), max_depth=2, mlp=True)
    s.set_mlp_params(M.init_params(5))
    rng = np.random.default_rng(8)
    npar = M.N_PARAMS
    for n in (4099, 777):  # second call smaller: stale partials must not leak in
        say("noalloc gradient, batch", n)
        x = np.concatenate([rng.random((n, 3)), rng.uniform(-1, 1, (n, 3))], 1).astype(np.float32)
        t = rng.normal(size=(n, 3)).astype(np.float32)
        w = rng.random((n, 3)).astype(np.float32)
        w[rng.random((n, 3)) < 0.2] = 0.0
        loss_ref, g_ref = s.mlp_grad(x, t, w)
        dx, dt, dw = (torch.from_numpy(a).cuda() for a in (x, t, w))
        dg = torch.full((npar + 1,), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        _capi.mars_mlp_grad_noalloc(ctx.h, s.id, C.c_void_p(dx.data_ptr()),
                                    C.c_void_p(dt.data_ptr()), C.c_void_p(dw.data_ptr()), n,
                                    C.c_void_p(dg.data_ptr()))
        torch.cuda.synchronize()
        g = dg.cpu().numpy()
        np.testing.assert_array_equal(g[:npar], g_ref)
        assert g[npar] == np.float32(loss_ref)
        assert np.all(np.isfinite(g))
    with pytest.raises(_capi.MarsError):
        _capi.mars_mlp_grad_noalloc(ctx.h, s.id, C.c_void_p(dx.data_ptr()),
                                    C.c_void_p(dt.data_ptr()), C.c_void_p(dw.data_ptr()),
                                    262145, C.c_void_p(dg.data_ptr()))
    s.release()
    ctx.close()
