"""The allocation-free MLP backward (vps_mlp_backward_noalloc) against vps_mlp_backward, through the C ABI.

Two calls in a row, the second with fewer samples: both must give the same gradient as the allocating
entry point (same kernels, same reduction order: bit for bit), and a sample count above the static work
memory's limit is rejected on the host before any work."""
import ctypes

import numpy as np
import pytest

from paper_2407_02100_amd import vps

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n, 8, generator=g).to("cuda")
    dy = (0.1 * torch.randn(n, 27, generator=g)).to("cuda")
    return x, dy


def test_noalloc_backward_matches_backward_twice():
    import torch
    from paper_2407_02100_amd import learned
    L = vps.lib()
    params = torch.from_numpy(learned.init_params(5)).to("cuda")
    params += 0.05 * torch.randn_like(params)
    with vps.Context(3, 2, 4, 1, coef="learned") as ctx:
        for n, seed in ((3000, 1), (700, 2)):  # the second call with a smaller input
            say(f"no-alloc backward: n = {n}")
            x, dy = _inputs(torch, n, seed)
            y = torch.empty(n, 27, device="cuda")
            act = torch.empty(n, 128, device="cuda")
            ctx.mlp_forward(params, x, y, act)
            g_ref = torch.full((params.numel(),), float("nan"), device="cuda")
            g_new = torch.full((params.numel(),), float("nan"), device="cuda")
            st = L.vps_mlp_backward(ctx.h, ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(act.data_ptr()), ctypes.c_void_p(dy.data_ptr()), n,
                                    ctypes.c_void_p(g_ref.data_ptr()))
            assert st == 0
            st = L.vps_mlp_backward_noalloc(ctx.h, ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(act.data_ptr()), ctypes.c_void_p(dy.data_ptr()), n,
                                            ctypes.c_void_p(g_new.data_ptr()))
            assert st == 0, L.vps_last_error(ctx.h)
            ctx.sync()
            a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_noalloc_backward_rejects_too_many_samples():
    import torch
    L = vps.lib()
    with vps.Context(3, 2, 4, 1, coef="learned") as ctx:
        n = 4947  # one more than (2^20 - 64 * 6491) / 128
        buf = torch.zeros(n * 128, device="cuda")
        p = torch.zeros(6491, device="cuda")
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())
        st = L.vps_mlp_backward_noalloc(ctx.h, ptr(p), ptr(buf), ptr(buf), ptr(buf), n, ptr(p))
        assert st == vps.VPS_E_ARG
        assert b"4946" in L.vps_last_error(ctx.h)
