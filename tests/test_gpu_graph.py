"""The finest-level V-cycle replayed from a captured HIP graph gives the bits of kernel-by-kernel launches.

A context created with vcycle_graph=True captures its V-cycle once per
(input, output) buffer pair and replays it; the default launches every kernel.
Replays are interleaved with other work of the same context and checked one
by one.
"""
import numpy as np
import pytest

import vps_inputs as vi
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("dim,k,N,L,dtype", [(3, 3, 16, 3, "f32"), (3, 2, 16, 3, "f64"), (2, 2, 32, 4, "f64"),
                                             (3, 4, 16, 3, "f32")])
def test_vcycle_replays_match_eager(vps, dim, k, N, L, dtype):
    import torch
    say("vcycle graph replays", dim, k, N, L, dtype)
    ctxs = [vps.Context(dim, k, N, L, 1, 1, vcycle_dtype=dtype, vcycle_graph=g) for g in (True, False)]
    try:
        for rep in range(4):
            r = dev(vi.seeded_vector(dim, k, N, 200 + rep))
            outs = []
            for ctx in ctxs:
                z = torch.empty_like(r)
                ctx.vcycle(r, z)
                # other work on the same context between the replays
                w = torch.empty_like(r)
                ctx.apply(L - 1, z, w)
                outs.append(host(z))
            assert np.array_equal(outs[0], outs[1]), rep
    finally:
        for ctx in ctxs:
            ctx.close()


@pytest.mark.parametrize("dim,k,N,L,dtype", [(3, 3, 16, 3, "f32"), (3, 2, 16, 3, "f64"), (2, 2, 32, 4, "f64")])
def test_solve_with_graph_matches_eager(vps, dim, k, N, L, dtype):
    import torch
    say("solve graph vs eager", dim, k, N, L, dtype)
    out = {}
    for eager in (False, True):
        with vps.Context(dim, k, N, L, 1, 1, vcycle_dtype=dtype, vcycle_graph=not eager) as ctx:
            res = []
            for seed in (210, 211, 210):  # the same right-hand side buffer contents twice: a cached graph
                b = dev(vi.seeded_vector(dim, k, N, seed))
                x = torch.empty_like(b)
                info = ctx.solve(b, x, rtol=1e-10, maxit=100)
                assert info["rel_residual_true"] <= 1e-10
                res.append((info["iterations"], host(x)))
            out[eager] = res
    for (ig, xg), (ie, xe) in zip(out[False], out[True]):
        assert ig == ie
        assert np.array_equal(xg, xe)


def test_graph_follows_a_new_coefficient(vps):
    """set_coefficient between solves drops the captured graphs; results follow the new field."""
    import torch
    k, N, L = 2, 16, 3
    say("graph and set_coefficient")
    b = dev(vi.seeded_vector(3, k, N, 212))
    out = {}
    for eager in (False, True):
        with vps.Context(3, k, N, L, 1, 1, coef="mean", vcycle_graph=not eager) as ctx:
            res = []
            for seed in (7, 8):
                ctx.set_coefficient(dev(vi.rho_cells(N, seed)))
                x = torch.empty_like(b)
                info = ctx.solve(b, x, rtol=1e-10, maxit=100)
                assert info["rel_residual_true"] <= 1e-10
                res.append((info["iterations"], host(x)))
            out[eager] = res
    for (ig, xg), (ie, xe) in zip(out[False], out[True]):
        assert ig == ie
        assert np.array_equal(xg, xe)
    assert not np.array_equal(out[False][0][1], out[False][1][1])
