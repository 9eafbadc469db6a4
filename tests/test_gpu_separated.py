"""GPU parity of the separated colorized smoother (Algorithm 3): global residual per color, then local solves.

With exact local solvers it reaches the same iterate as the combined form
(Algorithm 4): the oracle's Algorithm 3 sweep is the reference for both.
"""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, smoother
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N,smin", [(2, 7, 0), (3, 5, 0), (4, 5, 0), (4, 9, 1), (2, 36, 1)])
@pytest.mark.parametrize("reverse", [False, True])
def test_separated_sweep_fp64(vps, k, N, smin, reverse):
    say("separated sweep", k, N, smin, reverse)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 51)
    u0 = vi.seeded_vector(3, k, N, 52)
    want = smoother.sweep_colorized(A, b, u0, P, S, reverse=reverse)
    with vps.Context(3, k, N, 1, algorithm="separated", stream_min_cells=smin) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=1, reverse=reverse)
        assert rel(host(u), want) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_separated_matches_combined(vps, dtype):
    import torch
    k, N = 4, 20
    say("separated vs combined", dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = vi.seeded_vector(3, k, N, 53)
    u0 = vi.seeded_vector(3, k, N, 54)
    out = {}
    for alg in ("combined", "separated"):
        with vps.Context(3, k, N, 1, vcycle_dtype=dtype, algorithm=alg) as ctx:
            u = dev(u0, tdt)
            ctx.smooth(0, u, dev(b, tdt), sweeps=2)
            out[alg] = host(u)
    assert rel(out["separated"], out["combined"]) <= (1e-12 if dtype == "f64" else 2e-5)


def test_separated_solve(vps):
    import torch
    k, N, L = 3, 16, 3
    say("separated solve")
    b = vi.seeded_vector(3, k, N, 55)
    its = {}
    for alg in ("combined", "separated"):
        with vps.Context(3, k, N, L, 1, 1, algorithm=alg) as ctx:
            x = torch.empty(b.size, dtype=torch.float64, device="cuda")
            info = ctx.solve(dev(b), x, rtol=1e-10, maxit=50)
            assert info["rel_residual_true"] <= 1e-10
            xs = host(x)
            assert np.linalg.norm(b - assemble.matvec_kron(3, k, N, xs)) <= 1e-10 * np.linalg.norm(b)
            its[alg] = info["iterations"]
    assert its["separated"] == its["combined"]


def test_separated_color_full_size(vps):
    """One color at 513^3 (3D Q4, FP32): separated and combined give the same interiors."""
    import torch
    k, N, color = 4, 128, 2
    say("separated full size")
    b = vi.seeded_vector(3, k, N, 5)
    u0 = vi.seeded_vector(3, k, N, 105)
    out = {}
    for alg in ("combined", "separated"):
        with vps.Context(3, k, N, 1, vcycle_dtype="f32", algorithm=alg) as ctx:
            u = dev(u0, torch.float32)
            ctx.smooth_color(0, u, dev(b, torch.float32), color)
            out[alg] = host(u)
            del u
    assert rel(out["separated"], out["combined"]) <= 2e-5
