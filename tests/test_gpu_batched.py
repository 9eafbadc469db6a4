"""GPU parity of batch processing (Algorithm 5): slabs of vertex layers, all colors of a slab in turn."""
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


# sizes with more than 2B vertex layers (smaller levels sweep whole colors)
@pytest.mark.parametrize("dim,k,N,B", [(3, 2, 7, 1), (3, 2, 8, 3), (3, 4, 8, 3), (2, 2, 9, 3), (3, 3, 5, 1)])
@pytest.mark.parametrize("reverse", [False, True])
def test_batched_sweep_odd_layers(vps, dim, k, N, B, reverse):
    """Odd batch sizes change the patch order: compare with the oracle's batched sweep."""
    say("batched sweep", dim, k, N, B, reverse)
    A = assemble.assemble(dim, k, N)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(dim, k, N, 91)
    u0 = vi.seeded_vector(dim, k, N, 92)
    want = smoother.sweep_batched(A, b, u0, P, S, B, reverse)
    assert rel(want, smoother.sweep_colorized(A, b, u0, P, S, reverse)) > 1e-8  # a different iterate
    with vps.Context(dim, k, N, 1, batch_layers=B) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=1, reverse=reverse)
        assert rel(host(u), want) <= 1e-12


@pytest.mark.parametrize("k,N,B", [(4, 10, 3), (5, 8, 3), (5, 9, 1)])
def test_batched_sweep_odd_layers_rows(vps, k, N, B):
    """Odd batch sizes with rows of patches (degree 5: two waves per row), FP64, against the oracle's
    batched sweep."""
    say("batched sweep rows", k, N, B)
    A = assemble.assemble(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 93)
    u0 = vi.seeded_vector(3, k, N, 94)
    want = smoother.sweep_batched(A, b, u0, P, S, B, False)
    with vps.Context(3, k, N, 1, batch_layers=B, patches_per_wave=3) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=1)
        assert rel(host(u), want) <= 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("B", [2, 4, 8])
def test_batched_even_layers_bitwise(vps, dtype, B):
    """Even batch sizes keep the colorized order of every interacting pair: the same bits as whole colors."""
    import torch
    k, N = 4, 20
    say("batched even", dtype, B)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = vi.seeded_vector(3, k, N, 93)
    u0 = vi.seeded_vector(3, k, N, 94)
    out = []
    for bl in (0, B):
        with vps.Context(3, k, N, 1, vcycle_dtype=dtype, batch_layers=bl) as ctx:
            u = dev(u0, tdt)
            ctx.smooth(0, u, dev(b, tdt), sweeps=2)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1, reverse=True)
            out.append(host(u))
    assert np.array_equal(out[0], out[1])


def test_batched_small_level_sweeps_whole_colors(vps):
    """A level with at most 2B vertex layers is swept in whole colors (the plain colorized iterate)."""
    k, N, B = 2, 7, 3
    say("batched small level")
    A = assemble.assemble(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 96)
    u0 = vi.seeded_vector(3, k, N, 97)
    with vps.Context(3, k, N, 1, batch_layers=B) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=1)
        assert rel(host(u), smoother.sweep_colorized(A, b, u0, P, S)) <= 1e-12


def test_batched_solve_odd_layers(vps):
    """With the reversed sequence as post-smoothing the batched V-cycle stays symmetric: PCG converges."""
    import torch
    k, N, L = 2, 16, 3
    say("batched solve")
    b = vi.seeded_vector(3, k, N, 95)
    with vps.Context(3, k, N, L, 1, 1, batch_layers=3) as ctx:
        x = torch.empty(b.size, dtype=torch.float64, device="cuda")
        info = ctx.solve(dev(b), x, rtol=1e-10, maxit=60)
        xs = host(x)
    assert info["rel_residual_true"] <= 1e-10
    assert np.linalg.norm(b - assemble.matvec_kron(3, k, N, xs)) <= 1e-10 * np.linalg.norm(b)


def test_batched_even_layers_full_size(vps):
    """3D Q4 on 128^3 cells, FP32, slabs of 16 vertex layers and of the benchmark's slab size: the same bits
    as whole colors."""
    import torch
    k, N = 4, 128
    say("batched full size")
    b = vi.seeded_vector(3, k, N, 5)
    u0 = vi.seeded_vector(3, k, N, 105)
    out = []
    for bl in (0, 16, vi.WORKLOADS["poisson3d_q4_n128"]["batch_layers"]):
        with vps.Context(3, k, N, 1, vcycle_dtype="f32", batch_layers=bl) as ctx:
            u = dev(u0, torch.float32)
            ctx.smooth(0, u, dev(b, torch.float32), sweeps=1)
            out.append(host(u))
            del u
    assert np.array_equal(out[0], out[1])
    assert np.array_equal(out[0], out[2])
