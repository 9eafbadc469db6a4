"""GPU parity of the 3D smoother kernel that takes a row of x-adjacent patches of a color per wavefront.

G = floor(63 / 2k) patches side by side (15, 10, 7 for k = 2, 3, 4) span G*2k + 1
node columns, one lane per column; at k = 5 a workgroup of two waves takes G = 5
patches (51 or 52 columns).  Sizes give colors with full and ragged last
groups along x, several groups per color row, single-patch rows and the
single-patch domain; the update is the same exact local solve as with one
patch per wavefront.
"""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, smoother
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# (k, N): colors have (N - 1) // 2 or N // 2 patches along x against groups of 15 / 10 / 7 / 5
# (degree 5: a workgroup of two waves per group); packed groups from G patches per row on
ROW3_CASES = [(2, 32), (3, 22), (4, 18), (4, 9), (2, 5), (3, 4), (4, 3), (4, 2),
              (5, 14), (5, 12), (5, 11), (5, 8), (5, 3), (5, 2)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N", ROW3_CASES)
def test_row3_colors_fp64(vps, k, N):
    """Every color, FP64, against the oracle's colorized sweep (Algorithm 3 form) color by color."""
    say("row3 colors fp64", k, N)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 171)
    uo = vi.seeded_vector(3, k, N, 172)
    with vps.Context(3, k, N, 1, patches_per_wave=3) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(8):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("k,N", [(2, 32), (3, 22), (4, 18), (4, 6), (5, 14), (5, 7)])
@pytest.mark.parametrize("reverse", [False, True])
def test_row3_sweep_fp32(vps, k, N, reverse):
    """FP32 sweeps with rows of patches: against the oracle (FP32 rounding) and against one patch per wavefront."""
    import torch
    say("row3 sweep fp32", k, N, reverse)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 173).astype(np.float32).astype(np.float64)
    u0 = vi.seeded_vector(3, k, N, 174).astype(np.float32).astype(np.float64)
    want = smoother.sweep_colorized(A, b, u0, P, S, reverse=reverse)
    out = {}
    for ppw in (1, 3):
        with vps.Context(3, k, N, 1, vcycle_dtype="f32", patches_per_wave=ppw) as ctx:
            u = dev(u0, torch.float32)
            ctx.smooth(0, u, dev(b, torch.float32), sweeps=1, reverse=reverse)
            out[ppw] = host(u)
    assert rel(out[3], want) <= 2e-5
    assert rel(out[3], out[1]) <= 2e-5


@pytest.mark.parametrize("k,N", [(4, 10), (5, 8)])
def test_row3_batched_fp32_matches_whole_colors(vps, k, N):
    """Slabs of 2 vertex layers (even: Algorithm 4's iterate) with rows of patches, FP32, against the oracle."""
    import torch
    say("row3 batched fp32", k, N)
    b = vi.seeded_vector(3, k, N, 177).astype(np.float32).astype(np.float64)
    u0 = vi.seeded_vector(3, k, N, 178).astype(np.float32).astype(np.float64)
    out = {}
    for B in (0, 2):
        with vps.Context(3, k, N, 1, vcycle_dtype="f32", patches_per_wave=3, batch_layers=B) as ctx:
            u = dev(u0, torch.float32)
            ctx.smooth(0, u, dev(b, torch.float32), sweeps=1)
            out[B] = host(u)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    want = smoother.sweep_colorized(A, b, u0, P, S)
    assert rel(out[0], want) <= 2e-5
    assert rel(out[2], want) <= 2e-5
