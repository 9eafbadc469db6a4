"""GPU parity of the smoother kernel that takes two x-adjacent patches of a color per wavefront.

The pair shares one closure face, so the wavefront loads the union of the two
closures once; the update is the same exact local solve as with one patch per
wavefront.  Sizes give colors with an even and an odd number of patches along
x (a last pair with one patch) and several pairs along y and z.
"""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, smoother
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# (k, N): N - 1 interior vertices per direction; colors have (N - 1) // 2 or N // 2 patches along x
PAIR_CASES = [(2, 7), (2, 8), (3, 5), (3, 6), (4, 5), (4, 6), (2, 11)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N", PAIR_CASES)
def test_pair_colors_fp64(vps, k, N):
    """Every color, FP64, against the oracle's colorized sweep (Algorithm 3 form) color by color."""
    say("pair colors fp64", k, N)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 71)
    uo = vi.seeded_vector(3, k, N, 72)
    with vps.Context(3, k, N, 1, patches_per_wave=2) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(8):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("k,N", [(2, 8), (3, 5), (4, 6)])
@pytest.mark.parametrize("reverse", [False, True])
def test_pair_sweep_fp32(vps, k, N, reverse):
    """FP32 sweeps with pairs: against the oracle (FP32 rounding) and against one patch per wavefront."""
    import torch
    say("pair sweep fp32", k, N, reverse)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 73).astype(np.float32).astype(np.float64)
    u0 = vi.seeded_vector(3, k, N, 74).astype(np.float32).astype(np.float64)
    want = smoother.sweep_colorized(A, b, u0, P, S, reverse=reverse)
    out = {}
    for ppw in (1, 2):
        with vps.Context(3, k, N, 1, vcycle_dtype="f32", patches_per_wave=ppw) as ctx:
            u = dev(u0, torch.float32)
            ctx.smooth(0, u, dev(b, torch.float32), sweeps=1, reverse=reverse)
            out[ppw] = host(u)
    assert rel(out[2], want) <= 2e-5
    assert rel(out[2], out[1]) <= 2e-5


@pytest.mark.parametrize("dtype,k,N,auto", [("f32", 4, 32, 1), ("f32", 3, 32, 2), ("f64", 4, 32, 2), ("f64", 2, 32, 3),
                                          ("f64", 4, 16, 1), ("f32", 3, 9, 1), ("f32", 4, 64, 3), ("f64", 4, 64, 3),
                                          ("f64", 3, 64, 3), ("f32", 2, 16, 1), ("f64", 5, 64, 3), ("f32", 5, 32, 1)])
def test_automatic_patches_per_wave(vps, dtype, k, N, auto):
    """patches_per_wave=0 takes a row of patches per wave at degree 2 from 32 cells and degrees 3 to 5 from
    64, else pairs from 32 cells except FP32 at degree 4 and degree 5: the same bits as that choice made
    explicit; the other choices agree up to rounding."""
    import torch
    say("automatic patches per wave", dtype, k, N)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    b = vi.seeded_vector(3, k, N, 75)
    u0 = vi.seeded_vector(3, k, N, 76)
    out = {}
    forms = (0, 1, 3) if k == 5 else (0, 1, 2, 3)  # no pair kernel at degree 5
    for ppw in forms:
        with vps.Context(3, k, N, 1, vcycle_dtype=dtype, patches_per_wave=ppw) as ctx:
            u = dev(u0, tdt)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1)
            out[ppw] = host(u)
    assert np.array_equal(out[0], out[auto])
    assert not np.array_equal(out[1], out[forms[2]])  # a different rounding order
    for p in forms[2:]:
        assert rel(out[1], out[p]) <= (2e-5 if dtype == "f32" else 1e-13)


def test_pair_batched_fp64_matches_whole_colors(vps):
    """Slabs of 2 vertex layers (even: Algorithm 4's iterate) with pairs, FP64."""
    k, N = 3, 10
    say("pair batched fp64")
    b = vi.seeded_vector(3, k, N, 77)
    u0 = vi.seeded_vector(3, k, N, 78)
    out = {}
    for B in (0, 2):
        with vps.Context(3, k, N, 1, patches_per_wave=2, batch_layers=B) as ctx:
            u = dev(u0)
            ctx.smooth(0, u, dev(b), sweeps=1)
            out[B] = host(u)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    want = smoother.sweep_colorized(A, b, u0, P, S)
    assert rel(out[0], want) <= 1e-12
    assert rel(out[2], want) <= 1e-12


@pytest.mark.parametrize("k,N", [(2, 3), (2, 4), (3, 4), (4, 3), (4, 4)])
@pytest.mark.parametrize("form", ["wave", "pair", "separated"])
def test_rows_of_one_patch_fp64(vps, k, N, form):
    """Colors with a single patch (or a single pair) along x or y: the patch decomposition divides by 1."""
    say("rows of one patch", k, N, form)
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 79)
    uo = vi.seeded_vector(3, k, N, 80)
    kw = dict(wave=dict(patches_per_wave=1), pair=dict(patches_per_wave=2), separated=dict(algorithm="separated"))[form]
    with vps.Context(3, k, N, 1, **kw) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(8):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("form", ["wave", "pair", "separated"])
def test_single_patch_domain_fp64(vps, k, form):
    """N = 2: one patch covers the domain, so one sweep is the exact solve (b - A u = 0 afterwards)."""
    say("single patch domain", k, form)
    N = 2
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 81)
    u0 = vi.seeded_vector(3, k, N, 82)
    want = smoother.sweep_colorized(A, b, u0, P, S)
    kw = dict(wave=dict(patches_per_wave=1), pair=dict(patches_per_wave=2), separated=dict(algorithm="separated"))[form]
    with vps.Context(3, k, N, 1, **kw) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=1)
        got = host(u)
    assert rel(got, want) <= 1e-12
    assert np.abs(b - A @ got).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("N", [5, 6, 9])
def test_degree5_one_patch_kernel_fp64(vps, N):
    """k = 5: one patch per wave with the 81 interior lines in two passes; every color against the oracle."""
    say("degree 5 one-patch kernel", N)
    k = 5
    A = assemble.assemble_kron(3, k, N)
    P = smoother.Patches(3, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(3, k, N, 83)
    uo = vi.seeded_vector(3, k, N, 84)
    with vps.Context(3, k, N, 1) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(8):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_degree5_matches_generic_kernel(vps, dtype):
    """k = 5 sweeps, forward and reverse: the one-patch kernel against the LDS-staged generic kernel."""
    import torch
    k, N = 5, 12
    say("degree 5 vs generic", dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = vi.seeded_vector(3, k, N, 85)
    u0 = vi.seeded_vector(3, k, N, 86)
    out = []
    for pb in (0, 1):
        with vps.Context(3, k, N, 1, vcycle_dtype=dtype, patches_per_block=pb) as ctx:
            u = dev(u0, tdt)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1, reverse=True)
            out.append(host(u))
    assert rel(out[0], out[1]) <= (1e-12 if dtype == "f64" else 2e-5)
