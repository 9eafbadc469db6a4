"""GPU parity of the 2D smoother kernel that takes a row of x-adjacent patches of one color per wavefront.

Sizes give color rows of several groups with a ragged last group, rows of a
single patch, and (at the paper's 2048^2 shapes, in the configuration the
benchmark times) one color checked on sampled patches against the oracle's
exact local solve from the patch closure.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import vps_inputs as vi
from oracle import assemble, mesh, smoother
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# (k, N): patches per wave are 15, 10, 7, 6 for k = 2..5; N - 1 interior vertices per direction
ROW_CASES = [(2, 40), (2, 4), (3, 25), (3, 3), (4, 17), (4, 16), (5, 15), (5, 4)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N", ROW_CASES)
def test_row_colors_fp64(vps, k, N):
    """Every color, FP64, against the oracle's colorized sweep color by color."""
    say("2D row colors fp64", k, N)
    A = assemble.assemble_kron(2, k, N)
    P = smoother.Patches(2, k, N)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(2, k, N, 91)
    uo = vi.seeded_vector(2, k, N, 92)
    with vps.Context(2, k, N, 1, wave_rows_2d=1) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(4):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("k,N", [(2, 40), (3, 25), (4, 17), (5, 15)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_matches_generic_kernel(vps, k, N, dtype):
    """Two sweeps (forward and reverse) against the LDS-staged generic kernel."""
    import torch
    say("2D row vs generic", k, N, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = vi.seeded_vector(2, k, N, 93)
    u0 = vi.seeded_vector(2, k, N, 94)
    out = []
    for rows in (1, 2):
        with vps.Context(2, k, N, 1, vcycle_dtype=dtype, wave_rows_2d=rows) as ctx:
            u = dev(u0, tdt)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1)
            ctx.smooth(0, u, dev(b, tdt), sweeps=1, reverse=True)
            out.append(host(u))
    assert rel(out[0], out[1]) <= (1e-13 if dtype == "f64" else 2e-5)


@pytest.mark.parametrize("k,color", [(3, 1), (5, 2)])
def test_row_color_full_size_sampled(vps, k, color):
    """One color on the paper's 2D 2048^2 shapes (FP64) against the oracle's exact solve of sampled patches."""
    N = 2048
    say("2D row full size", k, color)
    u0 = vi.seeded_vector(2, k, N, 95)
    b = vi.seeded_vector(2, k, N, 96)
    with vps.Context(2, k, N, 1, wave_rows_2d=1) as ctx:
        u = dev(u0)
        ctx.smooth_color(0, u, dev(b), color)
        u1 = host(u)
        del u
    h = 1.0 / N
    Abar = smoother.patch_closure_operator(2, k, h)
    ipos = smoother.closure_interior_positions(2, k)
    gpos = np.setdiff1d(np.arange(Abar.shape[0]), ipos)
    cho = sla.cho_factor(Abar[np.ix_(ipos, ipos)])
    Aig = Abar[np.ix_(ipos, gpos)]
    rng = np.random.default_rng(13 + k)
    par = [(color >> e) & 1 for e in range(2)]
    cand = [[v for v in range(1, N) if v % 2 == par[e]] for e in range(2)]
    touched = np.zeros(u1.size, dtype=bool)
    for i in range(80):
        if i % 4 == 0:  # first and last patches of a row, group boundaries
            v = tuple(int(rng.choice([cand[e][0], cand[e][-1], cand[e][len(cand[e]) // 2]])) for e in range(2))
        else:
            v = tuple(int(rng.choice(cand[e])) for e in range(2))
        clo = mesh.patch_closure(2, k, N, v)
        inner = clo[ipos]
        want = sla.cho_solve(cho, b[inner] - Aig @ u0[clo[gpos]])
        assert np.abs(u1[inner] - want).max() <= 1e-11 * np.abs(want).max(), v
        touched[inner] = True
    # nothing outside the color's interiors is written
    n1 = k * N + 1
    masks = []
    for e in range(2):
        m = np.zeros(n1, dtype=bool)
        for vv in range(1, N):
            if vv % 2 == par[e]:
                m[k * (vv - 1) + 1:k * (vv + 1)] = True
        masks.append(m)
    mask = (masks[1][:, None] & masks[0][None, :]).reshape(-1)
    assert np.array_equal(u1[~mask], u0[~mask])
