"""GPU parity of the 2D row-streaming operator and residual (constant coefficient).

Grids span several column strips (64 - 2k output columns each) with a ragged
last strip and many cell-row chunks; the full-size cases (the paper's 2D
2048^2 shapes) are checked on sampled nodes, each computed from the 1D
matrices.
"""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, fe, transfer
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

CASES = [(1, 150), (2, 70), (3, 45), (4, 30), (5, 25), (2, 9)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_and_residual_2d(vps, k, N, dtype):
    import torch
    say("2D stream operator", k, N, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u0 = vi.seeded_vector(2, k, N, 41)
    b = vi.seeded_vector(2, k, N, 42)
    if dtype == "f32":  # the oracle sees the values the kernel sees
        u0 = u0.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    Au = assemble.matvec_kron(2, k, N, u0)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(2, k, N, 1, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        out = torch.full((u0.size,), 7.0, dtype=tdt, device="cuda")  # Dirichlet entries must be overwritten
        ctx.apply(0, dev(u0, tdt), out)
        assert rel(host(out), Au) <= tol
        out.fill_(7.0)
        ctx.residual(0, dev(b, tdt), dev(u0, tdt), out)
        assert rel(host(out), b - Au) <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vcycle_same_with_stream2_and_tile(vps, dtype):
    """2D Q3, 5 levels on 64^2 cells: both operator kernels give the same V-cycle within rounding."""
    import torch
    say("2D vcycle stream vs tile", dtype)
    k, N, L = 3, 64, 5
    r = dev(vi.seeded_vector(2, k, N, 43))
    z = []
    for smin in (1, 1 << 30):
        with vps.Context(2, k, N, L, 1, 1, vcycle_dtype=dtype, stream_min_cells=smin) as ctx:
            out = torch.empty_like(r)
            ctx.vcycle(r, out)
            z.append(host(out))
    assert rel(z[0], z[1]) <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("k", [3, 5])
def test_operator_full_size_sampled_2d(vps, k):
    """The paper's 2D shapes (2048^2 cells), FP64, on sampled nodes next to strip, chunk and domain edges."""
    import torch
    N = 2048
    say("2D stream operator full size", k)
    n1 = k * N + 1
    u0 = vi.seeded_vector(2, k, N, 44)
    with vps.Context(2, k, N, 1) as ctx:
        out = torch.full((u0.size,), 7.0, dtype=torch.float64, device="cuda")
        ctx.apply(0, dev(u0), out)
        got = host(out).reshape(n1, n1)
        del out
    M1, K1 = fe.assembled_1d(k, N)
    U = u0.reshape(n1, n1)
    rng = np.random.default_rng(17 + k)
    wo = 64 - 2 * k
    edge = [0, 1, k, wo - 1, wo, wo + 1, 2 * wo, n1 // 2, n1 - 2, n1 - 1]
    pts = [(int(rng.integers(0, n1)), int(rng.integers(0, n1))) for _ in range(200)]
    pts += [(int(rng.choice(edge)), int(rng.integers(0, n1))) for _ in range(100)]
    pts += [(int(rng.integers(0, n1)), int(rng.choice(edge))) for _ in range(100)]
    for x, y in pts:
        if min(x, y) == 0 or max(x, y) == n1 - 1:
            assert got[y, x] == 0.0
            continue
        xs = np.nonzero(M1[x])[0]
        ys = np.nonzero(M1[y])[0]
        blk = U[np.ix_(ys, xs)]
        w = np.outer(M1[y, ys], K1[x, xs]) + np.outer(K1[y, ys], M1[x, xs])
        want = float((w * blk).sum())
        assert abs(got[y, x] - want) <= 1e-13 * float(np.abs(w * blk).sum()) + 1e-300, (x, y)


TRANSFER_CASES = [(1, 80), (2, 40), (3, 25), (4, 18), (5, 15), (2, 5)]


@pytest.mark.parametrize("k,Nc", TRANSFER_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_restrict_2d(vps, k, Nc, dtype):
    import torch
    say("2D stream restrict", k, Nc, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rf = vi.seeded_vector(2, k, 2 * Nc, 45)
    if dtype == "f32":
        rf = rf.astype(np.float32).astype(np.float64)
    want = transfer.restrict_kron(2, k, Nc, rf)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(2, k, 2 * Nc, 2, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        rc = torch.full((want.size,), 3.0, dtype=tdt, device="cuda")
        ctx.restrict(1, dev(rf, tdt), rc)
        assert rel(host(rc), want) <= tol


@pytest.mark.parametrize("k,Nc", TRANSFER_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_prolong_2d(vps, k, Nc, dtype):
    import torch
    say("2D stream prolong", k, Nc, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ec = vi.seeded_vector(2, k, Nc, 46)
    uf = vi.seeded_vector(2, k, 2 * Nc, 47)
    if dtype == "f32":
        ec = ec.astype(np.float32).astype(np.float64)
        uf = uf.astype(np.float32).astype(np.float64)
    want = uf + transfer.prolong_kron(2, k, Nc, ec)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(2, k, 2 * Nc, 2, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        u = dev(uf, tdt)
        ctx.prolongate_add(1, dev(ec, tdt), u)
        assert rel(host(u), want) <= tol
