"""GPU parity of the smoother, operator, transfers and coarse solver against the oracle."""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, smoother, transfer, mesh
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# sizes chosen so that the colors have ragged batches along x (5 and 4 patches etc.)
CASES = [(2, 1, 10), (2, 2, 11), (2, 3, 10), (2, 4, 9), (2, 5, 7), (3, 1, 9), (3, 2, 7), (3, 3, 5), (3, 4, 5),
         (3, 5, 4)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


def _oracle(dim, k, N, rho=None, mode="shared", scaling=None):
    A = assemble.assemble(dim, k, N, rho)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, mode, rho=rho, scaling=scaling)
    return A, P, S


@pytest.mark.parametrize("dim,k,N", CASES)
def test_smooth_color_fp64(vps, dim, k, N):
    say("smooth_color", dim, k, N)
    A, P, S = _oracle(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 1)
    uo = vi.seeded_vector(dim, k, N, 2)
    with vps.Context(dim, k, N, 1) as ctx:
        u = dev(uo)
        bd = dev(b)
        for c in range(2 ** dim):
            ctx.smooth_color(0, u, bd, c)
            uo = smoother.apply_color(A, b, uo, P, S, c)
            assert rel(host(u), uo) <= 1e-12, (c, rel(host(u), uo))


@pytest.mark.parametrize("dim,k,N", [(2, 2, 11), (3, 2, 7), (3, 4, 5)])
@pytest.mark.parametrize("reverse", [False, True])
def test_sweep_fp64(vps, dim, k, N, reverse):
    say("sweep", dim, k, N, reverse)
    A, P, S = _oracle(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 3)
    u0 = vi.seeded_vector(dim, k, N, 4)
    want = smoother.sweep_colorized(A, b, u0, P, S, reverse)
    want = smoother.sweep_colorized(A, b, want, P, S, reverse)
    with vps.Context(dim, k, N, 1) as ctx:
        u = dev(u0)
        ctx.smooth(0, u, dev(b), sweeps=2, reverse=reverse)
        assert rel(host(u), want) <= 1e-12


@pytest.mark.parametrize("dim,k,N", [(2, 3, 10), (3, 2, 9), (3, 3, 5)])
def test_sweep_bitwise_independent_of_batch(vps, dim, k, N):
    """Each DoF is written by one patch per color, so the batch size cannot change any bit."""
    say("batch invariance", dim, k, N)
    b = dev(vi.seeded_vector(dim, k, N, 5))
    outs = []
    for pb in (1, 2, 4):
        try:
            ctx = vps.Context(dim, k, N, 1, patches_per_block=pb)
        except vps.VpsError:
            continue
        with ctx:
            u = dev(vi.seeded_vector(dim, k, N, 6))
            try:
                ctx.smooth(0, u, b, sweeps=1)
            except vps.VpsError:
                continue
            outs.append(host(u))
    assert len(outs) >= 2
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_fp32_sweep_close_to_fp64(vps):
    dim, k, N = 3, 3, 5
    say("fp32 sweep", dim, k, N)
    A, P, S = _oracle(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 7)
    u0 = vi.seeded_vector(dim, k, N, 8)
    want = smoother.sweep_colorized(A, b, u0, P, S)
    import torch
    with vps.Context(dim, k, N, 1, vcycle_dtype="f32") as ctx:
        u = dev(u0, torch.float32)
        ctx.smooth(0, u, dev(b, torch.float32), sweeps=1)
        assert rel(host(u), want) <= 1e-5


@pytest.mark.parametrize("dim,k,N", CASES)
def test_apply_and_residual(vps, dim, k, N):
    say("apply", dim, k, N)
    A = assemble.assemble(dim, k, N)
    u0 = vi.seeded_vector(dim, k, N, 9)
    b = vi.seeded_vector(dim, k, N, 10)
    import torch
    with vps.Context(dim, k, N, 1) as ctx:
        out = torch.full((u0.size,), 7.0, dtype=torch.float64, device="cuda")  # Dirichlet entries must be overwritten
        ctx.apply(0, dev(u0), out)
        assert rel(host(out), A @ u0) <= 1e-13
        ctx.residual(0, dev(b), dev(u0), out)
        assert rel(host(out), b - A @ u0) <= 1e-13


@pytest.mark.parametrize("dim,k,Nc", [(2, 1, 5), (2, 2, 3), (2, 4, 3), (2, 5, 3), (3, 1, 3), (3, 2, 3), (3, 3, 2),
                                      (3, 4, 2), (3, 5, 2)])
def test_transfers(vps, dim, k, Nc):
    say("transfer", dim, k, Nc)
    P = transfer.prolongation(dim, k, Nc)
    rf = vi.seeded_vector(dim, k, 2 * Nc, 11)
    ec = vi.seeded_vector(dim, k, Nc, 12)
    uf = vi.seeded_vector(dim, k, 2 * Nc, 13)
    import torch
    with vps.Context(dim, k, 2 * Nc, 2) as ctx:
        rc = torch.full((ec.size,), 3.0, dtype=torch.float64, device="cuda")
        ctx.restrict(1, dev(rf), rc)
        assert rel(host(rc), P.T @ rf) <= 1e-13
        u = dev(uf)
        ctx.prolongate_add(1, dev(ec), u)
        assert rel(host(u), uf + P @ ec) <= 1e-13


@pytest.mark.parametrize("dim,k,N0", [(2, 2, 4), (2, 4, 8), (3, 2, 4), (3, 4, 4), (3, 3, 4), (2, 5, 4), (3, 5, 2)])
def test_coarse_solve(vps, dim, k, N0):
    say("coarse", dim, k, N0)
    A = assemble.assemble(dim, k, N0)
    free = mesh.free_mask_flat(dim, k, N0)
    b = vi.seeded_vector(dim, k, N0, 14)
    x = np.zeros_like(b)
    x[free] = np.linalg.solve(A.toarray()[np.ix_(free, free)], b[free])
    import torch
    with vps.Context(dim, k, N0, 1) as ctx:
        xd = torch.full((b.size,), 5.0, dtype=torch.float64, device="cuda")
        ctx.coarse_solve(dev(b), xd)
        assert rel(host(xd), x) <= 1e-12


@pytest.mark.parametrize("k,N", [(4, 20), (3, 9), (2, 13)])
def test_patch_order_bitwise(vps, k, N):
    """The patches of one color are independent: every visiting order gives the same bits (one patch per wave)."""
    import torch
    say("patch order", k, N)
    b = vi.seeded_vector(3, k, N, 61)
    u0 = vi.seeded_vector(3, k, N, 62)
    out = []
    for order in range(4):
        with vps.Context(3, k, N, 1, patch_order=order, patches_per_wave=1) as ctx:
            u = dev(u0)
            ctx.smooth(0, u, dev(b), sweeps=1)
            out.append(host(u))
    for o in out[1:]:
        assert np.array_equal(o, out[0])
