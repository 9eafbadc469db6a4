"""GPU parity of the 3D plane-streaming operator, residual and restriction kernels.

Sizes span several x-y tiles with a ragged last tile and several z chunks;
the full-size cases (the 3D Q4 problem on 128^3 cells) are checked on
sampled nodes, each computed by the oracle from the 1D matrices.
"""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, transfer, fe, mesh
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu

# (k, N): N cells per direction; x-y tiles hold 32, 16, 8 (x) and 32, 16, 10, 8 (y) cells for k = 1..4
OP_CASES = [(1, 70), (2, 36), (3, 25), (4, 20)]
RESTRICT_CASES = [(1, 35), (2, 18), (3, 12), (4, 9)]
# (k, Nc): coarse cells; prolongation tiles hold 16, 8, 5, 4 (x) and 32, 16, 8, 8 (y) coarse cells
PROLONG_CASES = [(1, 35), (2, 18), (3, 11), (4, 9)]


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("k,N", OP_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_and_residual_tiles(vps, k, N, dtype):
    import torch
    say("stream operator", k, N, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u0 = vi.seeded_vector(3, k, N, 21)
    b = vi.seeded_vector(3, k, N, 22)
    if dtype == "f32":  # the oracle sees the values the kernel sees
        u0 = u0.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    Au = assemble.matvec_kron(3, k, N, u0)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(3, k, N, 1, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        out = torch.full((u0.size,), 7.0, dtype=tdt, device="cuda")  # Dirichlet entries must be overwritten
        ctx.apply(0, dev(u0, tdt), out)
        assert rel(host(out), Au) <= tol
        out.fill_(7.0)
        ctx.residual(0, dev(b, tdt), dev(u0, tdt), out)
        assert rel(host(out), b - Au) <= tol


@pytest.mark.parametrize("k,Nc", RESTRICT_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_restrict_tiles(vps, k, Nc, dtype):
    import torch
    say("stream restrict", k, Nc, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    rf = vi.seeded_vector(3, k, 2 * Nc, 23)
    if dtype == "f32":
        rf = rf.astype(np.float32).astype(np.float64)
    want = transfer.restrict_kron(3, k, Nc, rf)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(3, k, 2 * Nc, 2, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        rc = torch.full((want.size,), 3.0, dtype=tdt, device="cuda")
        ctx.restrict(1, dev(rf, tdt), rc)
        assert rel(host(rc), want) <= tol


@pytest.mark.parametrize("k,Nc", PROLONG_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_prolong_tiles(vps, k, Nc, dtype):
    import torch
    say("stream prolong", k, Nc, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ec = vi.seeded_vector(3, k, Nc, 24)
    uf = vi.seeded_vector(3, k, 2 * Nc, 25)
    if dtype == "f32":
        ec = ec.astype(np.float32).astype(np.float64)
        uf = uf.astype(np.float32).astype(np.float64)
    want = uf + transfer.prolong_kron(3, k, Nc, ec)
    tol = 1e-13 if dtype == "f64" else 2e-6
    with vps.Context(3, k, 2 * Nc, 2, vcycle_dtype=dtype, stream_min_cells=1) as ctx:
        u = dev(uf, tdt)
        ctx.prolongate_add(1, dev(ec, tdt), u)
        assert rel(host(u), want) <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vcycle_same_with_stream_and_tile_kernels(vps, dtype):
    """3D Q3, 5 levels on 64^3 cells: both kernel families give the same V-cycle within rounding."""
    import torch
    say("vcycle stream vs tile", dtype)
    k, N, L = 3, 64, 5
    r = dev(vi.seeded_vector(3, k, N, 26))
    z = []
    for smin in (1, 1 << 30):
        with vps.Context(3, k, N, L, 2, 2, vcycle_dtype=dtype, stream_min_cells=smin) as ctx:
            out = torch.empty_like(r)
            ctx.vcycle(r, out)
            z.append(host(out))
    assert rel(z[0], z[1]) <= (1e-12 if dtype == "f64" else 1e-5)


# ---- full size, sampled ----

def _sample_nodes(n1, k, count, seed):
    """Random nodes plus nodes next to tile, chunk and domain boundaries."""
    rng = np.random.default_rng(seed)
    pts = [tuple(rng.integers(0, n1, size=3)) for _ in range(count)]
    edge = [e for e in (0, 1, k - 1, k, k + 1, 8 * k - 1, 8 * k, 8 * k + 1, n1 // 2, n1 - 2, n1 - 1) if 0 <= e < n1]
    for _ in range(count):
        pts.append(tuple(int(rng.choice(edge)) if rng.random() < 0.7 else int(rng.integers(0, n1)) for _ in range(3)))
    return pts


def _band(i, k, n1):
    lo = i - k if i % k == 0 else i - i % k
    hi = i + k if i % k == 0 else i - i % k + k
    return max(lo, 0), min(hi, n1 - 1) + 1


def _apply_at(U, M1, K1, k, n1, node):
    """(A u) at one node from the 1D matrices, and the sum of the magnitudes of its terms."""
    x, y, z = node
    if min(node) == 0 or max(node) == n1 - 1:
        return 0.0, 0.0
    (x0, x1), (y0, y1), (z0, z1) = _band(x, k, n1), _band(y, k, n1), _band(z, k, n1)
    blk = U[z0:z1, y0:y1, x0:x1]
    mx, kx = M1[x, x0:x1], K1[x, x0:x1]
    my, ky = M1[y, y0:y1], K1[y, y0:y1]
    mz, kz = M1[z, z0:z1], K1[z, z0:z1]
    w = (np.einsum("c,b,a->cba", mz, my, kx) + np.einsum("c,b,a->cba", mz, ky, mx) +
         np.einsum("c,b,a->cba", kz, my, mx))
    return float((w * blk).sum()), float(np.abs(w * blk).sum())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_full_size_sampled(vps, dtype):
    """3D Q4, 128^3 cells (513^3 nodes): FP64 operator of CG, FP32 residual of the V-cycle."""
    import torch
    k, N = 4, 128
    say("stream operator full size", dtype)
    n1 = k * N + 1
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u0 = vi.seeded_vector(3, k, N, 31)
    b = vi.seeded_vector(3, k, N, 32)
    if dtype == "f32":
        u0 = u0.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    M1, K1 = fe.assembled_1d(k, N)
    U = u0.reshape(n1, n1, n1)
    B = b.reshape(n1, n1, n1)
    eps = 1e-15 if dtype == "f64" else 1e-6
    with vps.Context(3, k, N, 1, vcycle_dtype=dtype) as ctx:  # the default path at this size is the streaming one
        out = torch.full((u0.size,), 7.0, dtype=tdt, device="cuda")
        ud = dev(u0, tdt)
        if dtype == "f64":
            ctx.apply(0, ud, out)
        else:
            ctx.residual(0, dev(b, tdt), ud, out)
        got = host(out).reshape(n1, n1, n1)
    del ud, out
    for node in _sample_nodes(n1, k, 300, 5):
        v, mag = _apply_at(U, M1, K1, k, n1, node)
        x, y, z = node
        want = v if dtype == "f64" else (0.0 if min(node) == 0 or max(node) == n1 - 1 else B[z, y, x] - v)
        assert abs(got[z, y, x] - want) <= 20 * eps * (mag + abs(want)) + 1e-300, node
    # the Dirichlet faces are exactly zero
    for face in (got[0], got[-1], got[:, 0], got[:, -1], got[:, :, 0], got[:, :, -1]):
        assert not np.any(face)


def test_restrict_full_size_sampled(vps):
    """Restriction 513^3 -> 257^3 (3D Q4), FP32 as in the V-cycle, on sampled coarse nodes."""
    import torch
    k, Nc = 4, 64
    say("stream restrict full size")
    nf, nc = 2 * k * Nc + 1, k * Nc + 1
    rf = vi.seeded_vector(3, k, 2 * Nc, 33).astype(np.float32).astype(np.float64)
    P1 = transfer.prolongation_1d(k, Nc)
    with vps.Context(3, k, 2 * Nc, 2, vcycle_dtype="f32") as ctx:
        rc = torch.full((nc ** 3,), 3.0, dtype=torch.float32, device="cuda")
        ctx.restrict(1, dev(rf, torch.float32), rc)
        got = host(rc).reshape(nc, nc, nc)
    R = rf.reshape(nf, nf, nf)
    for node in _sample_nodes(nc, k, 300, 6):
        x, y, z = node
        if min(node) == 0 or max(node) == nc - 1:
            assert got[z, y, x] == 0.0
            continue
        cols = [np.nonzero(P1[:, i])[0] for i in (x, y, z)]
        w = np.einsum("c,b,a->cba", P1[cols[2], z], P1[cols[1], y], P1[cols[0], x])
        blk = R[np.ix_(cols[2], cols[1], cols[0])]
        want = float((w * blk).sum())
        assert abs(got[z, y, x] - want) <= 2e-5 * float(np.abs(w * blk).sum()) + 1e-30, node


def test_prolong_full_size_sampled(vps):
    """Prolongation 257^3 -> 513^3 (3D Q4), FP32 as in the V-cycle, on sampled fine nodes."""
    import torch
    k, Nc = 4, 64
    say("stream prolong full size")
    nf, nc = 2 * k * Nc + 1, k * Nc + 1
    ec = vi.seeded_vector(3, k, Nc, 34).astype(np.float32).astype(np.float64)
    uf = vi.seeded_vector(3, k, 2 * Nc, 35).astype(np.float32).astype(np.float64)
    P1 = transfer.prolongation_1d(k, Nc)
    with vps.Context(3, k, 2 * Nc, 2, vcycle_dtype="f32") as ctx:
        u = dev(uf, torch.float32)
        ctx.prolongate_add(1, dev(ec, torch.float32), u)
        got = host(u).reshape(nf, nf, nf)
    E = ec.reshape(nc, nc, nc)
    U = uf.reshape(nf, nf, nf)
    for node in _sample_nodes(nf, k, 300, 7):
        x, y, z = node
        if min(node) == 0 or max(node) == nf - 1:
            assert got[z, y, x] == U[z, y, x]
            continue
        rows = [np.nonzero(P1[i])[0] for i in (x, y, z)]
        w = np.einsum("c,b,a->cba", P1[z, rows[2]], P1[y, rows[1]], P1[x, rows[0]])
        blk = E[np.ix_(rows[2], rows[1], rows[0])]
        want = U[z, y, x] + float((w * blk).sum())
        assert abs(got[z, y, x] - want) <= 2e-5 * (float(np.abs(w * blk).sum()) + abs(U[z, y, x])) + 1e-30, node
