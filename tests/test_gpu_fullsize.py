"""GPU checks at the full workload sizes, in the configuration the benchmark times.

* 3D Q4 on 128^3 cells (513^3 nodes): one color of the smoother checked on
  sampled patches, each solved by the oracle from its closure (dense patch
  operator, exact local solve); the nodes outside the color's interiors are
  untouched; the residual vanishes on the color's interiors afterwards
  (exact local solves); the mixed-precision solve's true residual is
  recomputed on the host with the oracle's Kronecker-form product.
* The paper's 3D Q5 shape, 128^3 cells (641^3 nodes): one color on sampled
  patches as above, one patch per wave and a row of five per workgroup.
* 3D Q3 on 64^3 cells: plain FP64 and FP32-preconditioned solves, rechecked on
  the host, same solution.
* 3D Q2 on 64^3 cells with rho = exp(GRF): plain rhobar-FDM and learned
  scaling, rechecked on the host with the oracle's cell-by-cell product.
"""
import functools

import numpy as np
import pytest
import scipy.linalg as sla

import vps_inputs as vi
from oracle import assemble, mesh, smoother
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

K5, N5 = 4, 128  # 3D Q4, 128^3 cells


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


def _color_interior_mask(dim, k, n_cells, color):
    """Nodes strictly inside the patches of one color (1D masks, outer product)."""
    n1 = k * n_cells + 1
    masks = []
    for e in range(dim):
        m = np.zeros(n1, dtype=bool)
        for v in range(1, n_cells):
            if v % 2 == (color >> e) & 1:
                m[k * (v - 1) + 1:k * (v + 1)] = True
        masks.append(m)
    out = np.ones((n1,) * dim, dtype=bool)
    for e in range(dim):
        shape = [1] * dim
        shape[dim - 1 - e] = n1
        out = out & masks[e].reshape(shape)
    return out.reshape(-1)


def _sample_vertices(n_cells, color, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    par = [(color >> e) & 1 for e in range(3)]

    def pick(e, special):
        cand = [v for v in range(1, n_cells) if v % 2 == par[e]]
        if special:
            return int(rng.choice([cand[0], cand[-1], cand[len(cand) // 8], cand[len(cand) // 2]]))
        return int(rng.choice(cand))

    for i in range(count):
        out.append(tuple(pick(e, i % 3 == 0) for e in range(3)))
    return out


@pytest.mark.parametrize("dtype,color", [("f32", 0), ("f32", 5), ("f64", 3)])
@pytest.mark.parametrize("ppw", [1, 2, 3])
def test_color_on_sampled_patches_full_size(vps, dtype, color, ppw):
    """One color launch at 513^3 against the oracle's exact local solve of sampled patches (one patch, two
    patches or a row of seven per wave)."""
    import torch
    k, N = K5, N5
    say("full-size color", dtype, color, ppw)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    u0 = vi.seeded_vector(3, k, N, 105)
    b = vi.seeded_vector(3, k, N, 5)
    if dtype == "f32":  # the oracle sees the values the kernel sees
        u0 = u0.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    with vps.Context(3, k, N, 1, vcycle_dtype=dtype, patches_per_wave=ppw) as ctx:
        u = dev(u0, tdt)
        ctx.smooth_color(0, u, dev(b, tdt), color)
        u1 = host(u)
        del u
    mask = _color_interior_mask(3, k, N, color)
    assert np.array_equal(u1[~mask], u0[~mask])  # nothing outside the color's interiors is written
    h = 1.0 / N
    Abar = smoother.patch_closure_operator(3, k, h)
    ipos = smoother.closure_interior_positions(3, k)
    gpos = np.setdiff1d(np.arange(Abar.shape[0]), ipos)
    cho = sla.cho_factor(Abar[np.ix_(ipos, ipos)])
    Aig = Abar[np.ix_(ipos, gpos)]
    tol = 5e-5 if dtype == "f32" else 1e-11  # FP64: cond(A_j) * eps
    for v in _sample_vertices(N, color, 60, 11 + color):
        clo = mesh.patch_closure(3, k, N, v)
        inner = clo[ipos]
        want = sla.cho_solve(cho, b[inner] - Aig @ u0[clo[gpos]])
        got = u1[inner]
        assert np.abs(got - want).max() <= tol * np.abs(want).max(), v


@functools.lru_cache(maxsize=1)
def _q5_inputs():
    return vi.seeded_vector(3, 5, 128, 113), vi.seeded_vector(3, 5, 128, 13)


@pytest.mark.parametrize("dtype,color", [("f64", 3), ("f64", 6), ("f32", 5)])
@pytest.mark.parametrize("ppw", [1, 3])
def test_color_on_sampled_patches_paper_q5_shape(vps, dtype, color, ppw):
    """The paper's 3D Q5 shape, 128^3 cells (641^3 nodes): one color launch (one patch per wave, or a row of
    five patches per workgroup of two waves, the automatic choice there) against the oracle's exact local
    solve of sampled patches; cond(A_j) is about 68 at k = 5."""
    import torch
    k, N = 5, 128
    say("paper Q5 shape color", dtype, color, ppw)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    u0, b = _q5_inputs()
    if dtype == "f32":
        u0 = u0.astype(np.float32).astype(np.float64)
        b = b.astype(np.float32).astype(np.float64)
    with vps.Context(3, k, N, 1, vcycle_dtype=dtype, patches_per_wave=ppw) as ctx:
        u = dev(u0, tdt)
        ctx.smooth_color(0, u, dev(b, tdt), color)
        u1 = host(u)
        del u
    mask = _color_interior_mask(3, k, N, color)
    assert np.array_equal(u1[~mask], u0[~mask])
    Abar = smoother.patch_closure_operator(3, k, 1.0 / N)
    ipos = smoother.closure_interior_positions(3, k)
    gpos = np.setdiff1d(np.arange(Abar.shape[0]), ipos)
    cho = sla.cho_factor(Abar[np.ix_(ipos, ipos)])
    Aig = Abar[np.ix_(ipos, gpos)]
    tol = 5e-5 if dtype == "f32" else 1e-11
    for v in _sample_vertices(N, color, 40, 31 + color):
        clo = mesh.patch_closure(3, k, N, v)
        inner = clo[ipos]
        want = sla.cho_solve(cho, b[inner] - Aig @ u0[clo[gpos]])
        assert np.abs(u1[inner] - want).max() <= tol * np.abs(want).max(), v


def test_residual_vanishes_on_color_interiors_full_size(vps):
    """Exact local solves: after a color, b - A u is zero on that color's interiors (FP64, 513^3)."""
    import torch
    k, N, color = K5, N5, 6
    say("full-size residual after a color")
    u0 = vi.seeded_vector(3, k, N, 106)
    b = vi.seeded_vector(3, k, N, 6)
    mask = _color_interior_mask(3, k, N, color)
    with vps.Context(3, k, N, 1, vcycle_dtype="f64") as ctx:
        u, bd = dev(u0), dev(b)
        r = torch.empty_like(u)
        ctx.residual(0, bd, u, r)
        before = np.abs(host(r)[mask]).max()
        ctx.smooth_color(0, u, bd, color)
        ctx.residual(0, bd, u, r)
        rr = host(r)
    after = np.abs(rr[mask]).max()
    assert before > 0.1
    assert after <= 1e-10 * before  # cond(A_j) * eps
    assert np.abs(rr[~mask]).max() > 1e-3 * before  # elsewhere the residual is not annihilated


def test_solve_full_size_host_recheck(vps):
    """3D Q4, 128^3 cells, 6 levels, V(2,2), FP32 V-cycle in FP64 flexible CG, the slabs the benchmark
    sweeps: true residual on the host."""
    import torch
    w = vi.WORKLOADS["poisson3d_q4_n128"]
    say("full-size solve")
    b = vi.seeded_vector(3, w["degree"], w["n_cells"], w["rhs_seed"])
    with vps.Context(3, w["degree"], w["n_cells"], w["levels"], w["pre"], w["post"], vcycle_dtype=w["vcycle"],
                     batch_layers=w["batch_layers"]) as ctx:
        x = torch.empty(b.size, dtype=torch.float64, device="cuda")
        info = ctx.solve(dev(b), x, rtol=1e-10, maxit=50)
        xs = host(x)
        del x
    assert info["rel_residual_true"] <= 1e-10
    assert 2 <= info["iterations"] <= 12
    say("host recheck", info)
    res = np.linalg.norm(b - assemble.matvec_kron(3, w["degree"], w["n_cells"], xs)) / np.linalg.norm(b)
    assert res <= 1e-10
    assert abs(res - info["rel_residual_true"]) <= 1e-3 * res + 1e-14


def test_mixed_and_plain_solve_q3(vps):
    """3D Q3, 64^3 cells, 5 levels: FP32 V-cycle (flexible CG) and plain FP64 reach the same solution."""
    import torch
    w = vi.WORKLOADS["poisson3d_q3_n64"]
    k, N = w["degree"], w["n_cells"]
    say("Q3 64^3 mixed vs plain")
    b = vi.seeded_vector(3, k, N, w["rhs_seed"])
    out = {}
    for vt in ("f64", "f32"):
        with vps.Context(3, k, N, w["levels"], w["pre"], w["post"], vcycle_dtype=vt) as ctx:
            x = torch.empty(b.size, dtype=torch.float64, device="cuda")
            info = ctx.solve(dev(b), x, rtol=1e-10, maxit=50)
            out[vt] = (info, host(x))
    for vt, (info, xs) in out.items():
        res = np.linalg.norm(b - assemble.matvec_kron(3, k, N, xs)) / np.linalg.norm(b)
        assert info["rel_residual_true"] <= 1e-10 and res <= 1e-10, vt
    assert out["f32"][0]["iterations"] <= out["f64"][0]["iterations"] + 2
    x64, x32 = out["f64"][1], out["f32"][1]
    assert np.linalg.norm(x32 - x64) <= 1e-8 * np.linalg.norm(x64)


def test_learned_and_plain_solve_varcoef(vps):
    """3D Q2, 64^3 cells, rho = exp(GRF) (test seed 4): plain rhobar-FDM and learned scaling."""
    import torch
    from paper_2407_02100_amd import learned
    w = vi.WORKLOADS["varcoef3d_q2_n64"]
    k, N = w["degree"], w["n_cells"]
    say("Q2 64^3 variable coefficient, plain vs learned")
    X, T, C, R = learned.training_set([1000, 1001, 1002], n_cells=N, levels=w["levels"], total=60_000)
    params, hist = learned.train(X, T, epochs=20)
    assert hist["val_loss"][-1] < 0.1 * learned.baseline_loss(T)
    rho = vi.rho_cells(N, w["rho_seed"])
    b = vi.seeded_vector(3, k, N, w["rhs_seed"])
    out = {}
    for mode in ("mean", "learned"):
        with vps.Context(3, k, N, w["levels"], w["pre"], w["post"], coef=mode) as ctx:
            ctx.set_coefficient(dev(rho))
            if mode == "learned":
                assert all(f == 0 for f in learned.apply_scaling(ctx, params))
            x = torch.empty(b.size, dtype=torch.float64, device="cuda")
            info = ctx.solve(dev(b), x, rtol=1e-10, maxit=100)
            out[mode] = (info, host(x))
    for mode, (info, xs) in out.items():
        res = np.linalg.norm(b - assemble.matvec_cells(3, k, N, rho, xs)) / np.linalg.norm(b)
        assert info["rel_residual_true"] <= 1e-10 and res <= 1e-10, mode
    assert out["learned"][0]["iterations"] <= out["mean"][0]["iterations"] + 1
    assert np.linalg.norm(out["learned"][1] - out["mean"][1]) <= 1e-7 * np.linalg.norm(out["mean"][1])


def test_fp64_sweep_all_colors_full_size(vps):
    """One FP64 sweep at 513^3 in the bench's kernel choice (automatic: a row of seven patches per wave),
    color by color: each color's update of 40 sampled patches against the oracle's exact local solve from the
    GPU's state before that color, to the stated FP64 sweep tolerance, ||u_gpu - u_oracle||_2 <=
    1e-12 ||u_oracle||_2 over the sampled interiors (and 1e-11 per patch in the max norm)."""
    import torch
    k, N = K5, N5
    u0 = vi.seeded_vector(3, k, N, 107)
    b = vi.seeded_vector(3, k, N, 7)
    h = 1.0 / N
    Abar = smoother.patch_closure_operator(3, k, h)
    ipos = smoother.closure_interior_positions(3, k)
    gpos = np.setdiff1d(np.arange(Abar.shape[0]), ipos)
    cho = sla.cho_factor(Abar[np.ix_(ipos, ipos)])
    Aig = Abar[np.ix_(ipos, gpos)]
    with vps.Context(3, k, N, 1, vcycle_dtype="f64") as ctx:
        u, bd = dev(u0), dev(b)
        prev = u0
        for color in range(8):
            say("full-size FP64 sweep, color", color)
            ctx.smooth_color(0, u, bd, color)
            cur = host(u)
            mask = _color_interior_mask(3, k, N, color)
            assert np.array_equal(cur[~mask], prev[~mask])
            num = den = 0.0
            for v in _sample_vertices(N, color, 40, 31 + color):
                clo = mesh.patch_closure(3, k, N, v)
                inner = clo[ipos]
                want = sla.cho_solve(cho, b[inner] - Aig @ prev[clo[gpos]])
                got = cur[inner]
                assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max(), (color, v)
                num += float(np.sum((got - want) ** 2))
                den += float(np.sum(want ** 2))
            say("  relative 2-norm error over the sampled interiors", (num / den) ** 0.5)
            assert (num / den) ** 0.5 <= 1e-12, color
            prev = cur
