"""GPU parity of the V-cycle and the solvers against the oracle."""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import assemble, multigrid
from tests.gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vps():
    from paper_2407_02100_amd import vps as m
    return m


@pytest.mark.parametrize("dim,k,N,L,pre,post", [(2, 2, 16, 3, 1, 1), (2, 3, 8, 2, 2, 2), (3, 2, 8, 2, 1, 1),
                                                (3, 4, 8, 2, 1, 1)])
def test_vcycle_fp64(vps, dim, k, N, L, pre, post):
    say("vcycle", dim, k, N, L)
    H = multigrid.Hierarchy(dim, k, N, L, pre, post)
    r = vi.seeded_vector(dim, k, N, 21)
    want = H.vcycle(r)
    import torch
    with vps.Context(dim, k, N, L, pre, post) as ctx:
        z = torch.empty(r.size, dtype=torch.float64, device="cuda")
        ctx.vcycle(dev(r), z)
        assert rel(host(z), want) <= 1e-11


def test_vcycle_symmetric(vps):
    dim, k, N, L = 3, 3, 8, 2
    say("vcycle symmetry", dim, k, N)
    import torch
    with vps.Context(dim, k, N, L, 2, 2) as ctx:
        x = dev(vi.seeded_vector(dim, k, N, 22))
        y = dev(vi.seeded_vector(dim, k, N, 23))
        Vx = torch.empty_like(x)
        Vy = torch.empty_like(y)
        ctx.vcycle(x, Vx)
        ctx.vcycle(y, Vy)
        a = float((Vx * y).sum())
        b = float((x * Vy).sum())
        assert abs(a - b) <= 1e-11 * abs(a)
        assert float((Vx * x).sum()) > 0


def _recheck(dim, k, N, b, x):
    if N <= 32 or dim == 2:
        A = assemble.assemble_kron(dim, k, N)
        return np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    return np.linalg.norm(b - assemble.matvec_kron(dim, k, N, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("name", ["poisson2d_q2_n32", "poisson3d_q4_n32"])
def test_solve_workload_fp64(vps, name):
    w = vi.WORKLOADS[name]
    say("solve", name)
    dim, k, N = w["dim"], w["degree"], w["n_cells"]
    b = vi.seeded_vector(dim, k, N, w["rhs_seed"])
    import torch
    with vps.Context(dim, k, N, w["levels"], w["pre"], w["post"]) as ctx:
        x = torch.empty(b.size, dtype=torch.float64, device="cuda")
        info = ctx.solve(dev(b), x, rtol=1e-10, maxit=50)
        xs = host(x)
    assert info["rel_residual_true"] <= 1e-10
    assert _recheck(dim, k, N, b, xs) <= 1e-10
    assert 2 <= info["iterations"] <= 20
    if name == "poisson2d_q2_n32":
        H = multigrid.Hierarchy(dim, k, N, w["levels"], w["pre"], w["post"])
        xo, ito, _ = multigrid.pcg(H, b, 1e-10)
        assert abs(ito - info["iterations"]) <= 1
        assert np.linalg.norm(xs - xo) <= 1e-8 * np.linalg.norm(xo)


def test_solve_mixed_precision(vps):
    dim, k, N, L = 3, 3, 16, 3
    say("solve mixed", dim, k, N)
    b = vi.seeded_vector(dim, k, N, 31)
    import torch
    res = {}
    for vt in ("f64", "f32"):
        with vps.Context(dim, k, N, L, 1, 1, vcycle_dtype=vt) as ctx:
            x = torch.empty(b.size, dtype=torch.float64, device="cuda")
            info = ctx.solve(dev(b), x, rtol=1e-10, maxit=60)
            res[vt] = (info, host(x))
    for vt, (info, xs) in res.items():
        assert info["rel_residual_true"] <= 1e-10, vt
        assert _recheck(dim, k, N, b, xs) <= 1e-10
    assert res["f32"][0]["iterations"] <= res["f64"][0]["iterations"] + 3
    assert np.linalg.norm(res["f32"][1] - res["f64"][1]) <= 1e-8 * np.linalg.norm(res["f64"][1])


def test_solve_reports_not_converged_and_nonfinite(vps):
    dim, k, N, L = 2, 2, 16, 3
    import torch
    b = vi.seeded_vector(dim, k, N, 32)
    with vps.Context(dim, k, N, L) as ctx:
        x = torch.empty(b.size, dtype=torch.float64, device="cuda")
        info = ctx.solve(dev(b), x, rtol=1e-10, maxit=1, check=False)
        assert info["status"] == vps.VPS_E_NOT_CONVERGED
        bad = b.copy()
        bad[bad.size // 2] = np.nan
        info = ctx.solve(dev(bad), x, rtol=1e-10, maxit=5, check=False)
        assert info["status"] == vps.VPS_E_NONFINITE


def test_stationary_iteration_converges(vps):
    dim, k, N, L = 2, 3, 16, 3
    b = vi.seeded_vector(dim, k, N, 33)
    H = multigrid.Hierarchy(dim, k, N, L)
    f_or, hist_or = multigrid.stationary_factor(H, b, 3, 8)
    import torch
    with vps.Context(dim, k, N, L) as ctx:
        u = torch.zeros(b.size, dtype=torch.float64, device="cuda")
        hist = ctx.vcycle_iterate(dev(b), u, 8)
    assert rel(np.array(hist), np.array(hist_or)) <= 1e-6


@pytest.mark.parametrize("dim,k,N,L", [(2, 5, 16, 4), (3, 5, 8, 3)])
def test_solve_degree5(vps, dim, k, N, L):
    """Q5 (the paper's element) down to a single-patch coarse grid (2 cells per direction)."""
    say("solve Q5", dim, N, L)
    b = vi.seeded_vector(dim, k, N, 71)
    import torch
    with vps.Context(dim, k, N, L) as ctx:
        x = torch.empty(b.size, dtype=torch.float64, device="cuda")
        info = ctx.solve(dev(b), x, rtol=1e-10, maxit=60)
        xs = host(x)
    assert info["rel_residual_true"] <= 1e-10
    assert _recheck(dim, k, N, b, xs) <= 1e-10
    if dim == 2:
        H = multigrid.Hierarchy(dim, k, N, L)
        xo, ito, _ = multigrid.pcg(H, b, 1e-10)
        assert abs(ito - info["iterations"]) <= 1
