"""Pins of the oracle's multigrid and Krylov solvers."""
import numpy as np
import pytest

import vps_inputs as vi
from oracle import multigrid, manufactured, mesh


@pytest.mark.parametrize("dim,k,Ns", [(2, 1, (4, 8, 16)), (2, 2, (4, 8, 16)), (2, 3, (4, 8)), (2, 4, (4, 8)),
                                     (2, 5, (4, 8)), (3, 2, (4, 8)), (3, 3, (4, 8)), (3, 5, (4, 8))])
def test_manufactured_convergence_rate(dim, k, Ns):
    """L2 error ratio under refinement tends to 2^(k+1)."""
    errs = []
    for N in Ns:
        H = multigrid.Hierarchy(dim, k, N, 2)
        b = manufactured.load_vector(dim, k, N)
        x, it, res = multigrid.pcg(H, b, rtol=1e-12)
        assert res <= 1e-12
        errs.append(manufactured.l2_error(dim, k, N, x))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 1 - 0.25, (errs, rates)


@pytest.mark.parametrize("dim,k,N", [(2, 2, 4), (3, 2, 4)])
def test_brute_force_dense_solve(dim, k, N):
    H = multigrid.Hierarchy(dim, k, N, 2)
    b = vi.seeded_vector(dim, k, N, 11)
    x, it, res = multigrid.pcg(H, b, rtol=1e-12)
    free = mesh.free_mask_flat(dim, k, N)
    xs = np.zeros_like(b)
    xs[free] = np.linalg.solve(H.A.toarray()[np.ix_(free, free)], b[free])
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_vcycle_is_symmetric_positive():
    dim, k, N = 2, 3, 8
    H = multigrid.Hierarchy(dim, k, N, 3, pre=2, post=2)
    x = vi.seeded_vector(dim, k, N, 12)
    y = vi.seeded_vector(dim, k, N, 13)
    Vx, Vy = H.vcycle(x), H.vcycle(y)
    assert abs(Vx @ y - x @ Vy) <= 1e-12 * abs(Vx @ y)
    assert Vx @ x > 0 and Vy @ y > 0


def test_iteration_count_range_2d_q2():
    """A Q2 2D problem with 4 levels converges to 1e-10 in a handful of iterations."""
    w = vi.WORKLOADS["poisson2d_q2_n32"]
    H = multigrid.Hierarchy(w["dim"], w["degree"], w["n_cells"], w["levels"], w["pre"], w["post"])
    b = vi.seeded_vector(w["dim"], w["degree"], w["n_cells"], w["rhs_seed"])
    x, it, res = multigrid.pcg(H, b, rtol=1e-10)
    assert res <= 1e-10
    assert 3 <= it <= 12
    rho, _ = multigrid.stationary_factor(H, b, 3, 8)
    assert rho < 0.2


def test_flexible_cg_matches_cg_with_fixed_preconditioner():
    dim, k, N = 2, 2, 8
    H = multigrid.Hierarchy(dim, k, N, 3)
    b = vi.seeded_vector(dim, k, N, 14)
    x1, it1, _ = multigrid.pcg(H, b, 1e-10)
    x2, it2, _ = multigrid.pcg(H, b, 1e-10, flexible=True)
    assert abs(it1 - it2) <= 1
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)


def test_variable_coefficient_hierarchy_converges():
    """Exact local solves on a rough field: PCG reaches the dense solution."""
    dim, k, N = 3, 2, 8
    rho = vi.rho_cells(N, 3)
    H = multigrid.Hierarchy(dim, k, N, 2, rho=rho, mode="exact")
    b = vi.seeded_vector(dim, k, N, 15)
    x, it, res = multigrid.pcg(H, b, 1e-10)
    assert res <= 1e-10
    free = mesh.free_mask_flat(dim, k, N)
    xs = np.zeros_like(b)
    xs[free] = np.linalg.solve(H.A.toarray()[np.ix_(free, free)], b[free])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_variable_coefficient_mean_fdm_smooth_field():
    """rhobar-FDM local solvers on a smooth field (correlation length 4 cells) converge in PCG."""
    dim, k, N = 3, 2, 8
    rho = vi.rho_cells(N, 3, corr_len=0.5, std=0.5)
    H = multigrid.Hierarchy(dim, k, N, 2, rho=rho, mode="mean")
    b = vi.seeded_vector(dim, k, N, 16)
    x, it, res = multigrid.pcg(H, b, 1e-10, maxit=60)
    assert res <= 1e-10
