"""Pins of the oracle's variable-coefficient pieces against facts that do not use them.

* coarse-level coefficient (mean of the 2^d children, the rediscretisation
  reading of the coarse rho): block-constant fields and a field linear in the
  cell index, whose child mean is the value at the coarse cell's centre;
* local solver 'mean' (B_j = (rhobar_j A_b)^{-1}, the fast-diagonalisation
  inverse of Appendix A.3 built for the patch mean) and 'learned'
  (B_j = S diag(c_j / (rhobar_j Lambda)) S^T, eq:fdm:inverse with a per-mode
  factor): both are read out as matrices through ``LocalSolvers.apply`` and
  checked against the Rayleigh-quotient bound of A_j(rho) against A_b, the
  exactness on patches whose cells share one coefficient, and the action on
  tensor products of 1D eigenvectors computed here with SciPy;
* MLP features log(rho_c / rhobar).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assemble, learned, mesh, smoother


def _solver_matrix(S, j, q):
    """B_j of LocalSolvers S as a dense matrix (columns = B_j e_i through S.apply)."""
    return np.column_stack([S.apply(j, e) for e in np.eye(q)])


# ---- coarse-level coefficient -------------------------------------------------

@pytest.mark.parametrize("dim,n", [(2, 8), (3, 4), (3, 8)])
def test_coarsen_block_constant_field_returns_block_values(dim, n):
    rng = np.random.default_rng(11)
    nc = n // 2
    blocks = rng.uniform(0.1, 10.0, size=(nc,) * dim)  # [z][y][x] (x fastest when flattened)
    fine = blocks
    for ax in range(dim):
        fine = np.repeat(fine, 2, axis=ax)
    got = mesh.coarsen_cells(fine.reshape(-1), dim, n)
    assert np.allclose(got, blocks.reshape(-1), rtol=1e-15, atol=0)


@pytest.mark.parametrize("dim,n", [(2, 8), (3, 8)])
def test_coarsen_linear_field_gives_centre_values(dim, n):
    """rho = sum_e w_e c_e over cell indices (x fastest): the 2^d children of coarse cell C have
    c_e in {2 C_e, 2 C_e + 1}, so their mean is sum_e w_e (2 C_e + 1/2).  Distinct weights per axis
    catch a transposed axis or a wrong child offset."""
    w = [1.0, 10.0, 100.0][:dim]
    fine = np.zeros(n ** dim)
    for idx in itertools.product(range(n), repeat=dim):  # idx = (c_slowest, ..., c_x)
        c = idx[::-1]
        fine[mesh.flat_index(c, n)] = sum(w[e] * c[e] for e in range(dim))
    nc = n // 2
    want = np.zeros(nc ** dim)
    for idx in itertools.product(range(nc), repeat=dim):
        C = idx[::-1]
        want[mesh.flat_index(C, nc)] = sum(w[e] * (2 * C[e] + 0.5) for e in range(dim))
    assert np.allclose(mesh.coarsen_cells(fine, dim, n), want, rtol=0, atol=1e-12)


def test_coarsen_preserves_the_total():
    rng = np.random.default_rng(12)
    f = np.exp(rng.standard_normal(8 ** 3))
    c = mesh.coarsen_cells(f, 3, 8)
    assert abs(c.sum() * 8 - f.sum()) <= 1e-12 * f.sum()


# ---- local solver 'mean' ---------------------------------------------------------

def _rho_field(dim, n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * np.exp(1.2 * rng.standard_normal(n ** dim))


@pytest.mark.parametrize("dim,k,n", [(2, 2, 4), (3, 2, 3)])
def test_mean_solver_with_constant_rho_equals_exact(dim, k, n):
    """rho = alpha everywhere: A_j = alpha A_b and rhobar_j = alpha, so 'mean' is the exact local solver."""
    alpha = 3.7
    rho = np.full(n ** dim, alpha)
    A = assemble.assemble(dim, k, n, rho)
    P = smoother.Patches(dim, k, n)
    Sm = smoother.LocalSolvers(A, P, "mean", rho=rho)
    Se = smoother.LocalSolvers(A, P, "exact")
    q = (2 * k - 1) ** dim
    for j in range(len(P)):
        Bm, Be = _solver_matrix(Sm, j, q), _solver_matrix(Se, j, q)
        assert np.abs(Bm - Be).max() <= 1e-12 * np.abs(Be).max()


@pytest.mark.parametrize("dim,k,n", [(2, 2, 4), (3, 2, 3)])
def test_mean_solver_spectrum_within_coefficient_bounds(dim, k, n):
    """x^T A_j(rho) x / x^T A_b x lies in [min rho_c, max rho_c] over the patch's cells (A_j is a
    rho-weighted sum of the same nonnegative cell energies), so with B_j = (rhobar A_b)^{-1} the
    eigenvalues of B_j A_j lie in [rho_min / rhobar, rho_max / rhobar].  rhobar is far from 1 here, so
    multiplying instead of dividing by it lands outside the interval."""
    rho = _rho_field(dim, n, 21, scale=6.0)
    A = assemble.assemble(dim, k, n, rho)
    P = smoother.Patches(dim, k, n)
    S = smoother.LocalSolvers(A, P, "mean", rho=rho)
    q = (2 * k - 1) ** dim
    for j in range(len(P)):
        I = P.interior[j]
        r = rho[P.cells(j)]
        ev = np.linalg.eigvals(_solver_matrix(S, j, q) @ A[I][:, I].toarray()).real
        assert ev.min() >= r.min() / r.mean() * (1 - 1e-10)
        assert ev.max() <= r.max() / r.mean() * (1 + 1e-10)
        assert ev.max() - ev.min() > 1e-3  # a genuinely variable patch


def test_mean_solver_exact_on_patches_with_one_coefficient():
    """rho = alpha except in one cell: patches that do not touch that cell see a constant coefficient,
    and 'mean' is their exact local solver; the patches around the odd cell are not."""
    dim, k, n = 3, 2, 4
    rho = np.full(n ** dim, 2.5)
    odd = mesh.flat_index((0, 0, 0), n)
    rho[odd] = 40.0
    A = assemble.assemble(dim, k, n, rho)
    P = smoother.Patches(dim, k, n)
    S = smoother.LocalSolvers(A, P, "mean", rho=rho)
    q = (2 * k - 1) ** dim
    touched = 0
    for j in range(len(P)):
        I = P.interior[j]
        BA = _solver_matrix(S, j, q) @ A[I][:, I].toarray()
        dev = np.abs(BA - np.eye(q)).max()
        if odd in P.cells(j):
            touched += 1
            assert dev > 1e-2
        else:
            assert dev <= 1e-12
    assert touched == 1


# ---- local solver 'learned' --------------------------------------------------------

def test_learned_solver_with_unit_scaling_equals_mean():
    """c = 1: eq:fdm:inverse built for rhobar (eigen-decomposition) equals the Cholesky solve with
    rhobar A_b; c = alpha: alpha times it."""
    dim, k, n = 3, 2, 3
    rho = _rho_field(dim, n, 22, scale=4.0)
    A = assemble.assemble(dim, k, n, rho)
    P = smoother.Patches(dim, k, n)
    q = (2 * k - 1) ** dim
    Sm = smoother.LocalSolvers(A, P, "mean", rho=rho)
    for alpha in (1.0, 0.3):
        Sl = smoother.LocalSolvers(A, P, "learned", rho=rho, scaling=np.full((len(P), q), alpha))
        for j in range(len(P)):
            Bm, Bl = _solver_matrix(Sm, j, q), _solver_matrix(Sl, j, q)
            assert np.abs(Bl - alpha * Bm).max() <= 1e-12 * np.abs(Bm).max()


def test_learned_solver_scales_each_eigenmode():
    """Constant rho = alpha: with 1D generalized eigenpairs K t_a = lam_a M t_a of the patch interior
    (computed here), B_j A_j maps t_a (x) t_b (x) t_c (x fastest) to c_m times itself, where
    m = a + q b + q^2 c.  A per-mode factor that depends on the x index and the z index differently
    catches a permuted mode order."""
    dim, k, n = 3, 2, 3
    q1 = 2 * k - 1
    q = q1 ** dim
    alpha = 1.9
    rho = np.full(n ** dim, alpha)
    A = assemble.assemble(dim, k, n, rho)
    P = smoother.Patches(dim, k, n)
    fx = np.array([0.5, 1.5, 3.0])
    fz = np.array([1.0, 0.7, 1.3])
    c = np.array([fx[a] * fz[cc] for cc in range(q1) for b in range(q1) for a in range(q1)])
    S = smoother.LocalSolvers(A, P, "learned", rho=rho, scaling=np.tile(c, (len(P), 1)))
    Mj, Kj = smoother.patch_1d_matrices(k, 1.0 / n)
    lam, T = sla.eigh(Kj, Mj)
    j = len(P) // 2
    I = P.interior[j]
    Aj = A[I][:, I].toarray()
    B = _solver_matrix(S, j, q)
    for cc in range(q1):
        for b in range(q1):
            for a in range(q1):
                v = np.kron(T[:, cc], np.kron(T[:, b], T[:, a]))
                m = a + q1 * b + q1 * q1 * cc
                assert np.allclose(B @ (Aj @ v), c[m] * v, rtol=0, atol=1e-11 * np.abs(v).max())


# ---- MLP features ---------------------------------------------------------------------

def test_features_constant_rho_is_zero_and_scale_invariant():
    assert np.array_equal(learned.features(np.full(8, 3.3)), np.zeros(8))
    r = np.exp(np.random.default_rng(23).standard_normal((5, 8)))
    x = learned.features(r)
    assert np.allclose(learned.features(17.0 * r), x, rtol=0, atol=1e-14)


def test_features_are_logs_of_ratios_to_the_arithmetic_mean():
    """exp(x_c) = rho_c / rhobar, so exp(x) averages to exactly 1 (the arithmetic mean, not the geometric
    one: for which sum x_c = 0 would hold instead), and x is monotone in rho."""
    r = np.exp(1.5 * np.random.default_rng(24).standard_normal((6, 8)))
    x = learned.features(r)
    assert np.allclose(np.exp(x).mean(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.all(np.abs(x.sum(axis=1)) > 1e-3)
    for row_r, row_x in zip(r, x):
        assert np.array_equal(np.argsort(row_r), np.argsort(row_x))
    two = learned.features(np.array([1.0, 3.0]))
    assert np.allclose(two, [np.log(0.5), np.log(1.5)], rtol=0, atol=1e-15)
