"""Pins of the oracle's patch smoother against definitions that do not use it."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import vps_inputs as vi
from oracle import assemble, smoother, mesh


def _setup(dim, k, N, mode="exact", rho=None):
    A = assemble.assemble(dim, k, N, rho)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, mode, rho=rho)
    return A, P, S


@pytest.mark.parametrize("dim,k,N", [(2, 1, 4), (2, 2, 4), (2, 4, 4), (3, 2, 4), (3, 3, 3), (2, 5, 3), (3, 5, 2)])
def test_patch_block_is_kronecker_sum(dim, k, N):
    """A[I_j, I_j] equals the Kronecker sum of the 1D patch matrices (Appendix A.3) for every patch."""
    A = assemble.assemble(dim, k, N)
    P = smoother.Patches(dim, k, N)
    Ab = smoother.patch_matrix_const(dim, k, 1.0 / N)
    for I in P.interior:
        assert np.abs(A[I][:, I].toarray() - Ab).max() < 1e-13 * np.abs(Ab).max()


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2), (3, 4), (2, 5), (3, 5)])
def test_fdm_inverse_equals_dense_solve(dim, k):
    h = 1.0 / 16
    S, Lam, T, lam = smoother.fdm_factors(dim, k, h)
    Ab = smoother.patch_matrix_const(dim, k, h)
    r = np.random.default_rng(0).standard_normal(Ab.shape[0])
    d_fdm = S @ ((S.T @ r) / Lam)
    d_lu = sla.lu_solve(sla.lu_factor(Ab), r)
    assert np.linalg.norm(d_fdm - d_lu) <= 1e-13 * np.linalg.norm(d_lu)
    Mj, Kj = smoother.patch_1d_matrices(k, h)
    assert np.allclose(T.T @ Mj @ T, np.eye(T.shape[0]), atol=1e-12)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (3, 2), (2, 5), (3, 5)])
def test_single_patch_sweep_is_exact_solve(dim, k):
    """N = 2: the only patch covers all free nodes, so one sweep solves A u = b."""
    A, P, S = _setup(dim, k, 2)
    assert len(P) == 1
    b = vi.seeded_vector(dim, k, 2, 1)
    u0 = vi.seeded_vector(dim, k, 2, 2)
    u = smoother.sweep_colorized(A, b, u0, P, S)
    free = mesh.free_mask_flat(dim, k, 2)
    x = np.zeros_like(b)
    x[free] = np.linalg.solve(A.toarray()[np.ix_(free, free)], b[free])
    assert np.abs(u - x).max() < 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("dim,N", [(2, 6), (3, 4)])
def test_k1_is_multicolor_gauss_seidel(dim, N):
    """k = 1: one DoF per patch, so a sweep is point Gauss-Seidel in color order."""
    A, P, S = _setup(dim, 1, N)
    b = vi.seeded_vector(dim, 1, N, 3)
    u0 = vi.seeded_vector(dim, 1, N, 4)
    u = smoother.sweep_colorized(A, b, u0, P, S)
    order = np.concatenate([np.concatenate([P.interior[j] for j in P.by_color[c]]) for c in range(2 ** dim)])
    Ap = A[order][:, order].tocsr()
    L = sp.tril(Ap, format="csr")
    r = (b - A @ u0)[order]
    d = spla.spsolve_triangular(L, r, lower=True)
    want = u0.copy()
    want[order] += d
    assert np.abs(u - want).max() < 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("dim,k,N,reverse", [(2, 2, 4, False), (2, 3, 5, True), (3, 2, 4, False), (3, 1, 5, True)])
def test_alg1_alg2_alg3_agree(dim, k, N, reverse):
    """The three implementations of the same smoother agree in the same patch order (Section 3.3)."""
    A, P, S = _setup(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 5)
    u0 = vi.seeded_vector(dim, k, N, 6)
    u1 = smoother.sweep_product(A, b, u0, P, S, reverse)
    u2 = smoother.sweep_local_residual(b, u0, P, reverse=reverse)
    u3 = smoother.sweep_colorized(A, b, u0, P, S, reverse)
    sc = np.abs(u3).max()
    assert np.abs(u1 - u3).max() <= 1e-13 * sc
    assert np.abs(u2 - u3).max() <= 1e-13 * sc


def test_alg2_variable_coefficient_matches_alg3():
    dim, k, N = 2, 2, 4
    rho = np.exp(np.random.default_rng(1).standard_normal(N ** dim))
    A, P, S = _setup(dim, k, N, rho=rho)
    b = vi.seeded_vector(dim, k, N, 5)
    u0 = vi.seeded_vector(dim, k, N, 6)
    u2 = smoother.sweep_local_residual(b, u0, P, rho=rho)
    u3 = smoother.sweep_colorized(A, b, u0, P, S)
    assert np.abs(u2 - u3).max() <= 1e-13 * np.abs(u3).max()


@pytest.mark.parametrize("dim,k,N", [(2, 3, 6), (3, 2, 4)])
def test_residual_vanishes_on_updated_interiors(dim, k, N):
    A, P, S = _setup(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 7)
    u = vi.seeded_vector(dim, k, N, 8)
    for c in range(2 ** dim):
        u = smoother.apply_color(A, b, u, P, S, c)
        r = b - A @ u
        for j in P.by_color[c]:
            assert np.abs(r[P.interior[j]]).max() < 1e-12 * np.abs(b).max()


def test_energy_error_non_increasing_per_patch():
    """Each exact patch step is an A-orthogonal projection of the error."""
    dim, k, N = 2, 2, 5
    A, P, S = _setup(dim, k, N)
    free = mesh.free_mask_flat(dim, k, N)
    b = vi.seeded_vector(dim, k, N, 9)
    xs = np.zeros_like(b)
    xs[free] = np.linalg.solve(A.toarray()[np.ix_(free, free)], b[free])
    u = vi.seeded_vector(dim, k, N, 10)
    err = lambda v: float((xs - v) @ (A @ (xs - v)))
    prev = err(u)
    for c in range(4):
        for j in P.by_color[c]:
            r = b - A @ u
            I = P.interior[j]
            u[I] += S.apply(j, r[I])
            e = err(u)
            assert e <= prev * (1 + 1e-12)
            prev = e


@pytest.mark.parametrize("dim,k,N", [(2, 2, 6), (3, 3, 4)])
def test_color_sets_do_not_interact(dim, k, N):
    """Same-color patches: disjoint interiors, and no interior node of one in the closure of another."""
    P = smoother.Patches(dim, k, N)
    for c in range(2 ** dim):
        js = P.by_color[c]
        seen = set()
        for j in js:
            Ij = set(P.interior[j].tolist())
            assert not (Ij & seen)
            seen |= Ij
        for a in js:
            clo = set(mesh.patch_closure(dim, k, N, P.verts[a]).tolist())
            for bb in js:
                if bb != a:
                    assert not (clo & set(P.interior[bb].tolist()))


def test_mean_solver_spectrum_bounds():
    """Plain rhobar-FDM: the eigenvalues of B_j A_j lie in [rho_min/rhobar, rho_max/rhobar]."""
    from oracle import learned
    rng = np.random.default_rng(2)
    for _ in range(5):
        rho8 = np.exp(1.5 * rng.standard_normal(8))
        Aj = learned.patch_operator(3, 2, 1.0, rho8)
        Ab = smoother.patch_matrix_const(3, 2, 1.0)
        ev = sla.eigvals(np.linalg.solve(rho8.mean() * Ab, Aj)).real
        assert ev.min() >= rho8.min() / rho8.mean() * (1 - 1e-12)
        assert ev.max() <= rho8.max() / rho8.mean() * (1 + 1e-12)


@pytest.mark.parametrize("dim,k,N,B", [(2, 2, 7, 2), (3, 2, 5, 1), (3, 1, 6, 3)])
@pytest.mark.parametrize("reverse", [False, True])
def test_batched_sweep_equals_patch_by_patch(dim, k, N, B, reverse):
    """Algorithm 5 in the grouped form equals the residual recomputed before every patch in the same order."""
    A = assemble.assemble(dim, k, N)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, "exact")
    b = vi.seeded_vector(dim, k, N, 81)
    u0 = vi.seeded_vector(dim, k, N, 82)
    want = np.array(u0)
    for group in smoother.batched_order(P, B, reverse):
        for j in group:
            r = b - A @ want
            I = P.interior[j]
            want[I] += S.apply(j, r[I])
    got = smoother.sweep_batched(A, b, u0, P, S, B, reverse)
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # every patch exactly once
    seen = sorted(j for g in smoother.batched_order(P, B) for j in g)
    assert seen == list(range(len(P)))


@pytest.mark.parametrize("dim,k,N", [(2, 2, 6), (3, 2, 4)])
def test_batched_sweep_one_batch_is_colorized(dim, k, N):
    """A batch holding every layer is the plain colorized sweep (Algorithm 3/4 order)."""
    A = assemble.assemble(dim, k, N)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, "exact")
    b = vi.seeded_vector(dim, k, N, 83)
    u0 = vi.seeded_vector(dim, k, N, 84)
    for rev in (False, True):
        assert np.allclose(smoother.sweep_batched(A, b, u0, P, S, N, rev), smoother.sweep_colorized(A, b, u0, P, S, rev),
                           rtol=0, atol=1e-13)


@pytest.mark.parametrize("B,same", [(2, True), (4, True), (1, False), (3, False)])
def test_batched_sweep_even_layers_keep_the_colorized_iterate(B, same):
    """Two patches interact only if their vertices differ by at most 1 in every direction.  With batches of
    an even number of vertex layers, a batch boundary has an even layer below an odd one, so every
    interacting pair is visited in the colorized order (colors with even slowest-direction parity first):
    the iterate is exactly the colorized one.  Odd batch sizes reverse some pairs: a different iterate,
    each step still an A-orthogonal projection (the energy error decreases)."""
    dim, k, N = 3, 2, 6
    A = assemble.assemble(dim, k, N)
    P = smoother.Patches(dim, k, N)
    S = smoother.LocalSolvers(A, P, "exact")
    b = vi.seeded_vector(dim, k, N, 85)
    u0 = vi.seeded_vector(dim, k, N, 86)
    free = np.flatnonzero(A.diagonal() != 0)
    us = np.zeros_like(b)
    us[free] = spla.spsolve(A[free][:, free].tocsc(), b[free])
    energy = lambda v: float((us - v) @ (A @ (us - v)))
    ub = smoother.sweep_batched(A, b, u0, P, S, B)
    uc = smoother.sweep_colorized(A, b, u0, P, S)
    if same:
        assert np.array_equal(ub, uc)
    else:
        assert np.abs(ub - uc).max() > 1e-6
    assert energy(ub) < energy(u0)
