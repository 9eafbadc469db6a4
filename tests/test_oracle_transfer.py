"""Pins of the oracle's transfer operators."""
import numpy as np
import pytest

from oracle import assemble, transfer, mesh


@pytest.mark.parametrize("dim,k,Nc", [(2, 1, 2), (2, 2, 2), (2, 3, 3), (2, 4, 2), (3, 1, 2), (3, 2, 2), (3, 3, 1)])
def test_galerkin_identity(dim, k, Nc):
    """Nested conforming spaces: P^T A_fine P = A_coarse (constant coefficient)."""
    P = transfer.prolongation(dim, k, Nc)
    Af = assemble.assemble(dim, k, 2 * Nc)
    Ac = assemble.assemble(dim, k, Nc)
    assert abs(P.T @ Af @ P - Ac).max() < 1e-12 * abs(Ac).max()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_polynomial_reproduction_1d(k):
    """The 1D prolongation maps the coarse interpolant of any p in P_k to the fine one."""
    rng = np.random.default_rng(k)
    c = rng.standard_normal(k + 1)
    Nc = 3
    P1 = transfer.prolongation_1d(k, Nc)
    uc = np.polyval(c, mesh.node_coords_1d(k, Nc))
    uf = np.polyval(c, mesh.node_coords_1d(k, 2 * Nc))
    assert np.abs(P1 @ uc - uf).max() < 1e-12 * max(1.0, np.abs(uf).max())


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_polynomial_reproduction_masked(dim, k):
    """The masked d-dim prolongation reproduces prod_e x_e(1-x_e) q_e(x_e), deg q_e = k-2."""
    rng = np.random.default_rng(10 * dim + k)
    Nc = 2

    def interp(N, coefs):
        x = mesh.node_coords_1d(k, N)
        u = None
        for c in coefs:  # coefs[0] for x, coefs[1] for y, ...
            g = x * (1 - x) * np.polyval(c, x)
            u = g if u is None else np.multiply.outer(g, u)
        return u.reshape(-1)

    coefs = [rng.standard_normal(k - 1) for _ in range(dim)]
    P = transfer.prolongation(dim, k, Nc)
    assert np.abs(P @ interp(Nc, coefs) - interp(2 * Nc, coefs)).max() < 1e-12


def test_prolongation_rows_sum_to_one_inside():
    """Constants are reproduced: interior fine rows of the unmasked 1D operator sum to 1."""
    for k in (1, 2, 3, 4):
        P1 = transfer.prolongation_1d(k, 4)
        assert np.allclose(P1.sum(axis=1), 1.0, atol=1e-13)


@pytest.mark.parametrize("dim,k,Nc", [(2, 1, 3), (2, 4, 2), (3, 1, 3), (3, 2, 2), (3, 3, 2), (3, 4, 1)])
def test_restrict_kron_is_transpose_of_prolongation(dim, k, Nc):
    """The axis-by-axis restriction equals P^T with the sparse tensor-product P."""
    P = transfer.prolongation(dim, k, Nc)
    rf = np.random.default_rng(dim * 10 + k).standard_normal(P.shape[0])
    rf[~mesh.free_mask_flat(dim, k, 2 * Nc)] = 0.0
    assert np.allclose(transfer.restrict_kron(dim, k, Nc, rf), P.T @ rf, rtol=0, atol=1e-13 * abs(rf).max())


@pytest.mark.parametrize("dim,k,Nc", [(2, 2, 3), (3, 1, 3), (3, 4, 2)])
def test_restrict_kron_galerkin(dim, k, Nc):
    """P^T A_fine P e = A_coarse e, with the restriction and both operators applied axis by axis."""
    P = transfer.prolongation(dim, k, Nc)
    e = np.random.default_rng(3).standard_normal(P.shape[1])
    e[~mesh.free_mask_flat(dim, k, Nc)] = 0.0
    lhs = transfer.restrict_kron(dim, k, Nc, assemble.matvec_kron(dim, k, 2 * Nc, P @ e))
    rhs = assemble.matvec_kron(dim, k, Nc, e)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * abs(rhs).max())


@pytest.mark.parametrize("dim,k,Nc", [(2, 1, 3), (2, 4, 2), (3, 1, 3), (3, 2, 2), (3, 3, 2), (3, 4, 1)])
def test_prolong_kron_is_prolongation(dim, k, Nc):
    """The axis-by-axis prolongation equals the sparse tensor-product P."""
    P = transfer.prolongation(dim, k, Nc)
    ec = np.random.default_rng(dim * 10 + k + 1).standard_normal(P.shape[1])
    ec[~mesh.free_mask_flat(dim, k, Nc)] = 0.0
    assert np.allclose(transfer.prolong_kron(dim, k, Nc, ec), P @ ec, rtol=0, atol=1e-13 * abs(ec).max())


@pytest.mark.parametrize("k", [2, 3, 4])
def test_prolong_kron_reproduces_coarse_polynomials(k):
    """A Q_k polynomial vanishing on the boundary: its coarse interpolant is prolonged to its fine interpolant."""
    Nc = 2
    xc = mesh.node_coords_1d(k, Nc)
    xf = mesh.node_coords_1d(k, 2 * Nc)
    Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(xf, xf, xf, indexing="ij")
    g = lambda X, Y, Z: X * (1 - X) * Y * (1 - Y) * Z * (1 - Z) * X ** (k - 2)
    got = transfer.prolong_kron(3, k, Nc, g(Xc, Yc, Zc).reshape(-1))
    assert np.allclose(got, g(Xf, Yf, Zf).reshape(-1), rtol=0, atol=1e-13)
