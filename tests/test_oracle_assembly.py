"""Pins of the oracle's global operator (cell-by-cell assembly)."""
import os

import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

import vps_inputs as vi
from oracle import assemble, mesh


def test_q1_stencil_2d():
    """2D Q1 Laplacian: (1/3)(8 at the centre, -1 at the 8 neighbours), h-independent."""
    for N in (4, 8):
        A = assemble.assemble(2, 1, N).toarray()
        n1 = N + 1
        c = 2 * n1 + 2
        row = A[c].reshape(n1, n1)
        want = np.zeros((n1, n1))
        want[1:4, 1:4] = -1.0 / 3.0
        want[2, 2] = 8.0 / 3.0
        assert np.allclose(row, want, atol=1e-14)


def test_problem_size_formula_matches_paper_table():
    path = os.path.join(os.path.dirname(__file__), "golden", "problem_sizes.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        d, k, n, size = (int(s) for s in line.split())
        assert vi.nodes_1d(k, n) ** d == size


@pytest.mark.parametrize("dim,k,N", [(2, 1, 4), (2, 3, 4), (2, 4, 2), (3, 1, 3), (3, 2, 2), (3, 3, 2)])
def test_kron_equals_cell_assembly(dim, k, N):
    A = assemble.assemble(dim, k, N)
    B = assemble.assemble_kron(dim, k, N)
    assert abs(A - B).max() < 1e-13 * abs(A).max()
    u = vi.seeded_vector(dim, k, N, 7)
    assert np.allclose(assemble.matvec_kron(dim, k, N, u), A @ u, rtol=0, atol=1e-12 * abs(A).max())


def _poly_energy_1d_factors():
    # w(x) = x(1-x): int w^2 = 1/30, int w'^2 = 1/3
    w = np.array([0.0, 1.0, -1.0])
    return w


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_energy_of_bubble(dim, k):
    """u = prod x_e(1-x_e) lies in Q_k (k>=2); u^T A u = int |grad u|^2 = dim/3 * (1/30)^(dim-1)."""
    N = 3
    A = assemble.assemble(dim, k, N)
    x = mesh.node_coords_1d(k, N)
    w = x * (1 - x)
    u = w
    for _ in range(dim - 1):
        u = np.multiply.outer(w, u)
    u = u.reshape(-1)
    exact = dim / 3.0 * (1.0 / 30.0) ** (dim - 1)
    assert abs(u @ A @ u - exact) < 1e-13


def test_variable_coefficient_energy_cellwise():
    """u^T A(rho) u = sum_c rho_c int_c |grad u|^2, cell integrals by exact polynomial antiderivatives."""
    dim, k, N = 2, 2, 4
    rng = np.random.default_rng(3)
    rho = np.exp(rng.standard_normal(N * N))
    A = assemble.assemble(dim, k, N, rho)
    x = mesh.node_coords_1d(k, N)
    w = x * (1 - x)
    u = np.multiply.outer(w, w).reshape(-1)
    wc = np.array([0.0, 1.0, -1.0])
    dwc = npoly.polyder(wc)

    def integ(c, a, b):
        P = npoly.polyint(c)
        return npoly.polyval(b, P) - npoly.polyval(a, P)

    total = 0.0
    for cy in range(N):
        for cx in range(N):
            ax, bx = cx / N, (cx + 1) / N
            ay, by = cy / N, (cy + 1) / N
            gx = integ(npoly.polymul(dwc, dwc), ax, bx) * integ(npoly.polymul(wc, wc), ay, by)
            gy = integ(npoly.polymul(wc, wc), ax, bx) * integ(npoly.polymul(dwc, dwc), ay, by)
            total += rho[cy * N + cx] * (gx + gy)
    assert abs(u @ A @ u - total) < 1e-13 * total


def test_dirichlet_rows_zero_and_symmetric():
    A = assemble.assemble(3, 2, 3)
    free = mesh.free_mask_flat(3, 2, 3)
    Ad = A.toarray()
    assert np.all(Ad[~free] == 0) and np.all(Ad[:, ~free] == 0)
    assert np.allclose(Ad, Ad.T, atol=1e-15)
    ev = np.linalg.eigvalsh(Ad[np.ix_(free, free)])
    assert ev.min() > 0


@pytest.mark.parametrize("dim,k,N", [(2, 2, 6), (2, 3, 5), (3, 1, 5), (3, 2, 4), (3, 4, 3)])
def test_matvec_cells_equals_assembled(dim, k, N):
    """The unassembled variable-coefficient product equals the assembled CSR matrix times u."""
    rng = np.random.default_rng(dim * 100 + k * 10 + N)
    rho = np.exp(rng.standard_normal(N ** dim))
    u = rng.standard_normal((k * N + 1) ** dim)
    u[~mesh.free_mask_flat(dim, k, N)] = 0.0
    A = assemble.assemble(dim, k, N, rho)
    assert np.allclose(assemble.matvec_cells(dim, k, N, rho, u), A @ u, rtol=0, atol=1e-12 * abs(A @ u).max())
