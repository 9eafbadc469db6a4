"""Global operators A_l of the discrete problem A u = b (Section 2, eq:matrix).

``assemble`` is the plain definition: cell-by-cell summation of element
matrices of a(u, v) = int rho grad u . grad v into a sparse matrix over all
nodes, followed by elimination of the Dirichlet rows and columns (Appendix
A.2: homogeneous Dirichlet data on the boundary of the unit hypercube).  On an
axis-aligned cell of size h the element matrix of the Laplacian is the
Kronecker sum of Appendix A.3, sum_e (x)_{e'} (K if e'==e else M), with the 1D
cell matrices M = h*Mref, K = Kref/h.

``assemble_kron`` and ``matvec_kron`` are a second, independent route for the
constant-coefficient case (the global matrix is a Kronecker sum of assembled
1D matrices); they serve large meshes where cell-by-cell assembly is too
costly and are pinned against ``assemble`` on small meshes.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .fe import reference_matrices, assembled_1d
from .mesh import n1d, free_mask_flat


def kron_list(mats):
    """kron(mats[-1], ..., mats[0]): the factor mats[0] acts on x (fastest index)."""
    out = mats[-1]
    for m in reversed(mats[:-1]):
        out = np.kron(out, m)
    return out


def element_matrix(dim: int, k: int, h: float) -> np.ndarray:
    """Laplace element matrix on a cell of size h, local nodes x fastest."""
    Mr, Kr = reference_matrices(k)
    M = h * Mr
    K = Kr / h
    E = np.zeros(((k + 1) ** dim,) * 2)
    for e in range(dim):
        E += kron_list([K if ep == e else M for ep in range(dim)])
    return E


def cell_node_indices(dim: int, k: int, n_cells: int) -> np.ndarray:
    """idx[cell, local] = global node of local node ``local`` of ``cell``.

    Cells and local nodes are both lexicographic with x fastest.
    """
    n1 = n1d(k, n_cells)
    cells = np.arange(n_cells ** dim)
    cidx = []
    rem = cells.copy()
    for _ in range(dim):
        cidx.append(rem % n_cells)
        rem //= n_cells
    loc = np.arange((k + 1) ** dim)
    lidx = []
    rem = loc.copy()
    for _ in range(dim):
        lidx.append(rem % (k + 1))
        rem //= (k + 1)
    out = np.zeros((cells.size, loc.size), dtype=np.int64)
    stride = 1
    for e in range(dim):
        out += (k * cidx[e][:, None] + lidx[e][None, :]) * stride
        stride *= n1
    return out


def dirichlet_eliminate(A: sp.spmatrix, free: np.ndarray) -> sp.csr_matrix:
    D = sp.diags(free.astype(np.float64))
    out = (D @ A @ D).tocsr()
    out.eliminate_zeros()
    out.sort_indices()
    return out


def assemble(dim: int, k: int, n_cells: int, rho: np.ndarray | None = None) -> sp.csr_matrix:
    """A with entries a(phi_j, phi_i), Dirichlet rows/columns removed (zeroed).

    rho: per-cell coefficient (flat, x fastest) or None for rho = 1.
    """
    h = 1.0 / n_cells
    E = element_matrix(dim, k, h)
    idx = cell_node_indices(dim, k, n_cells)
    ncell, m = idx.shape
    w = np.ones(ncell) if rho is None else np.asarray(rho, dtype=np.float64).reshape(-1)
    rows = np.broadcast_to(idx[:, :, None], (ncell, m, m)).reshape(-1)
    cols = np.broadcast_to(idx[:, None, :], (ncell, m, m)).reshape(-1)
    vals = (w[:, None, None] * E[None, :, :]).reshape(-1)
    n = n1d(k, n_cells) ** dim
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    return dirichlet_eliminate(A, free_mask_flat(dim, k, n_cells))


def assemble_kron(dim: int, k: int, n_cells: int) -> sp.csr_matrix:
    """Constant-coefficient A as sum_e kron(... K1 at position e ... M1 ...)."""
    M1, K1 = assembled_1d(k, n_cells)
    M1 = sp.csr_matrix(M1)
    K1 = sp.csr_matrix(K1)
    A = None
    for e in range(dim):
        mats = [K1 if ep == e else M1 for ep in range(dim)]
        term = mats[-1]
        for mm in reversed(mats[:-1]):
            term = sp.kron(term, mm, format="csr")
        A = term if A is None else A + term
    return dirichlet_eliminate(A, free_mask_flat(dim, k, n_cells))


def matvec_kron(dim: int, k: int, n_cells: int, u: np.ndarray) -> np.ndarray:
    """A u for constant coefficient without forming A (1D factors along each axis).

    u is a full nodal vector (Dirichlet entries must be 0); the result has its
    Dirichlet entries set to 0.  Memory: a few copies of u.
    """
    M1, K1 = assembled_1d(k, n_cells)
    M1 = sp.csr_matrix(M1)
    K1 = sp.csr_matrix(K1)
    n1 = n1d(k, n_cells)
    U = np.asarray(u, dtype=np.float64).reshape((n1,) * dim)

    def along(mat, X, e):
        # apply mat along direction e (e=0 is x = last numpy axis)
        ax = dim - 1 - e
        Xm = np.moveaxis(X, ax, 0)
        sh = Xm.shape
        Y = (mat @ Xm.reshape(n1, -1)).reshape(sh)
        return np.moveaxis(Y, 0, ax)

    out = np.zeros_like(U)
    for e in range(dim):
        T = U
        for ep in range(dim):
            T = along(K1 if ep == e else M1, T, ep)
        out += T
    out = out.reshape(-1)
    out[~free_mask_flat(dim, k, n_cells)] = 0.0
    return out


def matvec_cells(dim: int, k: int, n_cells: int, rho: np.ndarray | None, u: np.ndarray) -> np.ndarray:
    """A(rho) u without storing A: the cell-by-cell sum of ``assemble`` applied to u.

    Each cell contributes rho_c E (u restricted to its nodes) to its nodes
    (the same element matrix and node numbering as ``assemble``); the
    Dirichlet entries of the result are set to 0 and those of u must be 0.
    """
    h = 1.0 / n_cells
    E = element_matrix(dim, k, h)
    idx = cell_node_indices(dim, k, n_cells)
    w = np.ones(idx.shape[0]) if rho is None else np.asarray(rho, dtype=np.float64).reshape(-1)
    u = np.asarray(u, dtype=np.float64)
    contrib = (u[idx] @ E.T) * w[:, None]
    n = n1d(k, n_cells) ** dim
    out = np.bincount(idx.reshape(-1), weights=contrib.reshape(-1), minlength=n)
    out[~free_mask_flat(dim, k, n_cells)] = 0.0
    return out


def all_cells(dim: int, n_cells: int):
    for rev in itertools.product(range(n_cells), repeat=dim):
        yield tuple(reversed(rev))
