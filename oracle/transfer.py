"""Grid transfer between levels (Section 2, the two transfer operators).

Prolongation is the embedding V_l -> V_{l+1}: a fine node takes the value of
the coarse finite element function at its position, i.e. the coarse basis
functions evaluated at the fine nodes.  Restriction is its Euclidean adjoint,
the transpose.  Both act on free nodes only (Dirichlet entries are zero on
every level).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fe import gll_nodes, lagrange_values
from .mesh import node_coords_1d, free_mask_flat


def prolongation_1d(k: int, n_coarse: int) -> np.ndarray:
    """P1[i_fine, i_coarse] = l_{i_coarse}(x_fine) on the coarse cell holding x_fine.

    Entries are set, never summed: a fine node on a coarse cell boundary takes
    its value from one cell (the coarse vertex basis function is 1 there and all
    others vanish, so either cell gives the same row).
    """
    xf = node_coords_1d(k, 2 * n_coarse)
    xi = gll_nodes(k)
    hc = 1.0 / n_coarse
    P = np.zeros((xf.size, k * n_coarse + 1))
    for i, x in enumerate(xf):
        c = min(int(np.floor(x / hc + 1e-12)), n_coarse - 1)
        loc = (x - c * hc) / hc
        vals = lagrange_values(xi, np.array([loc]))[:, 0]
        for a in range(k + 1):
            P[i, c * k + a] = vals[a]
    return P


def prolongation(dim: int, k: int, n_coarse: int) -> sp.csr_matrix:
    """Prolongation from the level with n_coarse cells to the one with 2*n_coarse.

    Tensor product of the 1D evaluation matrices (coarse Q_k basis functions
    are products of 1D Lagrange polynomials), restricted to free nodes.
    """
    P1 = sp.csr_matrix(prolongation_1d(k, n_coarse))
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    Df = sp.diags(free_mask_flat(dim, k, 2 * n_coarse).astype(np.float64))
    Dc = sp.diags(free_mask_flat(dim, k, n_coarse).astype(np.float64))
    out = (Df @ P @ Dc).tocsr()
    out.eliminate_zeros()
    return out


def _along(mat, X, e, dim):
    """Apply a 1D matrix along direction e of a nodal array (e = 0 is x, the last numpy axis)."""
    ax = dim - 1 - e
    Xm = np.moveaxis(X, ax, 0)
    sh = Xm.shape
    Y = (mat @ Xm.reshape(sh[0], -1)).reshape((mat.shape[0],) + sh[1:])
    return np.moveaxis(Y, 0, ax)


def restrict_kron(dim: int, k: int, n_coarse: int, r_fine: np.ndarray) -> np.ndarray:
    """P^T r_fine without forming P: the transpose of the 1D prolongation along each axis.

    Same result as ``prolongation(dim, k, n_coarse).T @ r_fine`` (the tensor
    product of the 1D transposes, with the Dirichlet entries of both levels
    masked), for grids too large for the sparse Kronecker product.
    """
    P1t = sp.csr_matrix(prolongation_1d(k, n_coarse).T)
    nf = k * 2 * n_coarse + 1
    free_f = free_mask_flat(dim, k, 2 * n_coarse)
    X = np.where(free_f, np.asarray(r_fine, dtype=np.float64), 0.0).reshape((nf,) * dim)
    for e in range(dim):
        X = _along(P1t, X, e, dim)
    out = X.reshape(-1)
    out[~free_mask_flat(dim, k, n_coarse)] = 0.0
    return out


def prolong_kron(dim: int, k: int, n_coarse: int, e_coarse: np.ndarray) -> np.ndarray:
    """P e_coarse without forming P: the 1D prolongation along each axis, Dirichlet entries masked."""
    P1 = sp.csr_matrix(prolongation_1d(k, n_coarse))
    nc = k * n_coarse + 1
    X = np.where(free_mask_flat(dim, k, n_coarse), np.asarray(e_coarse, dtype=np.float64), 0.0).reshape((nc,) * dim)
    for e in range(dim):
        X = _along(P1, X, e, dim)
    out = X.reshape(-1)
    out[~free_mask_flat(dim, k, 2 * n_coarse)] = 0.0
    return out
