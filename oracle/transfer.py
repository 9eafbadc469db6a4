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
