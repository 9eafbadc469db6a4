"""Discretisation checks with a manufactured solution (oracle).

Problem of Appendix A.2 with the sign convention -Laplace(u) = f (the printed
equation drops the minus sign; with it the operator is SPD).  The exact
solution u = prod_e sin(pi x_e) vanishes on the boundary and has
f = dim * pi^2 * prod_e sin(pi x_e).  Load vector b_i = int f phi_i by
(k+2)-point Gauss per direction and cell; L2 error by (k+3)-point Gauss.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fe import gll_nodes, gauss_rule, lagrange_values
from .assemble import cell_node_indices
from .mesh import free_mask_flat, n1d


def _tensor_rule(dim, n):
    x, w = gauss_rule(n)
    pts = []
    wts = []
    for rev in itertools.product(range(n), repeat=dim):
        idx = tuple(reversed(rev))
        pts.append([x[i] for i in idx])
        wts.append(np.prod([w[i] for i in idx]))
    return np.array(pts), np.array(wts)


def _basis_at(dim, k, pts):
    """phi[local, q] for the tensor Lagrange basis (local x fastest) at reference points."""
    xi = gll_nodes(k)
    vals = [lagrange_values(xi, pts[:, e]) for e in range(dim)]
    m = (k + 1) ** dim
    out = np.ones((m, pts.shape[0]))
    for loc in range(m):
        rem = loc
        for e in range(dim):
            a = rem % (k + 1)
            rem //= (k + 1)
            out[loc] *= vals[e][a]
    return out


def _cell_origins(dim, n_cells):
    cells = np.arange(n_cells ** dim)
    org = np.zeros((cells.size, dim))
    rem = cells.copy()
    for e in range(dim):
        org[:, e] = (rem % n_cells) / n_cells
        rem //= n_cells
    return org


def exact_u(x):
    return np.prod(np.sin(np.pi * x), axis=-1)


def rhs_f(x):
    return x.shape[-1] * np.pi ** 2 * np.prod(np.sin(np.pi * x), axis=-1)


def load_vector(dim, k, n_cells, f=rhs_f):
    h = 1.0 / n_cells
    pts, wts = _tensor_rule(dim, k + 2)
    phi = _basis_at(dim, k, pts)
    org = _cell_origins(dim, n_cells)
    idx = cell_node_indices(dim, k, n_cells)
    b = np.zeros(n1d(k, n_cells) ** dim)
    for c in range(org.shape[0]):
        xq = org[c][None, :] + h * pts
        fq = f(xq) * wts * h ** dim
        np.add.at(b, idx[c], phi @ fq)
    b[~free_mask_flat(dim, k, n_cells)] = 0.0
    return b


def l2_error(dim, k, n_cells, U, u=exact_u):
    h = 1.0 / n_cells
    pts, wts = _tensor_rule(dim, k + 3)
    phi = _basis_at(dim, k, pts)
    org = _cell_origins(dim, n_cells)
    idx = cell_node_indices(dim, k, n_cells)
    err2 = 0.0
    for c in range(org.shape[0]):
        xq = org[c][None, :] + h * pts
        uh = U[idx[c]] @ phi
        err2 += np.sum(wts * h ** dim * (uh - u(xq)) ** 2)
    return np.sqrt(err2)
