"""Uniform Cartesian levels, vertex patches and their colors (oracle).

Nodal vectors store the full grid of (k*N+1)^d values, x fastest, with the
Dirichlet nodes held at 0 (see ``vps_inputs``).  A vertex patch (Section 2.1,
item 1) is the union of the 2^d cells around an interior vertex v in
[1, N-1]^d.  Its subspace V_j (Section 2.1, item 2, with homogeneous
Dirichlet conditions on the patch boundary) has the (2k-1)^d nodes strictly
inside the patch; the extended space of Section 3.1 adds the patch boundary,
giving (2k+1)^d closure nodes.  Patches of one color must have disjoint
interiors and must not read what another writes (Section 3.2, equation
eq:colorized and the disjointness condition after it); with 2 cells per
patch and direction the vertex parity c(v) = sum_e (v_e mod 2) 2^e gives 2^d
such colors.
"""
from __future__ import annotations

import itertools

import numpy as np

from .fe import gll_nodes


def n1d(k: int, n_cells: int) -> int:
    return k * n_cells + 1


def node_coords_1d(k: int, n_cells: int) -> np.ndarray:
    """Positions of the k*N+1 nodes of one direction on [0, 1]."""
    xi = gll_nodes(k)
    x = np.empty(k * n_cells + 1)
    for c in range(n_cells):
        x[c * k: c * k + k + 1] = (c + xi) / n_cells
    x[-1] = 1.0
    return x


def flat_index(idx, n1: int) -> int:
    """Flat index of a multi-index ordered (x, y, z, ...), x fastest."""
    out = 0
    stride = 1
    for i in idx:
        out += i * stride
        stride *= n1
    return out


def free_mask_flat(dim: int, k: int, n_cells: int) -> np.ndarray:
    n1 = n1d(k, n_cells)
    axes = [np.arange(n1)] * dim
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # (z, y, x) order
    m = np.ones((n1,) * dim, dtype=bool)
    for g in grids:
        m &= (g > 0) & (g < n1 - 1)
    return m.reshape(-1)


def vertex_color(v) -> int:
    """Color of the patch of interior vertex v = (v_x, v_y, ...)."""
    return sum((int(ve) % 2) << e for e, ve in enumerate(v))


def patch_vertices(dim: int, n_cells: int):
    """All interior vertices, lexicographic with x fastest."""
    rng = range(1, n_cells)
    out = []
    for rev in itertools.product(rng, repeat=dim):
        out.append(tuple(reversed(rev)))
    return out


def box_indices(dim: int, n1: int, lo, hi) -> np.ndarray:
    """Flat indices of the node box prod_e [lo_e, hi_e] (inclusive), x fastest."""
    ranges = [np.arange(lo[e], hi[e] + 1) for e in range(dim)]
    idx = np.zeros(1, dtype=np.int64)
    stride = 1
    for e in range(dim):
        idx = (idx[None, :] + ranges[e][:, None] * stride).reshape(-1)
        stride *= n1
    return idx


def patch_interior(dim: int, k: int, n_cells: int, v) -> np.ndarray:
    """Global indices I_j of the patch interior, lexicographic x fastest."""
    n1 = n1d(k, n_cells)
    lo = [k * (ve - 1) + 1 for ve in v]
    hi = [k * (ve + 1) - 1 for ve in v]
    return box_indices(dim, n1, lo, hi)


def patch_closure(dim: int, k: int, n_cells: int, v) -> np.ndarray:
    """Global indices of the closure (extended patch space of Section 3.1)."""
    n1 = n1d(k, n_cells)
    lo = [k * (ve - 1) for ve in v]
    hi = [k * (ve + 1) for ve in v]
    return box_indices(dim, n1, lo, hi)


def patch_cells(dim: int, v):
    """The 2^d cells of the patch of vertex v, lexicographic (x fastest)."""
    out = []
    for rev in itertools.product((0, 1), repeat=dim):
        off = tuple(reversed(rev))
        out.append(tuple(v[e] - 1 + off[e] for e in range(dim)))
    return out


def cell_flat(dim: int, n_cells: int, c) -> int:
    return flat_index(c, n_cells)


def colors_in_order(dim: int, reverse: bool = False):
    cols = list(range(2 ** dim))
    return cols[::-1] if reverse else cols


def coarsen_cells(rho: np.ndarray, dim: int, n_cells: int) -> np.ndarray:
    """Coefficient of the next coarser level: mean of the 2^d children of each cell."""
    f = rho.reshape((n_cells,) * dim)
    nc = n_cells // 2
    acc = np.zeros((nc,) * dim)
    for off in itertools.product((0, 1), repeat=dim):
        sl = tuple(slice(o, None, 2) for o in off)
        acc += f[sl]
    return (acc / 2 ** dim).reshape(-1)
