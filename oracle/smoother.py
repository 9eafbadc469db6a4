"""Multiplicative vertex-patch smoother (oracle, explicit dense local solves).

Definitions followed (Sections 2.1 and 3):

* local solver (eq:main:2): P_j v = Pi_j^T B_j Pi_j A v with B_j = A_j^{-1}
  (exact) or an approximation of it (the text after eq:main:2 allows that);
* smoother (eq:s-ell): the product over patches of (I - P_j), applied to the
  error, i.e. u <- u + Pi_j^T B_j Pi_j (b - A u) patch after patch;
* colored form (eq:colorized): within one color the patches have disjoint
  interiors and do not read each other's writes, so one factor per color,
  u <- u + (sum_{j in C_k} Pi_j^T B_j Pi_j)(b - A u), gives the same iterate.

``sweep_colorized`` (eq:colorized, one factor per color) is the oracle of a
sweep; ``sweep_product`` (eq:s-ell, one factor per patch) and
``sweep_local_residual`` (eq:s-ell with the residual formed from the patch's
own cells, Section 3.1) exist for the order-equivalence pins on tiny meshes;
``sweep_batched`` takes the factors of eq:colorized over the (batch, color)
sets of Section 4.1.  Patch order: colors ascending for a forward sweep,
descending for a reverse sweep; inside a color the order is irrelevant.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assemble import element_matrix, kron_list
from .fe import assembled_1d
from .mesh import (patch_vertices, vertex_color, patch_interior, patch_closure,
                   patch_cells, cell_flat, colors_in_order)


class Patches:
    """All vertex patches of one level with their colors and index sets."""

    def __init__(self, dim: int, k: int, n_cells: int):
        self.dim, self.k, self.n_cells = dim, k, n_cells
        self.verts = patch_vertices(dim, n_cells)
        self.colors = [vertex_color(v) for v in self.verts]
        self.interior = [patch_interior(dim, k, n_cells, v) for v in self.verts]
        self.by_color = {c: [] for c in range(2 ** dim)}
        for j, c in enumerate(self.colors):
            self.by_color[c].append(j)

    def __len__(self):
        return len(self.verts)

    def cells(self, j):
        return [cell_flat(self.dim, self.n_cells, c) for c in patch_cells(self.dim, self.verts[j])]


def patch_1d_matrices(k: int, h: float):
    """Interior blocks M_j, K_j (q x q, q = 2k-1) of the 2-cell 1D patch matrices."""
    M, K = assembled_1d(k, 2, h)
    return M[1:-1, 1:-1], K[1:-1, 1:-1]


def fdm_factors(dim: int, k: int, h: float):
    """S = T (x) ... (x) T and Lambda of the fast diagonalization (Appendix A.3).

    T solves the generalized eigenproblem K_j T = M_j T diag(lam) with
    T^T M_j T = I (SciPy's symmetric-definite solver), so that
    A_b = S^{-T} diag(Lambda) S^{-1} and A_b^{-1} = S diag(1/Lambda) S^T,
    Lambda_m = sum_e lam_{m_e}  (m lexicographic, x fastest).
    """
    Mj, Kj = patch_1d_matrices(k, h)
    lam, T = sla.eigh(Kj, Mj)
    S = kron_list([T] * dim)
    q = lam.size
    L = np.zeros((q,) * dim)
    for e in range(dim):
        shape = [1] * dim
        shape[dim - 1 - e] = q
        L = L + lam.reshape(shape)
    return S, L.reshape(-1), T, lam


def patch_matrix_const(dim: int, k: int, h: float) -> np.ndarray:
    """A_b = sum_e (x)(K_j at e, M_j elsewhere): constant-coefficient patch matrix."""
    Mj, Kj = patch_1d_matrices(k, h)
    A = np.zeros(((2 * k - 1) ** dim,) * 2)
    for e in range(dim):
        A += kron_list([Kj if ep == e else Mj for ep in range(dim)])
    return A


def patch_closure_operator(dim: int, k: int, h: float, rho_cells=None) -> np.ndarray:
    """Local operator on the patch closure, sum over its 2^d cells of rho_c * E.

    Rows and columns are the (2k+1)^d closure nodes, x fastest; the cells are
    in lexicographic order (x fastest), matching ``Patches.cells``.
    """
    p = 2 * k + 1
    E = element_matrix(dim, k, h)
    m = (k + 1) ** dim
    Abar = np.zeros((p ** dim, p ** dim))
    ncell = 2 ** dim
    rho = np.ones(ncell) if rho_cells is None else np.asarray(rho_cells, dtype=np.float64)
    for ci in range(ncell):
        off = [(ci >> e) & 1 for e in range(dim)]
        loc = np.zeros(m, dtype=np.int64)
        for li in range(m):
            rem = li
            g = 0
            stride = 1
            for e in range(dim):
                le = rem % (k + 1)
                rem //= (k + 1)
                g += (k * off[e] + le) * stride
                stride *= p
            loc[li] = g
        Abar[np.ix_(loc, loc)] += rho[ci] * E
    return Abar


def closure_interior_positions(dim: int, k: int) -> np.ndarray:
    """Positions of the interior nodes inside the closure numbering."""
    p = 2 * k + 1
    out = []
    for flat in range(p ** dim):
        rem = flat
        ok = True
        for _ in range(dim):
            a = rem % p
            rem //= p
            if a == 0 or a == p - 1:
                ok = False
        if ok:
            out.append(flat)
    return np.array(out, dtype=np.int64)


class LocalSolvers:
    """The local solvers B_j of one level.

    mode 'exact'   : B_j = (A[I_j, I_j])^{-1}, one dense Cholesky per patch
    mode 'shared'  : constant coefficient; all A[I_j, I_j] are equal (checked on
                     a sample) and one factor is used
    mode 'mean'    : B_j = (rhobar_j * A_b)^{-1}, A_b the rho=1 patch matrix
    mode 'learned' : B_j = S diag(c_j / (rhobar_j Lambda)) S^T, c_j per patch
    """

    def __init__(self, A, patches: Patches, mode: str = "exact", rho=None,
                 scaling=None, check_samples: int = 20):
        self.mode = mode
        self.patches = patches
        dim, k, n = patches.dim, patches.k, patches.n_cells
        h = 1.0 / n
        self.factors = None
        if mode == "exact":
            self.factors = []
            for I in patches.interior:
                Aj = A[I][:, I].toarray()
                self.factors.append(sla.cho_factor(Aj))
        elif mode == "shared":
            Ab = patch_matrix_const(dim, k, h)
            step = max(1, len(patches) // max(1, check_samples))
            for j in range(0, len(patches), step):
                I = patches.interior[j]
                Aj = A[I][:, I].toarray()
                if not np.allclose(Aj, Ab, rtol=1e-13, atol=1e-13 * np.abs(Ab).max()):
                    raise ValueError("patch matrices differ; use mode='exact'")
            self.shared = sla.cho_factor(Ab)
        elif mode in ("mean", "learned"):
            rho = np.asarray(rho, dtype=np.float64).reshape(-1)
            self.rhobar = np.array([rho[patches.cells(j)].mean() for j in range(len(patches))])
            if mode == "mean":
                self.shared = sla.cho_factor(patch_matrix_const(dim, k, h))
            else:
                self.S, self.Lam, _, _ = fdm_factors(dim, k, h)
                self.scaling = np.asarray(scaling, dtype=np.float64).reshape(len(patches), -1)
        else:
            raise ValueError(mode)

    def apply(self, j: int, r: np.ndarray) -> np.ndarray:
        if self.mode == "exact":
            return sla.cho_solve(self.factors[j], r)
        if self.mode == "shared":
            return sla.cho_solve(self.shared, r)
        if self.mode == "mean":
            return sla.cho_solve(self.shared, r) / self.rhobar[j]
        s = self.scaling[j] / (self.rhobar[j] * self.Lam)
        return self.S @ (s * (self.S.T @ r))


def group_factor(A, b, u, patches: Patches, solvers: LocalSolvers, group) -> np.ndarray:
    """One factor of the colorized product (eq:colorized) for the index set ``group``.

    Returns u + (sum_{j in group} Pi_j^T B_j Pi_j)(b - A u): the residual of
    the current iterate, restricted to each patch interior (Pi_j), mapped by
    the local solver B_j (eq:main:2, with b - A u in place of A v) and
    embedded back (Pi_j^T).  For a single patch this is the factor I - P_j of
    eq:s-ell applied to the error.
    """
    r = b - A @ u
    d = np.zeros_like(r)
    for j in group:
        I = patches.interior[j]
        d[I] += solvers.apply(j, r[I])
    return np.asarray(u, dtype=np.float64) + d


def apply_color(A, b, u, patches: Patches, solvers: LocalSolvers, color: int) -> np.ndarray:
    """The factor of eq:colorized for one color C_k (its patches have disjoint interiors)."""
    return group_factor(A, b, u, patches, solvers, patches.by_color[color])


def patch_sequence(patches: Patches, reverse: bool = False):
    """Patch order of one sweep: colors ascending (descending if reverse), inside a color by index."""
    return [j for c in colors_in_order(patches.dim, reverse) for j in patches.by_color[c]]


def sweep_product(A, b, u, patches: Patches, solvers: LocalSolvers, reverse: bool = False) -> np.ndarray:
    """eq:s-ell: one factor (I - P_j) per patch, the residual recomputed before each (Algorithm 1 computes
    this; tiny meshes only)."""
    for j in patch_sequence(patches, reverse):
        u = group_factor(A, b, u, patches, solvers, [j])
    return u


def sweep_colorized(A, b, u, patches: Patches, solvers: LocalSolvers, reverse: bool = False) -> np.ndarray:
    """eq:colorized: one factor per color, colors ascending (descending if reverse).  Equal to eq:s-ell in
    the same patch order because same-color patches do not read each other's writes (Algorithms 3 and 4
    compute this)."""
    for c in colors_in_order(patches.dim, reverse):
        u = apply_color(A, b, u, patches, solvers, c)
    return np.array(u, dtype=np.float64, copy=True)


def batch_of(patches: Patches, j: int, batch_layers: int) -> int:
    """Batch of patch j: its vertex coordinate in the slowest direction, in slabs of batch_layers layers."""
    return (patches.verts[j][patches.dim - 1] - 1) // batch_layers


def batched_order(patches: Patches, batch_layers: int, reverse: bool = False):
    """Index sets of batch processing (Section 4.1): each color cut into batches of whole patch layers along
    the slowest direction (lexicographic order kept), the batches outermost, the colors inside.  The
    reverse sweep takes the sets backwards."""
    nb = (patches.n_cells - 2) // batch_layers + 1
    groups = []
    for bi in range(nb):
        for c in colors_in_order(patches.dim):
            groups.append([j for j in patches.by_color[c] if batch_of(patches, j, batch_layers) == bi])
    return groups[::-1] if reverse else groups


def sweep_batched(A, b, u, patches: Patches, solvers: LocalSolvers, batch_layers: int,
                  reverse: bool = False) -> np.ndarray:
    """eq:colorized with the (batch, color) index sets of Section 4.1 as the factors (Algorithm 5 computes
    this)."""
    u = np.array(u, dtype=np.float64, copy=True)
    for group in batched_order(patches, batch_layers, reverse):
        if group:
            u = group_factor(A, b, u, patches, solvers, group)
    return u


def sweep_local_residual(b, u, patches: Patches, rho=None, reverse: bool = False) -> np.ndarray:
    """eq:s-ell with the residual of each patch formed locally (Section 3.1): gather the closure (eq:gather),
    r_j = b_j - Abar_j ubar_j from the patch's own cells restricted to the interior rows (eq:main:4),
    d_j = A_j^{-1} r_j with A_j the interior block of the same local operator, scatter (eq:scatter).
    No global matrix is used (Algorithm 2 computes this)."""
    dim, k, n = patches.dim, patches.k, patches.n_cells
    h = 1.0 / n
    u = np.array(u, dtype=np.float64, copy=True)
    inner = closure_interior_positions(dim, k)
    rho_flat = None if rho is None else np.asarray(rho, dtype=np.float64).reshape(-1)
    const_op = None
    for j in patch_sequence(patches, reverse):
        v = patches.verts[j]
        if rho_flat is None:
            if const_op is None:
                const_op = patch_closure_operator(dim, k, h)
            Abar = const_op
        else:
            Abar = patch_closure_operator(dim, k, h, rho_flat[patches.cells(j)])
        clo = patch_closure(dim, k, n, v)
        I = patch_interior(dim, k, n, v)
        r = b[I] - Abar[inner] @ u[clo]
        u[I] += np.linalg.solve(Abar[np.ix_(inner, inner)], r)
    return u
