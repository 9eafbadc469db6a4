"""1D Q_k Lagrange element on the unit interval (oracle, FP64).

The FE space is the interpolatory continuous Q_k space of Section 2 (nodal
degrees of freedom, shared at cell vertices).  The paper does not fix the node
placement; its implementation uses deal.II's FE_Q, whose default support points
are the Gauss-Lobatto-Legendre (GLL) points, so these are used here.  The
bilinear form of the Poisson problem (Appendix A.2) reduces on a Cartesian
cell to tensor products of the 1D mass and stiffness matrices computed below
(Appendix A.3, first displayed equation).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k: int) -> np.ndarray:
    """The k+1 GLL points mapped to [0, 1]: the end points and the roots of P_k'."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    if k == 1:
        return np.array([0.0, 1.0])
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    inner = npleg.legroots(npleg.legder(coef))
    inner = np.sort(np.real(inner))
    # one Newton polish step per root on P_k'(x) = 0
    d1 = npleg.legder(coef)
    d2 = npleg.legder(coef, 2)
    for _ in range(3):
        inner = inner - npleg.legval(inner, d1) / npleg.legval(inner, d2)
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gauss_rule(n: int):
    """n-point Gauss-Legendre rule on [0, 1] (exact for degree 2n-1)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """V[a, i] = l_a(x_i) for the Lagrange basis on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.ones((n, x.size))
    for a in range(n):
        for b in range(n):
            if b != a:
                out[a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
    return out


def lagrange_derivatives(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """D[a, i] = l_a'(x_i), by the product rule written out term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    out = np.zeros((n, x.size))
    for a in range(n):
        for c in range(n):
            if c == a:
                continue
            term = np.full(x.size, 1.0 / (nodes[a] - nodes[c]))
            for b in range(n):
                if b != a and b != c:
                    term *= (x - nodes[b]) / (nodes[a] - nodes[b])
            out[a] += term
    return out


def reference_matrices(k: int):
    """Reference 1D mass and stiffness matrices on [0, 1].

    M_ab = int_0^1 l_a l_b,  K_ab = int_0^1 l_a' l_b', by (k+2)-point Gauss
    (exact: the integrands have degree <= 2k).  On a cell of size h the cell
    matrices are h*M and K/h.
    """
    nodes = gll_nodes(k)
    xq, wq = gauss_rule(k + 2)
    V = lagrange_values(nodes, xq)
    D = lagrange_derivatives(nodes, xq)
    M = (V * wq) @ V.T
    K = (D * wq) @ D.T
    return M, K


def assembled_1d(k: int, n_cells: int, h: float | None = None):
    """Globally assembled 1D mass and stiffness matrices (dense, all nodes).

    Used for the Kronecker form of the constant-coefficient operator and for the
    patch matrices (a patch is two cells in every direction).
    """
    if h is None:
        h = 1.0 / n_cells
    Mr, Kr = reference_matrices(k)
    n1 = k * n_cells + 1
    M = np.zeros((n1, n1))
    K = np.zeros((n1, n1))
    for c in range(n_cells):
        sl = slice(c * k, c * k + k + 1)
        M[sl, sl] += h * Mr
        K[sl, sl] += Kr / h
    return M, K
