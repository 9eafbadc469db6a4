"""Targets for the learned per-eigenmode scaling of the patch inverse (oracle).

Variable coefficient -div(rho grad u) = f with one rho per cell.  The local
operator A_j(rho) of a patch is the interior block of the sum of its 2^d
cells' element matrices (eq:main:2 with the restriction of A to V_j).  The
approximate local solver keeps the fast-diagonalization form of Appendix A.3
(eq:fdm:inverse) built for the patch mean rhobar and rescales each eigenmode:
B_j = S diag(c_m / (rhobar Lambda_m)) S^T (approximate local solvers are
allowed, see the remark after eq:main:2).

Target: the energy-optimal diagonal.  With Y = S^T A_j S, the choice
B_j = S diag(d) S^T that minimises ||I - A_j^{1/2} B_j A_j^{1/2}||_F^2
= sum_i (lambda_i(B_j A_j) - 1)^2 satisfies (Y o Y) d = diag(Y) (o: entrywise
product); the target is c*_m = rhobar Lambda_m d_m.  For constant rho,
Y = rho diag(Lambda) and c* = 1.  (The diagonal of S^{-1} A_j^{-1} S^{-T} was
also considered; it pushes lambda_max(B_j A_j) above 2 on high-contrast
patches and makes the multiplicative smoother diverge, so it is not used.)
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .smoother import patch_closure_operator, closure_interior_positions, fdm_factors


def patch_operator(dim: int, k: int, h: float, rho_cells) -> np.ndarray:
    """A_j(rho): interior block of the patch's local operator (cells lexicographic)."""
    Abar = patch_closure_operator(dim, k, h, rho_cells)
    inner = closure_interior_positions(dim, k)
    return Abar[np.ix_(inner, inner)]


def targets(dim: int, k: int, rho_cells, h: float = 1.0) -> np.ndarray:
    """c*_m for one patch (length (2k-1)^dim): energy-optimal per-mode scaling."""
    rho_cells = np.asarray(rho_cells, dtype=np.float64)
    S, Lam, _, _ = fdm_factors(dim, k, h)
    Aj = patch_operator(dim, k, h, rho_cells)
    Y = S.T @ Aj @ S
    d = sla.cho_solve(sla.cho_factor(Y * Y), np.diag(Y).copy())
    return rho_cells.mean() * Lam * d


def solver_matrix(dim: int, k: int, rho_cells, c, h: float = 1.0) -> np.ndarray:
    """B_j = S diag(c / (rhobar Lambda)) S^T as a dense matrix."""
    S, Lam, _, _ = fdm_factors(dim, k, h)
    return S @ np.diag(np.asarray(c) / (np.mean(rho_cells) * Lam)) @ S.T


def features(rho_cells) -> np.ndarray:
    """MLP input of a patch: log(rho_c / rhobar) for its 2^d cells."""
    rho_cells = np.asarray(rho_cells, dtype=np.float64)
    return np.log(rho_cells / rho_cells.mean(axis=-1, keepdims=True))


def scaling_from_output(y: np.ndarray, lo: float = 0.25, hi: float = 4.0) -> np.ndarray:
    """c = clamp(exp(y), lo, hi); non-finite rows fall back to c = 1."""
    c = np.clip(np.exp(y), lo, hi)
    bad = ~np.all(np.isfinite(y), axis=-1)
    c[bad] = 1.0
    return c
