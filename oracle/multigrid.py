"""Geometric multigrid V-cycle and the outer Krylov solvers (oracle, FP64).

V-cycle (Section 2, the standard finite element V-cycle with smoother S_l and
transfers): on level l > 0, pre-smooth from a zero initial guess with forward
sweeps, restrict the residual, recurse, add the prolongated correction,
post-smooth with reverse sweeps (colors in descending order, which makes
V(nu, nu) symmetric); on level 0 solve exactly (dense Cholesky).  The
operators are rediscretised on every level (eq:matrix on each mesh); for a
variable coefficient the coarse coefficient is the mean of the 2^d children.

The outer solvers are preconditioned CG (x0 = 0) and, for an inexact
preconditioner, flexible CG with the Polak-Ribiere-type beta.  Stopping test:
||b - A x||_2 <= rtol ||b||_2 over the free nodes, with the true residual
recomputed once the recursive one passes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assemble import assemble, assemble_kron
from .mesh import free_mask_flat, coarsen_cells
from .smoother import Patches, LocalSolvers, sweep_colorized
from .transfer import prolongation


class Level:
    def __init__(self, dim, k, n_cells, rho=None, mode="exact", scaling=None, use_kron=False):
        self.dim, self.k, self.n_cells = dim, k, n_cells
        self.rho = rho
        if rho is None and use_kron:
            self.A = assemble_kron(dim, k, n_cells)
        else:
            self.A = assemble(dim, k, n_cells, rho)
        self.free = free_mask_flat(dim, k, n_cells)
        self.patches = Patches(dim, k, n_cells) if n_cells >= 2 else None
        self.mode = mode
        self.scaling = scaling
        self._solvers = None

    @property
    def solvers(self):
        if self._solvers is None:
            self._solvers = LocalSolvers(self.A, self.patches, self.mode,
                                         rho=self.rho, scaling=self.scaling)
        return self._solvers

    def smooth(self, b, u, sweeps, reverse):
        for _ in range(sweeps):
            u = sweep_colorized(self.A, b, u, self.patches, self.solvers, reverse)
        return u


class Hierarchy:
    """Levels 0 (coarsest, n_cells / 2^(L-1) cells) ... L-1 (finest)."""

    def __init__(self, dim, k, n_cells, n_levels, pre=1, post=1, rho=None,
                 mode=None, scalings=None, use_kron=False):
        if n_cells % (2 ** (n_levels - 1)) != 0:
            raise ValueError("n_cells must be divisible by 2^(levels-1)")
        if mode is None:
            mode = "shared" if rho is None else "mean"
        self.dim, self.k, self.pre, self.post = dim, k, pre, post
        cells = [n_cells // 2 ** (n_levels - 1 - l) for l in range(n_levels)]
        rhos = [None] * n_levels
        if rho is not None:
            rhos[-1] = np.asarray(rho, dtype=np.float64).reshape(-1)
            for l in range(n_levels - 2, -1, -1):
                rhos[l] = coarsen_cells(rhos[l + 1], dim, cells[l + 1])
        self.levels = []
        for l in range(n_levels):
            sc = None if scalings is None else scalings[l]
            self.levels.append(Level(dim, k, cells[l], rhos[l], mode, sc, use_kron))
        self.P = [None] + [prolongation(dim, k, cells[l - 1]) for l in range(1, n_levels)]
        A0 = self.levels[0].A
        f0 = self.levels[0].free
        self.coarse_free = np.flatnonzero(f0)
        self.coarse_factor = sla.cho_factor(A0[self.coarse_free][:, self.coarse_free].toarray())

    @property
    def A(self):
        return self.levels[-1].A

    def coarse_solve(self, b):
        x = np.zeros_like(b)
        x[self.coarse_free] = sla.cho_solve(self.coarse_factor, b[self.coarse_free])
        return x

    def vcycle(self, b, l=None):
        if l is None:
            l = len(self.levels) - 1
        if l == 0:
            return self.coarse_solve(b)
        lev = self.levels[l]
        u = np.zeros_like(b)
        u = lev.smooth(b, u, self.pre, reverse=False)
        r = b - lev.A @ u
        rc = self.P[l].T @ r
        e = self.vcycle(rc, l - 1)
        u = u + self.P[l] @ e
        u = lev.smooth(b, u, self.post, reverse=True)
        return u


def pcg(H: Hierarchy, b, rtol=1e-10, maxit=200, flexible=False, precond=None):
    """Preconditioned CG from x0 = 0; returns (x, iterations, true relative residual).

    flexible=True uses beta = (z_new, r_new - r_old) / (z_old, r_old).
    """
    A = H.A
    V = H.vcycle if precond is None else precond
    b = np.asarray(b, dtype=np.float64)
    bn = np.linalg.norm(b)
    x = np.zeros_like(b)
    if bn == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = V(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        it += 1
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r_old = r
        r = r - alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            rt = b - A @ x
            if np.linalg.norm(rt) <= rtol * bn:
                return x, it, np.linalg.norm(rt) / bn
            r = rt
        z_new = V(r)
        if flexible:
            beta = (z_new @ (r - r_old)) / rz
        else:
            beta = (r @ z_new) / rz
        rz = r @ z_new
        p = z_new + beta * p
    rt = b - A @ x
    return x, it, np.linalg.norm(rt) / bn


def stationary_factor(H: Hierarchy, b, first=3, last=12):
    """Geometric-mean residual reduction of u <- u + V(b - A u) over iterations first..last."""
    A = H.A
    u = np.zeros_like(b)
    norms = [np.linalg.norm(b)]
    for _ in range(last):
        u = u + H.vcycle(b - A @ u)
        norms.append(np.linalg.norm(b - A @ u))
    return (norms[last] / norms[first - 1]) ** (1.0 / (last - first + 1)), norms
