"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module holds no arithmetic of the smoother, the operator or the multigrid
method.  It only knows the storage layout of a nodal vector and draws seeded
random numbers:

* a level with ``n_cells`` cells per direction and Q_k elements stores the full
  nodal grid of ``(k*n_cells+1)**dim`` values, x fastest (numpy shape
  ``(n1,)*dim`` with the last axis being x);
* Dirichlet nodes (any index 0 or ``n1-1``) hold 0;
* right-hand sides and initial guesses are i.i.d. uniform on [-1, 1] on the
  free nodes, drawn in lexicographic order from ``numpy.random.default_rng``;
* the variable coefficient is ``rho = exp(g)`` per cell, ``g`` a Gaussian
  random field (Gaussian covariance, circulant embedding on a 2x padded torus).

The workloads below are the five problem shapes the project is measured on.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "nodes_1d",
    "grid_shape",
    "free_mask",
    "seeded_vector",
    "grf_cells",
    "rho_cells",
    "WORKLOADS",
]


def nodes_1d(degree: int, n_cells: int) -> int:
    """Nodes per direction of a Q_k grid with ``n_cells`` cells per direction."""
    return degree * n_cells + 1


def grid_shape(dim: int, degree: int, n_cells: int) -> tuple:
    return (nodes_1d(degree, n_cells),) * dim


def free_mask(dim: int, degree: int, n_cells: int) -> np.ndarray:
    """Boolean grid: True on nodes that are not on the boundary of [0,1]^dim."""
    n1 = nodes_1d(degree, n_cells)
    m1 = np.zeros(n1, dtype=bool)
    m1[1:-1] = True
    m = m1
    for _ in range(dim - 1):
        m = np.logical_and.outer(m1, m)
    return m


def seeded_vector(dim: int, degree: int, n_cells: int, seed: int,
                  dtype=np.float64) -> np.ndarray:
    """Flat nodal vector: U[-1,1] i.i.d. on free nodes (lexicographic draw), 0 on Dirichlet."""
    mask = free_mask(dim, degree, n_cells).reshape(-1)
    rng = np.random.default_rng(seed)
    out = np.zeros(mask.size, dtype=np.float64)
    out[mask] = rng.uniform(-1.0, 1.0, size=int(mask.sum()))
    return out.astype(dtype, copy=False)


def grf_cells(n_cells: int, seed: int, corr_len: float = 1.0 / 8.0,
              std: float = 1.0, dim: int = 3) -> np.ndarray:
    """Gaussian random field sampled at cell centres of a uniform mesh on [0,1]^dim.

    Covariance std^2 * exp(-|r|^2 / (2 corr_len^2)).  Sampled exactly (up to the
    clipping of round-off-sized negative eigenvalues) by circulant embedding on a
    periodic grid of 2*n_cells points per direction (period 2), then the first
    n_cells^dim block is kept.  No renormalisation.  Returns shape (n,)*dim with
    the last axis being x.
    """
    n = int(n_cells)
    m = 2 * n
    h = 1.0 / n
    idx = np.arange(m)
    dist1 = np.minimum(idx, m - idx) * h
    r2 = np.zeros((m,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = m
        r2 = r2 + (dist1 ** 2).reshape(shape)
    cov = std * std * np.exp(-r2 / (2.0 * corr_len * corr_len))
    lam = np.real(np.fft.fftn(cov))
    lam = np.where(lam > 0.0, lam, 0.0)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((m,) * dim) + 1j * rng.standard_normal((m,) * dim)
    field = np.real(np.fft.ifftn(np.sqrt(lam) * z)) * np.sqrt(float(m ** dim))
    return np.ascontiguousarray(field[(slice(0, n),) * dim])


def rho_cells(n_cells: int, seed: int, corr_len: float = 1.0 / 8.0,
              std: float = 1.0, dim: int = 3) -> np.ndarray:
    """Per-cell coefficient rho = exp(g), g from :func:`grf_cells`; flat, x fastest."""
    return np.exp(grf_cells(n_cells, seed, corr_len, std, dim)).reshape(-1)


# The five measured problem shapes.  ``levels`` counts the multigrid levels
# (coarsest level has 4 cells per direction), ``pre``/``post`` the smoothing
# sweeps of the V-cycle, ``vcycle`` the arithmetic of the preconditioner.
WORKLOADS = {
    "poisson2d_q2_n32": dict(dim=2, degree=2, n_cells=32, levels=4, pre=1, post=1,
                             vcycle="f64", coef="const", rhs_seed=1, u0_seed=101),
    "poisson3d_q4_n32": dict(dim=3, degree=4, n_cells=32, levels=4, pre=1, post=1,
                             vcycle="f64", coef="const", rhs_seed=2, u0_seed=102),
    "poisson3d_q3_n64": dict(dim=3, degree=3, n_cells=64, levels=5, pre=1, post=1,
                             vcycle="f32", coef="const", rhs_seed=3, u0_seed=103),
    "varcoef3d_q2_n64": dict(dim=3, degree=2, n_cells=64, levels=5, pre=1, post=1,
                             vcycle="f64", coef="learned", rhs_seed=4, u0_seed=104,
                             rho_seed=4, train_seed_base=1000, train_patches=200_000),
    # batched color sweeps: each workgroup a batch of same-color patches (a row of 7 x-adjacent
    # patches on the large levels), and on the finest level all colors of a slab of 44 vertex layers
    # in turn (Algorithm 5, the same iterate; 3 slabs); whole colors are timed beside it.  The FP64
    # reference sweeps whole colors (measured faster there)
    "poisson3d_q4_n128": dict(dim=3, degree=4, n_cells=128, levels=6, pre=2, post=2,
                              vcycle="f32", coef="const", rhs_seed=5, u0_seed=105,
                              batch_layers=44, batch_layers_f64=0),
    # the paper's own shapes (Poisson, a single 2^d-cell patch refined 10 times in 2D and 6 times
    # in 3D; multigrid down to that patch), FP64 as in the paper
    "paper2d_q3_n2048": dict(dim=2, degree=3, n_cells=2048, levels=11, pre=1, post=1,
                             vcycle="f64", coef="const", rhs_seed=11, u0_seed=111),
    "paper2d_q5_n2048": dict(dim=2, degree=5, n_cells=2048, levels=11, pre=1, post=1,
                             vcycle="f64", coef="const", rhs_seed=12, u0_seed=112),
    "paper3d_q5_n128": dict(dim=3, degree=5, n_cells=128, levels=7, pre=1, post=1,
                            vcycle="f64", coef="const", rhs_seed=13, u0_seed=113),
}
