"""Learned per-eigenmode scaling of the patch inverse: data, training, use.

Variable coefficient -div(rho grad u) = f with rho per cell.  The plain
approximate local solver is the fast-diagonalization inverse built for the
patch mean rhobar (Appendix A.3; approximate local solvers are allowed, see
the remark after eq:main:2).  The learned form scales each eigenmode by a
factor c_m predicted from the patch's cell coefficients by a small MLP
(8 -> 64 -> 64 -> 27, tanh, FP32), trained to reproduce log(c*_m) where c*
is the energy-optimal diagonal computed exactly from the dense patch
operator.

Every arithmetic step runs in libvps kernels (targets, features, forward,
loss gradient, backward, Adam, inference); this module moves data between
them with torch tensors as device buffers.  Training data: patches of
training fields rho = exp(GRF) (seeds 1000+i) on several levels of their
coarsening hierarchy.
"""
from __future__ import annotations

import time

import numpy as np

from . import vps

N_HIDDEN = 64


def init_params(seed: int, nin: int = 8, nout: int = 27) -> np.ndarray:
    """Xavier-uniform weights, zero biases, in the flat layout of include/vps.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in [(N_HIDDEN, nin), (N_HIDDEN,), (N_HIDDEN, N_HIDDEN), (N_HIDDEN,), (nout, N_HIDDEN), (nout,)]:
        if len(shape) == 2:
            a = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-a, a, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def level_counts(total: int):
    """Samples per level (finest first) following the level mix of the hierarchy."""
    return [int(0.75 * total), int(0.20 * total), total - int(0.75 * total) - int(0.20 * total)]


def training_set(seeds, n_cells: int = 64, levels: int = 5, total: int = 200_000, sample_seed: int = 7,
                 corr_len: float = 1.0 / 8.0):
    """(X features FP32, T log-targets FP32, C targets FP64, rho8 FP64) on the GPU.

    Per field: all patches of every level are read with vps_patch_rho8; the
    finest level contributes 75%, the next 20% and the coarser ones 5% of the
    samples (drawn without replacement, seeded).
    """
    import torch
    import vps_inputs as vi
    per_field = [c // len(seeds) for c in level_counts(total)]
    rng = np.random.default_rng(sample_seed)
    chunks = []
    for s in seeds:
        rho = torch.from_numpy(vi.rho_cells(n_cells, s, corr_len=corr_len)).to("cuda")
        with vps.Context(3, 2, n_cells, levels, coef="learned") as ctx:
            ctx.set_coefficient(rho)
            groups = [[levels - 1], [levels - 2], list(range(1, levels - 2))]
            for want, lv in zip(per_field, groups):
                pool = []
                for l in lv:
                    npch = ctx.level_patches(l)
                    r8 = torch.empty((npch, 8), dtype=torch.float64, device="cuda")
                    ctx.patch_rho8(l, r8)
                    pool.append(r8)
                pool = torch.cat(pool)
                k = min(want, pool.shape[0])
                idx = torch.from_numpy(rng.choice(pool.shape[0], size=k, replace=False)).to("cuda")
                chunks.append(pool.index_select(0, idx))
    rho8 = torch.cat(chunks).contiguous()
    perm = torch.from_numpy(rng.permutation(rho8.shape[0])).to("cuda")
    rho8 = rho8.index_select(0, perm).contiguous()
    n = rho8.shape[0]
    X = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    T = torch.empty((n, 27), dtype=torch.float32, device="cuda")
    C = torch.empty((n, 27), dtype=torch.float64, device="cuda")
    with vps.Context(3, 2, 4, 1, coef="learned") as ctx:
        ctx.rho8_features(rho8, X)
        ctx.patch_targets(rho8, C, T)
        ctx.sync()
    return X, T, C, rho8


def train(X, T, epochs: int = 40, batch: int = 1024, lr: float = 1e-3, seed: int = 0, val_frac: float = 0.1,
          params0=None, log=None):
    """Adam on mean squared error of log-scaling; returns (params FP32 tensor, history)."""
    import torch
    n = X.shape[0]
    nval = int(val_frac * n)
    Xv, Tv = X[:nval], T[:nval]
    Xt, Tt = X[nval:], T[nval:]
    nt = Xt.shape[0]
    p = torch.from_numpy(init_params(seed) if params0 is None else np.asarray(params0, np.float32)).to("cuda")
    g = torch.zeros_like(p)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    y = torch.empty((batch, 27), dtype=torch.float32, device="cuda")
    act = torch.empty((batch, 2 * N_HIDDEN), dtype=torch.float32, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    yv = torch.empty((max(nval, 1), 27), dtype=torch.float32, device="cuda")
    dyv = torch.empty_like(yv)
    hist = []
    step = 0
    t0 = time.perf_counter()
    with vps.Context(3, 2, 4, 1, coef="learned") as ctx:
        for ep in range(epochs):
            for s0 in range(0, nt, batch):
                s1 = min(nt, s0 + batch)
                nb = s1 - s0
                xb, tb = Xt[s0:s1], Tt[s0:s1]
                ctx.mlp_forward(p, xb, y[:nb], act[:nb])
                ctx.mlp_loss_grad(y[:nb], tb, dy[:nb])
                ctx.mlp_backward(p, xb, act[:nb], dy[:nb], g)
                step += 1
                ctx.mlp_adam(p, g, m, v, step, lr)
            if nval:
                ctx.mlp_forward(p, Xv, yv[:nval])
                ctx.mlp_loss_grad(yv[:nval], Tv, dyv[:nval], loss)
                ctx.sync()
                hist.append(float(loss.item()))
                if log:
                    log(f"epoch {ep + 1}: validation loss {hist[-1]:.5f}")
    torch.cuda.synchronize()
    return p, {"val_loss": hist, "steps": step, "seconds": time.perf_counter() - t0, "train_samples": nt,
               "val_samples": nval}


def baseline_loss(T):
    """Validation-style loss of the plain solver (log c = 0 for every mode)."""
    return float((T.double() ** 2).mean().item())


def apply_scaling(ctx, params):
    """Infer the scaling of every smoothed level of ctx; returns the fallback counts per level."""
    return [ctx.mlp_infer_patches(l, params) for l in range(1, ctx.n_levels)]


def convergence_factor(hist, first: int = 3, last: int = 12):
    """Geometric-mean residual reduction per stationary V-cycle over iterations first..last."""
    last = min(last, len(hist) - 1)
    if hist[first - 1] == 0.0:
        return 0.0
    return (hist[last] / hist[first - 1]) ** (1.0 / (last - first + 1))


def apply_exact_targets(ctx):
    """Set every smoothed level's scaling to the exact training targets clamp(c*, 1/4, 4) of its patches
    (what a perfect network would output); returns the non-finite counts per level (set to 1)."""
    import torch
    bad = []
    for l in range(1, ctx.n_levels):
        n = ctx.level_patches(l)
        r8 = torch.empty((n, 8), dtype=torch.float64, device="cuda")
        ctx.patch_rho8(l, r8)
        C = torch.empty((n, 27), dtype=torch.float64, device="cuda")
        T = torch.empty((n, 27), dtype=torch.float32, device="cuda")
        ctx.patch_targets(r8, C, T)
        c = torch.exp(T)
        ok = torch.isfinite(c)
        bad.append(int((~ok).sum().item()))
        c = torch.where(ok, c, torch.ones_like(c)).contiguous()
        ctx.set_patch_scaling(l, c)
    ctx.sync()
    return bad


def compare(params, n_cells: int = 64, levels: int = 5, rho_seed: int = 4, rhs_seed: int = 4, rtol: float = 1e-10,
            maxit: int = 300, corr_len: float = 1.0 / 8.0, iters: int = 12, exact: bool = True):
    """Plain rhobar-FDM vs learned scaling on one field: convergence factor and time to rtol.  With
    exact=True also the exact targets the network is trained on ('exact': a perfect network) and the exact
    dense local solvers A_j(rho)^{-1} ('exact_solver': the ceiling of any per-patch correction)."""
    import torch
    import vps_inputs as vi
    rho = torch.from_numpy(vi.rho_cells(n_cells, rho_seed, corr_len=corr_len)).to("cuda")
    b = torch.from_numpy(vi.seeded_vector(3, 2, n_cells, rhs_seed)).to("cuda")
    out = {}
    coefs = {"mean": "mean", "learned": "learned", "exact": "learned", "exact_solver": "exact"}
    for mode in ("mean", "learned") + (("exact", "exact_solver") if exact else ()):
        with vps.Context(3, 2, n_cells, levels, coef=coefs[mode]) as ctx:
            ctx.set_coefficient(rho)
            if mode == "learned":
                fb = apply_scaling(ctx, params)
            elif mode == "exact":
                fb = apply_exact_targets(ctx)
            else:
                fb = None
            u = torch.zeros_like(b)
            hist = ctx.vcycle_iterate(b, u, iters)
            x = torch.empty_like(b)
            ctx.solve(b, x, rtol=rtol, maxit=maxit, check=False)  # warm-up
            info = ctx.solve(b, x, rtol=rtol, maxit=maxit, check=False)
            out[mode] = {"factor": convergence_factor(hist), "residual_history": hist,
                         "iterations": info["iterations"], "seconds": info["seconds"],
                         "rel_residual_true": info["rel_residual_true"], "status": info["status"],
                         "fallback_per_level": fb}
    return out


def save_params(path: str, params) -> None:
    np.save(path, params.detach().cpu().numpy() if hasattr(params, "detach") else np.asarray(params))


def load_params(path: str, device: str = "cuda"):
    """Parameters written by save_params (a plain .npy array; nothing in the file is executed)."""
    import torch
    return torch.from_numpy(np.load(path, allow_pickle=False).astype(np.float32)).to(device)
