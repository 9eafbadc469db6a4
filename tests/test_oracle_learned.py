"""Pins of the learned-scaling oracle: targets, MLP gradients, Adam."""
import numpy as np
import pytest

from oracle import learned, mlp


def test_constant_rho_gives_unit_targets():
    for k in (1, 2, 3):
        c = learned.targets(3, k, np.full(8, 2.5))
        assert np.abs(c - 1.0).max() < 1e-12
    assert np.abs(learned.targets(2, 2, np.full(4, 0.3)) - 1.0).max() < 1e-12


def test_targets_scale_invariant_and_h_invariant():
    rng = np.random.default_rng(1)
    r = np.exp(rng.standard_normal(8))
    c = learned.targets(3, 2, r)
    assert np.abs(learned.targets(3, 2, 7.0 * r) - c).max() < 1e-12
    assert np.abs(learned.targets(3, 2, r, h=1.0 / 64) - c).max() < 1e-10


def _objective(r, c):
    """sum_i (lambda_i(B_j A_j) - 1)^2 computed from eigenvalues (not from the normal equations)."""
    import scipy.linalg as sla
    B = learned.solver_matrix(3, 2, r, c)
    Aj = learned.patch_operator(3, 2, 1.0, r)
    ev = sla.eigvals(B @ Aj).real
    return float(np.sum((ev - 1.0) ** 2))


def test_targets_minimise_energy_objective():
    """Perturbing c* in any mode or random direction does not decrease the objective."""
    rng = np.random.default_rng(2)
    for _ in range(3):
        r = np.exp(1.2 * rng.standard_normal(8))
        c = learned.targets(3, 2, r)
        f0 = _objective(r, c)
        for m in range(0, 27, 5):
            for s in (1e-3, -1e-3):
                cp = c.copy(); cp[m] *= 1 + s
                assert _objective(r, cp) >= f0 - 1e-12
        for _ in range(4):
            cp = c * (1 + 1e-3 * rng.standard_normal(27))
            assert _objective(r, cp) >= f0 - 1e-12


def test_targets_improve_high_contrast_patches():
    """rhobar-FDM has lambda_max(B A) = rho_max/rhobar; the clamped c* lowers it, below 2 for contrast <= 3."""
    import scipy.linalg as sla
    rng = np.random.default_rng(5)
    hit = 0
    for _ in range(30):
        r = np.exp(1.5 * rng.standard_normal(8))
        ratio = r.max() / r.mean()
        if ratio <= 2.2:
            continue
        hit += 1
        Aj = learned.patch_operator(3, 2, 1.0, r)
        plain = sla.eigvals(learned.solver_matrix(3, 2, r, np.ones(27)) @ Aj).real
        c = np.clip(learned.targets(3, 2, r), 0.25, 4.0)
        opt = sla.eigvals(learned.solver_matrix(3, 2, r, c) @ Aj).real
        assert abs(plain.max() - ratio) < 1e-10
        assert opt.min() > 0 and opt.max() < plain.max()
        if ratio <= 3.0:
            assert opt.max() < 2.0
    assert hit >= 5


def _swap_xy_cells(r):
    # cells lexicographic x fastest: index = cx + 2 cy + 4 cz
    out = np.empty_like(r)
    for cz in range(2):
        for cy in range(2):
            for cx in range(2):
                out[cy + 2 * cx + 4 * cz] = r[cx + 2 * cy + 4 * cz]
    return out


def test_targets_symmetries():
    """Swapping the x and y axes swaps mode indices; reflecting x leaves the targets unchanged."""
    q = 3
    rng = np.random.default_rng(3)
    r = np.exp(rng.standard_normal(8))
    c = learned.targets(3, 2, r).reshape(q, q, q)          # [mz, my, mx]
    cs = learned.targets(3, 2, _swap_xy_cells(r)).reshape(q, q, q)
    assert np.abs(cs - np.transpose(c, (0, 2, 1))).max() < 1e-12
    refl = np.array([r[(1 - (i % 2)) + 2 * ((i // 2) % 2) + 4 * (i // 4)] for i in range(8)])
    assert np.abs(learned.targets(3, 2, refl) - c.reshape(-1)).max() < 1e-12


def test_mlp_backward_matches_finite_differences():
    n_in, n_h, n_out = 8, 6, 5
    rng = np.random.default_rng(4)
    p = mlp.init_params(0, n_in, n_h, n_out) + 0.1 * rng.standard_normal(mlp.n_params(n_in, n_h, n_out))
    X = rng.standard_normal((7, n_in))
    T = rng.standard_normal((7, n_out))
    Y, cache = mlp.forward(p, X, n_in, n_h, n_out)
    g = mlp.backward(p, cache, mlp.loss_grad(Y, T), n_in, n_h, n_out)
    eps = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        pp = p.copy(); pp[i] += eps
        pm = p.copy(); pm[i] -= eps
        fd[i] = (mlp.loss(mlp.forward(pp, X, n_in, n_h, n_out)[0], T)
                 - mlp.loss(mlp.forward(pm, X, n_in, n_h, n_out)[0], T)) / (2 * eps)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_mlp_parameter_count():
    assert mlp.n_params(8, 64, 27) == 6491


def test_adam_first_step_closed_form():
    """With m0 = v0 = 0 the first bias-corrected step is -lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3])
    p0 = np.zeros(3)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_scaling_clamp_and_fallback():
    y = np.array([[0.0, 10.0, -10.0], [np.nan, 0.0, 0.0]])
    c = learned.scaling_from_output(y)
    assert np.allclose(c[0], [1.0, 4.0, 0.25])
    assert np.all(c[1] == 1.0)
