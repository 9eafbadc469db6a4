"""Checks of the seeded input generators (layout, determinism, GRF statistics)."""
import numpy as np

import vps_inputs as vi


def test_seeded_vector_layout():
    v = vi.seeded_vector(3, 2, 4, 1)
    assert v.size == 9 ** 3
    g = v.reshape(9, 9, 9)
    assert np.all(g[0] == 0) and np.all(g[-1] == 0)
    assert np.all(g[:, 0] == 0) and np.all(g[:, :, -1] == 0)
    inner = g[1:-1, 1:-1, 1:-1]
    assert inner.min() >= -1 and inner.max() <= 1 and np.all(inner != 0)
    assert np.array_equal(v, vi.seeded_vector(3, 2, 4, 1))
    assert not np.array_equal(v, vi.seeded_vector(3, 2, 4, 2))


def test_grf_statistics():
    """Unit variance and Gaussian correlation exp(-r^2/(2 l^2)) at lag r = l (averaged over seeds)."""
    n = 32
    vals, lag = [], []
    for s in range(8):
        g = vi.grf_cells(n, s, corr_len=1.0 / 8.0)
        vals.append(g.var())
        sh = n // 8  # lag of one correlation length along x
        lag.append(np.mean(g[:, :, :-sh] * g[:, :, sh:]))
    assert abs(np.mean(vals) - 1.0) < 0.15
    assert abs(np.mean(lag) - np.exp(-0.5)) < 0.15


def test_workloads_are_consistent():
    for name, w in vi.WORKLOADS.items():
        assert w["n_cells"] % 2 ** (w["levels"] - 1) == 0
        # coarsest mesh: 4 cells per direction; the paper's shapes go down to their single patch
        assert w["n_cells"] // 2 ** (w["levels"] - 1) == (2 if name.startswith("paper") else 4)


def test_learned_params_save_load_round_trip(tmp_path):
    """Checkpoint of the MLP parameters: save_params / load_params give back the same FP32 values."""
    import torch
    from paper_2407_02100_amd import learned
    p = learned.init_params(3)
    assert p.dtype == np.float32 and p.size == 6491
    path = str(tmp_path / "mlp.npy")
    learned.save_params(path, torch.from_numpy(p))
    back = learned.load_params(path, device="cpu")
    assert back.dtype == torch.float32 and np.array_equal(back.numpy(), p)
    learned.save_params(path, p)  # plain arrays too
    assert np.array_equal(learned.load_params(path, device="cpu").numpy(), p)
