"""CPU checks of the binding's argument validation: every wrong dtype, element count, level or device is
rejected with VPS_E_ARG on the host, before the library is called (a wrong size would otherwise make a
kernel read or write past the tensor).  The context here is a shape-only stand-in (no library handle):
the checks must fire before anything reaches the C ABI."""
import pytest
import torch

from paper_2407_02100_amd import vps


def fake(dim=3, degree=2, n_cells=8, n_levels=3):
    c = vps.Context.__new__(vps.Context)
    c._shape(dim, degree, n_cells, n_levels)
    return c


def f64(n):
    return torch.zeros(n, dtype=torch.float64)


def f32(n):
    return torch.zeros(n, dtype=torch.float32)


def rejected(fn, *args, match=None):
    with pytest.raises(vps.VpsError) as e:
        fn(*args)
    assert e.value.status == vps.VPS_E_ARG
    if match:
        assert match in str(e.value), str(e.value)


def test_shape_bookkeeping():
    c = fake(3, 2, 8, 3)
    assert c._cells == [2, 4, 8]
    assert c._nodes == [5 ** 3, 9 ** 3, 17 ** 3]
    assert c._patches == [1, 27, 343]
    assert (c._nin, c._nout, c._nparams) == (8, 27, 6491)


def test_solver_vectors_must_be_f64_of_the_finest_size():
    c = fake()
    n = c._nodes[-1]
    rejected(c.solve, f32(n), f64(n), match="float64")
    rejected(c.solve, f64(n), f32(n), match="float64")
    rejected(c.solve, f64(n - 1), f64(n), match="elements")
    rejected(c.vcycle, f64(n), f64(n + 1), match="elements")
    rejected(c.vcycle, f32(n), f32(n), match="float64")
    rejected(c.vcycle_iterate, f64(c._nodes[1]), f64(n), 2, match="elements")
    # right dtype and size: the next check is the device (these tensors are on the CPU)
    rejected(c.solve, f64(n), f64(n), match="GPU")


def test_level_operators_check_level_size_and_one_dtype():
    c = fake()
    for lvl in range(3):
        n = c._nodes[lvl]
        rejected(c.smooth, lvl, f64(n), f32(n), match="one dtype")
        rejected(c.smooth, lvl, f64(n + 1), f64(n + 1), match="elements")
        rejected(c.smooth_color, lvl, f32(n), f64(n), 0, match="one dtype")
        rejected(c.apply, lvl, f64(n), f64(n - 1), match="elements")
        rejected(c.residual, lvl, f32(n), f32(n), f64(n), match="one dtype")
    rejected(c.smooth, 3, f64(1), f64(1), match="level")
    rejected(c.smooth, -1, f64(1), f64(1), match="level")
    rejected(c.restrict, 2, f64(c._nodes[2]), f64(c._nodes[2]), match="elements")
    rejected(c.restrict, 0, f64(1), f64(1), match="level")
    rejected(c.restrict, 2, f64(c._nodes[2]), f32(c._nodes[1]), match="one dtype")
    rejected(c.prolongate_add, 1, f64(c._nodes[1]), f64(c._nodes[1]), match="elements")
    rejected(c.coarse_solve, f64(c._nodes[1]), f64(c._nodes[0]), match="elements")
    rejected(c.smooth, 2, torch.zeros(c._nodes[2], dtype=torch.int64), torch.zeros(c._nodes[2], dtype=torch.int64),
             match="dtype")
    rejected(c.smooth, 2, f64(c._nodes[2]), f64(c._nodes[2]), match="GPU")


def test_coefficient_and_learned_buffers():
    c = fake()
    cells = 8 ** 3
    rejected(c.set_coefficient, f32(cells), match="float64")
    rejected(c.set_coefficient, f64(cells - 1), match="elements")
    rejected(c.set_patch_scaling, 2, f64(343 * 27), match="float32")
    rejected(c.set_patch_scaling, 2, f32(343 * 27 - 1), match="elements")
    rejected(c.patch_features, 2, f32(343 * 7), match="elements")
    rejected(c.patch_rho8, 1, f32(27 * 8), match="float64")
    r8 = f64(10 * 8).reshape(10, 8)
    rejected(c.rho8_features, r8, f64(80), match="float32")
    rejected(c.patch_targets, r8, f64(10 * 26), match="elements")
    rejected(c.patch_targets, r8, f64(270), f64(270), match="float32")
    x = f32(80).reshape(10, 8)
    p = f32(6491)
    rejected(c.mlp_forward, f32(6490), x, f32(270), match="elements")
    rejected(c.mlp_forward, p, x, f32(269), match="elements")
    rejected(c.mlp_forward, p, x, f32(270), f32(10 * 127), match="elements")
    rejected(c.mlp_loss_grad, f32(270).reshape(10, 27), f32(270), f64(270), match="float32")
    rejected(c.mlp_backward, p, x, f32(1280), f32(270), f32(6490), match="elements")
    rejected(c.mlp_adam, p, p, p, f32(6490), 1, match="elements")
    rejected(c.mlp_infer_patches, 2, f64(6491), match="float32")
    rejected(c.mlp_forward, p, x, f32(270), match="GPU")


def test_non_tensors_are_rejected():
    c = fake()
    n = c._nodes[-1]
    rejected(c.solve, f64(n), "not a tensor", match="torch tensor")
