"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects invalid configurations on the host (no GPU work is started)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vps.h")
LIB = os.path.join(ROOT, "paper_2407_02100_amd", "libvps.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vps_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libvps.so is not built (run python -m paper_2407_02100_amd.build)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_symbol():
    from paper_2407_02100_amd import vps
    for n in declared_functions():
        assert n in vps.SIGNATURES, n


def test_status_strings(lib):
    from paper_2407_02100_amd import vps
    assert vps.status_string(0) == "ok"
    assert vps.status_string(-2) == "unsupported configuration"
    assert vps.status_string(-99) == "unknown status"


@pytest.mark.parametrize("cfg,status", [
    (dict(dim=4, degree=2, n_cells=8, n_levels=2), -2),
    (dict(dim=3, degree=6, n_cells=8, n_levels=2), -2),
    (dict(dim=3, degree=2, n_cells=12, n_levels=4), -2),   # 12 not divisible by 8
    (dict(dim=3, degree=2, n_cells=8, n_levels=4), -2),    # coarsest level has 1 cell
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_block=3), -2),
    (dict(dim=3, degree=5, n_cells=8, n_levels=2, patches_per_block=2), -2),  # exceeds the LDS in FP64
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, pre=-1), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, stream_min_cells=-1), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, algorithm=2), -1),
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, algorithm=1), -2),   # separated: 3D only
    (dict(dim=3, degree=1, n_cells=8, n_levels=2, algorithm=1), -2),   # separated: degree >= 2
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patch_order=4), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, batch_layers=-1), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, algorithm=1, batch_layers=2), -2),
    (dict(dim=3, degree=4, n_cells=204, n_levels=2), -2),  # 817^3 FP64 values exceed 32-bit byte offsets
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_wave=4), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, vcycle_graph=2), -1),
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, wave_rows_2d=3), -1),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, wave_rows_2d=1), -2),   # row kernel: 2D only
    (dict(dim=2, degree=1, n_cells=8, n_levels=2, wave_rows_2d=1), -2),   # row kernel: degree >= 2
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_wave=-1), -1),
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, patches_per_wave=2), -2),   # pairs: 3D only
    (dict(dim=3, degree=1, n_cells=8, n_levels=2, patches_per_wave=2), -2),   # pairs: degree 2..4
    (dict(dim=3, degree=5, n_cells=8, n_levels=2, patches_per_wave=2), -2),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_wave=2, patch_order=1), -2),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_wave=2, algorithm=1), -2),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, patches_per_wave=2, patches_per_block=2), -2),
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, patches_per_wave=3), -2),   # rows of patches: 3D only
    (dict(dim=3, degree=1, n_cells=8, n_levels=2, patches_per_wave=3), -2),   # rows of patches: degree 2..5
    (dict(dim=3, degree=5, n_cells=8, n_levels=2, patches_per_wave=3, patch_order=1), -2),
    (dict(dim=3, degree=3, n_cells=8, n_levels=2, patches_per_wave=3, patch_order=3), -2),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, coef=4), -1),
    (dict(dim=2, degree=2, n_cells=8, n_levels=2, coef=3), -2),   # exact local solvers: Q2 in 3D only
    (dict(dim=3, degree=3, n_cells=8, n_levels=2, coef=3), -2),
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, coef=3, vcycle=1), -2),   # ... FP64 only
    (dict(dim=3, degree=2, n_cells=8, n_levels=2, coef=3, batch_layers=2), -2),
])
def test_create_rejects_invalid_configurations(lib, cfg, status):
    from paper_2407_02100_amd import vps
    c = vps.vps_config(cfg["dim"], cfg["degree"], cfg["n_cells"], cfg["n_levels"], cfg.get("pre", 1), 1,
                       cfg.get("vcycle", 0), cfg.get("coef", 0),
                       cfg.get("patches_per_block", 0), cfg.get("stream_min_cells", 0), cfg.get("algorithm", 0),
                       cfg.get("patch_order", 0), cfg.get("batch_layers", 0), cfg.get("patches_per_wave", 0),
                       cfg.get("vcycle_graph", 0), cfg.get("wave_rows_2d", 0))
    h = ctypes.c_void_p()
    st = vps.lib().vps_create(ctypes.byref(c), None, ctypes.byref(h))
    assert st == status
    assert not h.value


def test_binding_loads_a_single_hip_runtime():
    """libvps must bind to the HIP runtime torch already uses (one runtime per process)."""
    import subprocess
    import sys
    code = ("import paper_2407_02100_amd.vps as v; v.lib(); "
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_null_arguments_are_rejected(lib):
    from paper_2407_02100_amd import vps
    L = vps.lib()
    assert L.vps_create(None, None, None) == -1
    assert L.vps_destroy(None) == 0
    assert L.vps_level_nodes(None, 0) == 0
    assert L.vps_sync(None) == -1
