"""Host logic of bench.py (no GPU): the node counts behind the algorithmic bytes of a sweep, the slab
ranges of the batched sweep, the launch counts, the name of the finest-level smoother kernel, and the
refusal of more than one GPU.

The counts are checked against brute force: every patch of a color (one per interior vertex of the
color's parity) enumerated with its closure and interior node boxes, and the unions counted.
"""
import itertools
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def brute_counts(dim, k, n, vlo=1, vhi=None):
    """Per color: (nodes in the union of the closures, nodes in the union of the interiors) of the patches
    whose vertex has the color's parity and whose slowest coordinate lies in [vlo, vhi]."""
    vhi = n - 1 if vhi is None else vhi
    out = []
    for color in range(2 ** dim):
        clo, inner = set(), set()
        for v in itertools.product(range(1, n), repeat=dim):
            if any((v[e] & 1) != ((color >> e) & 1) for e in range(dim)):
                continue
            if not (vlo <= v[dim - 1] <= vhi):
                continue
            clo.update(itertools.product(*[range(k * (c - 1), k * (c + 1) + 1) for c in v]))
            inner.update(itertools.product(*[range(k * (c - 1) + 1, k * (c + 1)) for c in v]))
        out.append((len(clo), len(inner)))
    return out


@pytest.mark.parametrize("dim,k,n", [(2, 1, 6), (2, 2, 6), (2, 3, 5), (2, 5, 4), (3, 1, 5), (3, 2, 4), (3, 4, 3),
                                     (3, 3, 6), (3, 5, 3), (3, 5, 5)])
def test_color_counts_match_brute_force(dim, k, n):
    assert bench.color_counts(dim, k, n) == brute_counts(dim, k, n)


@pytest.mark.parametrize("dim,k,n,vlo,vhi", [(3, 2, 8, 1, 2), (3, 2, 8, 3, 4), (3, 2, 8, 5, 7), (2, 3, 9, 3, 6),
                                             (3, 1, 7, 2, 2), (2, 2, 6, 4, 5)])
def test_color_counts_of_a_slab_match_brute_force(dim, k, n, vlo, vhi):
    assert bench.color_counts(dim, k, n, vlo, vhi) == brute_counts(dim, k, n, vlo, vhi)


@pytest.mark.parametrize("n,B", [(8, 2), (9, 2), (128, 32), (128, 48), (128, 64), (129, 32), (64, 7), (16, 0)])
def test_batches_partition_the_vertex_layers(n, B):
    """The slabs cover the vertex layers 1..n-1 once, in order, B layers each (the last may be shorter);
    levels with at most 2B layers sweep whole colors."""
    r = bench.batches(n, B)
    if B <= 0 or n - 1 <= 2 * B:
        assert r == [(1, n - 1)]
        return
    layers = [v for lo, hi in r for v in range(lo, hi + 1)]
    assert layers == list(range(1, n))
    assert all(hi - lo + 1 == B for lo, hi in r[:-1]) and 1 <= r[-1][1] - r[-1][0] + 1 <= B


def test_sweep_bytes_of_the_513_workload():
    """The algorithmic bytes per launch quoted for the 3D Q4 128^3 FP32 sweep: 1,230,084,285 per color on
    whole colors (8 launches), 308,298,314.25 per launch in slabs of 32 layers (32 launches, the closure
    planes shared by neighbouring slabs read twice)."""
    whole = bench.sweep_bytes(3, 4, 128, 4)
    assert bench.launches_per_sweep(3, 128) == 8 and whole == 8 * 1_230_084_285
    slabs = bench.sweep_bytes(3, 4, 128, 4, 32)
    assert bench.launches_per_sweep(3, 128, 32) == 32 and slabs == 32 * 308_298_314.25
    assert slabs > whole
    # each color reads most of the grid once (a color whose patches start at vertex 2 skips the first
    # cell layer in that direction) and writes its interiors, the fraction f = (q / 2k)^d = (7/8)^3 of
    # the nodes
    n = (4 * 128 + 1) ** 3
    counts = bench.color_counts(3, 4, 128)
    assert 0.95 * n < sum(c for c, _ in counts) / 8 <= n
    assert abs(sum(i for _, i in counts) / 8 / n - (7 / 8) ** 3) < 0.02


def test_sweep_bytes_of_the_paper_q5_shape():
    """The algorithmic bytes of one FP64 sweep of the paper's 3D Q5 128^3 shape (641^3 nodes), whole colors."""
    byt = bench.sweep_bytes(3, 5, 128, 8)
    assert byt == sum((c + 2 * i) * 8 for c, i in bench.color_counts(3, 5, 128))
    assert byt == 40_356_944_496
    n = 641 ** 3
    assert 8 * n * 8 * 0.95 < byt - 2 * 8 * sum(i for _, i in bench.color_counts(3, 5, 128)) <= 8 * n * 8


@pytest.mark.parametrize("dim,k,n,vcycle,coef,want", [
    (3, 4, 128, "f32", "const", "patch_row3_kernel"), (3, 4, 64, "f64", "const", "patch_row3_kernel"),
    (3, 4, 32, "f32", "const", "patch_wave3_kernel"), (3, 4, 32, "f64", "const", "patch_pair3_kernel"),
    (3, 3, 32, "f32", "const", "patch_pair3_kernel"), (3, 2, 32, "f64", "const", "patch_row3_kernel"),
    (3, 2, 16, "f64", "const", "patch_wave3_kernel"), (3, 5, 128, "f64", "const", "patch_row5_kernel"),
    (3, 5, 32, "f64", "const", "patch_big3_kernel"), (3, 5, 64, "f32", "const", "patch_row5_kernel"),
    (2, 3, 2048, "f64", "const", "patch_row2_kernel"), (3, 2, 64, "f64", "learned", "patch_color_kernel")])
def test_finest_smoother_kernel_follows_the_automatic_choice(dim, k, n, vcycle, coef, want):
    assert bench.finest_smoother_kernel(dim, k, n, vcycle, coef) == want


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_median_helper_handles_one_and_three_runs():
    import bench
    calls = []
    t, out = bench._median3(lambda: calls.append(1) or len(calls), 1)
    assert out == 1 and len(calls) == 1 and t >= 0.0
    t, out = bench._median3(lambda: calls.append(1) or len(calls))
    assert out == 4 and len(calls) == 4


def test_source_hash_ignores_comments_only():
    from paper_2407_02100_amd import traffic_probe as tp
    src = 'int a = 1; // x\n/* y */ const char* s = "// kept /* kept */"; char q = \'"\'; /* z\n w */ int b;\n'
    out = tp.strip_comments(src)
    assert "// kept /* kept */" in out and "x" not in out.replace("// kept", "") and "int b;" in out
    assert out.count("\n") == 2  # a block comment's newlines go with it; a line comment keeps its newline
    assert tp.strip_comments("a /* c */ b") == "a   b"


def test_committed_traffic_profiles_match_the_sources():
    """The committed FETCH/WRITE summaries were taken with the current kernel code (else the bench line's
    roofline.traffic is null)."""
    import json
    from paper_2407_02100_amd import traffic_probe as tp
    for name, dtype, bl in (("patch_sweep_traffic.json", "f32", 44), ("patch_sweep_traffic_f64.json", "f64", 0)):
        path = os.path.join(ROOT, "profiles", name)
        doc = json.load(open(path))
        assert doc["kernel_source_hash"] == tp.kernel_source_hash(), name
        assert bench.traffic_per_launch(path, "poisson3d_q4_n128", bl, dtype) == doc["bytes_per_launch"]
