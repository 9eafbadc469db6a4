"""Pins of the oracle's 1D element against closed forms (textbook integrals)."""
import os

import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

from oracle import fe

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fe_closed_forms.txt")


def _golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, val = [s.strip() for s in line.split("=", 1)]
        out[key] = val
    return out


def _mat(s):
    return np.array([[float(x) for x in row.split()] for row in s.split(";")])


def _frac(s):
    a, b = s.split("/")
    return float(a) / float(b)


def test_closed_form_k1_k2():
    g = _golden()
    M1, K1 = fe.reference_matrices(1)
    assert np.allclose(M1, _frac(g["mass_k1_scale"]) * _mat(g["mass_k1"]), atol=1e-15)
    assert np.allclose(K1, _mat(g["stiff_k1"]), atol=1e-14)
    M2, K2 = fe.reference_matrices(2)
    assert np.allclose(M2, _frac(g["mass_k2_scale"]) * _mat(g["mass_k2"]), atol=1e-15)
    assert np.allclose(K2, _frac(g["stiff_k2_scale"]) * _mat(g["stiff_k2"]), atol=1e-13)


def test_gll_closed_forms():
    x3 = fe.gll_nodes(3)
    s5 = 1.0 / np.sqrt(5.0)
    assert np.allclose(x3, [0.0, 0.5 * (1 - s5), 0.5 * (1 + s5), 1.0], atol=1e-15)
    x4 = fe.gll_nodes(4)
    s = np.sqrt(3.0 / 7.0)
    assert np.allclose(x4, [0.0, 0.5 * (1 - s), 0.5, 0.5 * (1 + s), 1.0], atol=1e-15)
    assert np.allclose(fe.gll_nodes(2), [0.0, 0.5, 1.0], atol=1e-15)
    # k = 5: the interior nodes are the roots of P_5', 21 x^4 - 14 x^2 + 1 = 0 on [-1, 1]
    a5, b5 = np.sqrt(1.0 / 3.0 - 2.0 * np.sqrt(7.0) / 21.0), np.sqrt(1.0 / 3.0 + 2.0 * np.sqrt(7.0) / 21.0)
    want = 0.5 * (1.0 + np.array([-1.0, -b5, -a5, a5, b5, 1.0]))
    assert np.allclose(fe.gll_nodes(5), want, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_mass_stiffness_on_polynomials(k):
    """u^T M u = int u^2 and u^T K u = int u'^2 for u in P_k (exact integrals)."""
    rng = np.random.default_rng(k)
    coef = rng.standard_normal(k + 1)
    nodes = fe.gll_nodes(k)
    u = npoly.polyval(nodes, coef)
    M, K = fe.reference_matrices(k)
    sq = npoly.polymul(coef, coef)
    d = npoly.polyder(coef)
    dsq = npoly.polymul(d, d)
    int_u2 = npoly.polyval(1.0, npoly.polyint(sq)) - npoly.polyval(0.0, npoly.polyint(sq))
    int_du2 = npoly.polyval(1.0, npoly.polyint(dsq)) - npoly.polyval(0.0, npoly.polyint(dsq))
    assert abs(u @ M @ u - int_u2) <= 1e-13 * max(1.0, abs(int_u2))
    assert abs(u @ K @ u - int_du2) <= 1e-12 * max(1.0, abs(int_du2))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_partition_of_unity(k):
    M, K = fe.reference_matrices(k)
    assert abs(M.sum() - 1.0) < 1e-14
    assert np.abs(K.sum(axis=1)).max() < 1e-12
    assert np.allclose(M, M.T) and np.allclose(K, K.T)


def test_assembled_1d_scaling():
    M, K = fe.assembled_1d(3, 4)
    assert abs(M.sum() - 1.0) < 1e-14
    # K applied to the linear function x gives 0 in the interior rows
    from oracle.mesh import node_coords_1d
    x = node_coords_1d(3, 4)
    assert np.abs((K @ x)[1:-1]).max() < 1e-12
