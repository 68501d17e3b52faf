"""Pins for the GLL tables of the oracle (paper Sec. IV: nodal GLL basis and
GLL quadrature).  Values come from closed forms in tests/golden and from
exactness properties, never from the oracle itself."""
import math
import os

import numpy as np
import pytest

from oracle import gll

GOLD = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.txt")


def _closed_forms():
    out = {}
    env = {"sqrt": math.sqrt}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        P, xs, ws = [t.strip() for t in line.split("|")]
        out[int(P)] = (np.array([eval(t, env) for t in xs.split(",")]),
                       np.array([eval(t, env) for t in ws.split(",")]))
    return out


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_closed_forms(P):
    x_ref, w_ref = _closed_forms()[P]
    x, w = gll.nodes_weights(P)
    assert np.allclose(x, x_ref, atol=1e-15, rtol=0)
    assert np.allclose(w, w_ref, atol=1e-15, rtol=0)


@pytest.mark.parametrize("P", range(1, 9))
def test_quadrature_exactness(P):
    x, w = gll.nodes_weights(P)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * P):          # exact through degree 2P-1
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    # Lobatto, not Gauss: degree 2P is not integrated exactly
    assert abs(np.dot(w, x ** (2 * P)) - 2.0 / (2 * P + 1)) > 1e-6


@pytest.mark.parametrize("P", range(1, 9))
def test_diff_matrix_on_monomials(P):
    x, _ = gll.nodes_weights(P)
    D = gll.diff_matrix(P)
    assert np.abs(D @ np.ones(P + 1)).max() < 1e-12
    for k in range(1, P + 1):
        assert np.abs(D @ x ** k - k * x ** (k - 1)).max() < 1e-11 * max(1, P * P)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_element_stiffness_exact_integral(P):
    """D^T W D equals the exact integral of l_a' l_b' (degree 2P-2 <= 2P-1),
    checked against Gauss-Legendre quadrature with more points."""
    x, _ = gll.nodes_weights(P)
    K = gll.element_stiffness_1d(P)
    gx, gw = np.polynomial.legendre.leggauss(P + 2)
    V = np.vander(x, P + 1, increasing=True)
    C = np.linalg.inv(V)          # columns: monomial coefficients of l_b
    dl = np.zeros((gx.size, P + 1))
    for b in range(P + 1):
        coeff = C[:, b]
        dl[:, b] = sum(k * coeff[k] * gx ** (k - 1) for k in range(1, P + 1))
    Kex = dl.T @ np.diag(gw) @ dl
    assert np.abs(K - Kex).max() < 1e-11
