"""Gauss-Lobatto-Legendre (GLL) nodal tables on the reference interval [-1, 1].

The paper discretises with a tensor-product nodal basis on GLL points and uses
GLL quadrature so that the mass and boundary matrices are diagonal (Sec. IV,
the paragraph after eq. (4)).  The textbook definitions used here:

* nodes: -1, the P-1 roots of L_P'(x), +1 (L_P the Legendre polynomial);
* weights: w_a = 2 / (P (P+1) L_P(x_a)^2);
* differentiation matrix D[a, b] = l_b'(x_a) for the Lagrange cardinal
  functions l_b on those nodes.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def _legendre_coeffs(P):
    c = np.zeros(P + 1)
    c[P] = 1.0
    return c


def nodes_weights(P):
    """GLL nodes (ascending) and weights for degree P >= 1."""
    if P < 1:
        raise ValueError("degree must be >= 1")
    c = _legendre_coeffs(P)
    if P == 1:
        inner = np.array([])
    else:
        inner = np.sort(np.real(npleg.legroots(npleg.legder(c))))
        # one Newton polish on L_P'(x) = 0 (roots are real and simple)
        d1 = npleg.legder(c)
        d2 = npleg.legder(c, 2)
        inner = inner - npleg.legval(inner, d1) / npleg.legval(inner, d2)
    x = np.concatenate([[-1.0], inner, [1.0]])
    LP = npleg.legval(x, c)
    w = 2.0 / (P * (P + 1) * LP ** 2)
    return x, w


def diff_matrix(P):
    """D[a, b] = l_b'(x_a) on the GLL nodes (closed form via L_P values)."""
    x, _ = nodes_weights(P)
    LP = npleg.legval(x, _legendre_coeffs(P))
    D = np.zeros((P + 1, P + 1))
    for a in range(P + 1):
        for b in range(P + 1):
            if a != b:
                D[a, b] = LP[a] / (LP[b] * (x[a] - x[b]))
    D[0, 0] = -P * (P + 1) / 4.0
    D[P, P] = P * (P + 1) / 4.0
    return D


def element_stiffness_1d(P):
    """Reference 1D stiffness D^T W D on [-1, 1] (GLL quadrature, exact here
    because l_a' l_b' has degree 2P-2 <= 2P-1)."""
    _, w = nodes_weights(P)
    D = diff_matrix(P)
    return D.T @ np.diag(w) @ D
