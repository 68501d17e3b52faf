"""Dense brute-force assembly for tiny meshes (independent check of ``sem``).

Builds every global basis function's element restriction from explicit
Lagrange cardinal polynomials (numpy Polynomial objects, differentiated
symbolically, not through the differentiation matrix D), evaluates the
integrands of eq. (4) at the GLL quadrature points of each element and sums
element by element into dense matrices.  This is the definition of A, M, H
and b (Sec. IV) written out with GLL quadrature (Sec. IV, after eq. (4)).
"""
import numpy as np
from numpy.polynomial import Polynomial

from . import gll


def _cardinals(P):
    x, _ = gll.nodes_weights(P)
    polys = []
    for b in range(P + 1):
        p = Polynomial([1.0])
        for m in range(P + 1):
            if m != b:
                p = p * Polynomial([-x[m], 1.0]) / (x[b] - x[m])
        polys.append(p)
    return x, polys


def assemble(mesh, c, f=None):
    """Dense A, M, H (and b = (f, phi) if f is given) on the global nodes."""
    P = mesh.P
    x, polys = _cardinals(P)
    _, w = gll.nodes_weights(P)
    val = np.array([[p(xq) for p in polys] for xq in x])             # val[q, a]
    der = np.array([[p.deriv()(xq) for p in polys] for xq in x])     # der[q, a]
    hx, hy = mesh.hx, mesh.hy
    Nx, N = mesh.Nx, mesh.N
    A = np.zeros((N, N))
    M = np.zeros((N, N))
    H = np.zeros((N, N))
    b = np.zeros(N, dtype=complex)
    c = np.asarray(c, dtype=float)
    nloc = (P + 1) ** 2
    for ey in range(mesh.ny):
        for ex in range(mesh.nx):
            gidx = np.array([(ey * P + bb) * Nx + ex * P + aa
                             for bb in range(P + 1) for aa in range(P + 1)])
            Ae = np.zeros((nloc, nloc))
            Me = np.zeros((nloc, nloc))
            for qy in range(P + 1):
                for qx in range(P + 1):
                    wq = w[qx] * w[qy] * hx * hy / 4.0
                    cq = c[gidx[qy * (P + 1) + qx]]
                    phi = np.array([val[qx, aa] * val[qy, bb]
                                    for bb in range(P + 1) for aa in range(P + 1)])
                    dx = np.array([der[qx, aa] * val[qy, bb] * 2.0 / hx
                                   for bb in range(P + 1) for aa in range(P + 1)])
                    dy = np.array([val[qx, aa] * der[qy, bb] * 2.0 / hy
                                   for bb in range(P + 1) for aa in range(P + 1)])
                    Ae += wq * (np.outer(dx, dx) + np.outer(dy, dy))
                    Me += wq * np.outer(phi, phi) / cq ** 2
                    if f is not None:
                        b[gidx] += wq * f[gidx[qy * (P + 1) + qx]] * phi
            A[np.ix_(gidx, gidx)] += Ae
            M[np.ix_(gidx, gidx)] += Me
    # boundary integrals <c^-1 phi_j, phi_i> by 1D GLL quadrature per edge
    Ny = mesh.Ny
    edges = []
    for ex in range(mesh.nx):
        for j in (0, Ny - 1):
            edges.append(([j * Nx + ex * P + a for a in range(P + 1)], hx))
    for ey in range(mesh.ny):
        for i in (0, Nx - 1):
            edges.append(([(ey * P + a) * Nx + i for a in range(P + 1)], hy))
    for nodes, h in edges:
        nodes = np.array(nodes)
        He = np.zeros((P + 1, P + 1))
        for q in range(P + 1):
            He += w[q] * h / 2.0 * np.outer(val[q], val[q]) / c[nodes[q]]
        H[np.ix_(nodes, nodes)] += He
    return A, M, H, b
