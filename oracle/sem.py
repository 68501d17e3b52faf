"""Spectral-element discretisation of the impedance Helmholtz problem on an
axis-aligned rectangle (paper Sec. II eq. (1); Sec. IV eqs. (3)-(4)).

Problem (time convention e^{-i omega t}, k = omega / c(x)):
    -Lap u - k^2 u = f in Omega,   d_n u - i k u = g on dOmega.
Weak form with the impedance term carrying the factor i (reading of eq. (3)
that matches eq. (4) and the definition of H):
    (grad u, grad phi) - (k^2 u, phi) - i <k u, phi> = (f, phi) + <g, phi>.
Discrete system, eq. (4):  S u = b,  S = A - i omega H - omega^2 M, with
    A_ij = (grad phi_j, grad phi_i),  M_ij = (c^-2 phi_j, phi_i),
    H_ij = <c^-1 phi_j, phi_i>,        b_j = (f, phi_j) + <g, phi_j>,
all integrals by GLL quadrature on the nodes (Sec. IV, after eq. (4)), so M
and H are diagonal and A is the Kronecker sum  A = Kx (x) Wy + Wx (x) Ky  of
the assembled 1D stiffness K and lumped 1D mass W.

Node numbering: global node (i, j), i along x, j along y, flat index
j * Nx + i with Nx = nx*P + 1.  Boundary traces are stored side by side in the
order left (x = x0), right (x = x1), bottom (y = y0), top (y = y1), each side
ordered by increasing coordinate: length 2*Ny + 2*Nx.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import gll


@dataclass(frozen=True)
class Rect:
    """nx x ny uniform quadrilateral elements of degree P on [x0,x1]x[y0,y1]."""
    nx: int
    ny: int
    P: int
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0

    @property
    def hx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def hy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def Nx(self):
        return self.nx * self.P + 1

    @property
    def Ny(self):
        return self.ny * self.P + 1

    @property
    def N(self):
        return self.Nx * self.Ny


def assemble_1d(n, P, h):
    """Assembled 1D stiffness (sparse) and lumped mass (vector) for n
    elements of length h: K = sum_e (2/h) D^T W D, W = sum_e (h/2) w."""
    Ke = gll.element_stiffness_1d(P) * (2.0 / h)
    _, w = gll.nodes_weights(P)
    N = n * P + 1
    rows, cols, vals = [], [], []
    W = np.zeros(N)
    for e in range(n):
        idx = np.arange(e * P, e * P + P + 1)
        rows.append(np.repeat(idx, P + 1))
        cols.append(np.tile(idx, P + 1))
        vals.append(Ke.ravel())
        W[idx] += 0.5 * h * w
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    K.sum_duplicates()
    return K, W


def node_coords_1d(n, P, a, b):
    """GLL node coordinates of n uniform elements on [a, b]."""
    x, _ = gll.nodes_weights(P)
    h = (b - a) / n
    out = np.empty(n * P + 1)
    for e in range(n):
        out[e * P:e * P + P + 1] = a + e * h + 0.5 * h * (x + 1.0)
    out[-1] = b
    return out


def node_coords(mesh):
    """(X, Y) flat arrays of length N in the global numbering."""
    xs = node_coords_1d(mesh.nx, mesh.P, mesh.x0, mesh.x1)
    ys = node_coords_1d(mesh.ny, mesh.P, mesh.y0, mesh.y1)
    X, Y = np.meshgrid(xs, ys)  # shape (Ny, Nx): row j, column i
    return X.ravel(), Y.ravel()


def operators(mesh):
    """A (sparse), the lumped area weights Wx(x)Wy (vector) and the 1D
    lumped masses (Wx, Wy)."""
    Kx, Wx = assemble_1d(mesh.nx, mesh.P, mesh.hx)
    Ky, Wy = assemble_1d(mesh.ny, mesh.P, mesh.hy)
    A = sp.kron(sp.diags(Wy), Kx) + sp.kron(Ky, sp.diags(Wx))
    area = np.kron(Wy, Wx)
    return A.tocsr(), area, Wx, Wy


def side_nodes(Nx, Ny):
    """Flat node indices of the four sides (left, right, bottom, top) of an
    Nx x Ny node grid, each ordered by increasing coordinate."""
    j = np.arange(Ny)
    i = np.arange(Nx)
    return [j * Nx, j * Nx + (Nx - 1), i, (Ny - 1) * Nx + i]


def side_weights(Wx, Wy):
    """Lumped 1D boundary weights for each side, matching ``side_nodes``."""
    return [Wy, Wy, Wx, Wx]


def boundary_diag(Nx, Ny, Wx, Wy, c):
    """Lumped H = sum over sides of diag(W_side / c) (corners get two terms)."""
    H = np.zeros(Nx * Ny)
    for nodes, w in zip(side_nodes(Nx, Ny), side_weights(Wx, Wy)):
        H[nodes] += w / c[nodes]
    return H


def split_trace(g, Nx, Ny):
    """Cut a boundary trace array (left, right, bottom, top) into sides."""
    g = np.asarray(g)
    return [g[:Ny], g[Ny:2 * Ny], g[2 * Ny:2 * Ny + Nx], g[2 * Ny + Nx:2 * Ny + 2 * Nx]]


def load(mesh, f, g=None):
    """b = (f, phi) + <g, phi> by GLL quadrature (eq. (4), definition of b)."""
    _, area, Wx, Wy = operators(mesh)
    b = area * np.asarray(f, dtype=complex)
    if g is not None:
        for nodes, w, gs in zip(side_nodes(mesh.Nx, mesh.Ny), side_weights(Wx, Wy),
                                split_trace(g, mesh.Nx, mesh.Ny)):
            b[nodes] += w * gs
    return b


def system(mesh, c, omega):
    """S = A - i omega H - omega^2 M, eq. (4), with lumped M and H."""
    A, area, Wx, Wy = operators(mesh)
    c = np.asarray(c, dtype=float)
    M = area / c ** 2
    H = boundary_diag(mesh.Nx, mesh.Ny, Wx, Wy, c)
    S = A - 1j * omega * sp.diags(H) - omega ** 2 * sp.diags(M)
    return S.tocsc(), A, M, H


def solve(mesh, c, omega, f, g=None):
    """Global discrete solution u* of S u = b by sparse LU (SuperLU)."""
    S, _, _, _ = system(mesh, c, omega)
    b = load(mesh, f, g)
    return spla.splu(S).solve(b)


def residual(mesh, c, omega, f, g, u):
    """Relative residual ||b - S u||_2 / ||b||_2 in FP64."""
    S, _, _, _ = system(mesh, c, omega)
    b = load(mesh, f, g)
    return np.linalg.norm(b - S @ u) / np.linalg.norm(b)


def plane_wave(mesh, omega, c, d):
    """Exact plane wave u = exp(i k d.x) (constant c) and its impedance data
    g = i k (d.n - 1) u on each side (eq. (1b)) as a boundary trace array."""
    k = omega / c
    X, Y = node_coords(mesh)
    u = np.exp(1j * k * (d[0] * X + d[1] * Y))
    normals = [(-1.0, 0.0), (1.0, 0.0), (0.0, -1.0), (0.0, 1.0)]
    parts = []
    for nodes, n in zip(side_nodes(mesh.Nx, mesh.Ny), normals):
        dn = d[0] * n[0] + d[1] * n[1]
        parts.append(1j * k * (dn - 1.0) * u[nodes])
    return u, np.concatenate(parts)
