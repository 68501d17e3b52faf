"""Spectral-element discretisation of the impedance Helmholtz problem on an
axis-aligned box: the paper's second workload (Sec. VII-B, hexahedral
elements on [-1,1]^3, uniform elements), the same weak form as ``sem`` with
one more tensor factor (Sec. IV: tensor-product GLL elements):
    A = Kx (x) Wy (x) Wz + Wx (x) Ky (x) Wz + Wx (x) Wy (x) Kz,
    M = (Wx Wy Wz) / c^2,   H = sum over the six faces of (face weights) / c,
    S = A - i omega H - omega^2 M,   b = (Wx Wy Wz) f + sum_faces W_face g.

Node numbering: node (i, j, k), flat index (k * Ny + j) * Nx + i.  Faces in
the order x0, x1, y0, y1, z0, z1; the nodes of an x-face ordered by (k, j),
of a y-face by (k, i), of a z-face by (j, i), the last index fastest.
Boundary data g is stored face after face in that order.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .sem import assemble_1d, node_coords_1d


@dataclass(frozen=True)
class Box:
    """nx x ny x nz uniform hexahedral elements of degree P."""
    nx: int
    ny: int
    nz: int
    P: int
    x0: float = -1.0
    x1: float = 1.0
    y0: float = -1.0
    y1: float = 1.0
    z0: float = -1.0
    z1: float = 1.0

    @property
    def hx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def hy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def hz(self):
        return (self.z1 - self.z0) / self.nz

    @property
    def Nx(self):
        return self.nx * self.P + 1

    @property
    def Ny(self):
        return self.ny * self.P + 1

    @property
    def Nz(self):
        return self.nz * self.P + 1

    @property
    def N(self):
        return self.Nx * self.Ny * self.Nz


def node_coords(mesh):
    """(X, Y, Z) flat arrays of length N in the global numbering."""
    xs = node_coords_1d(mesh.nx, mesh.P, mesh.x0, mesh.x1)
    ys = node_coords_1d(mesh.ny, mesh.P, mesh.y0, mesh.y1)
    zs = node_coords_1d(mesh.nz, mesh.P, mesh.z0, mesh.z1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def operators(mesh):
    """A (sparse), the lumped volume weights and the 1D lumped masses."""
    Kx, Wx = assemble_1d(mesh.nx, mesh.P, mesh.hx)
    Ky, Wy = assemble_1d(mesh.ny, mesh.P, mesh.hy)
    Kz, Wz = assemble_1d(mesh.nz, mesh.P, mesh.hz)
    dx, dy, dz = sp.diags(Wx), sp.diags(Wy), sp.diags(Wz)
    A = (sp.kron(dz, sp.kron(dy, Kx)) + sp.kron(dz, sp.kron(Ky, dx))
         + sp.kron(Kz, sp.kron(dy, dx)))
    vol = np.kron(Wz, np.kron(Wy, Wx))
    return A.tocsr(), vol, Wx, Wy, Wz


def face_nodes(Nx, Ny, Nz):
    """Flat node indices of the six faces (x0, x1, y0, y1, z0, z1)."""
    i, j, k = np.arange(Nx), np.arange(Ny), np.arange(Nz)
    kj = np.add.outer(k * Ny * Nx, j * Nx).ravel()
    ki = np.add.outer(k * Ny * Nx, i).ravel()
    ji = np.add.outer(j * Nx, i).ravel()
    return [kj, kj + (Nx - 1), ki, ki + (Ny - 1) * Nx, ji, ji + (Nz - 1) * Ny * Nx]


def face_weights(Wx, Wy, Wz):
    """Lumped 2D weights of each face, matching ``face_nodes``."""
    return [np.kron(Wz, Wy), np.kron(Wz, Wy), np.kron(Wz, Wx), np.kron(Wz, Wx),
            np.kron(Wy, Wx), np.kron(Wy, Wx)]


def boundary_diag(Nx, Ny, Nz, Wx, Wy, Wz, c):
    """Lumped H = sum over faces of diag(W_face / c) (edges and corners get
    one term per face)."""
    H = np.zeros(Nx * Ny * Nz)
    for nodes, w in zip(face_nodes(Nx, Ny, Nz), face_weights(Wx, Wy, Wz)):
        H[nodes] += w / c[nodes]
    return H


def split_faces(g, Nx, Ny, Nz):
    sizes = [Ny * Nz, Ny * Nz, Nx * Nz, Nx * Nz, Nx * Ny, Nx * Ny]
    return np.split(np.asarray(g), np.cumsum(sizes)[:-1])


def load(mesh, f, g=None):
    _, vol, Wx, Wy, Wz = operators(mesh)
    b = vol * np.asarray(f, dtype=complex)
    if g is not None:
        for nodes, w, gs in zip(face_nodes(mesh.Nx, mesh.Ny, mesh.Nz),
                                face_weights(Wx, Wy, Wz),
                                split_faces(g, mesh.Nx, mesh.Ny, mesh.Nz)):
            b[nodes] += w * gs
    return b


def system(mesh, c, omega):
    A, vol, Wx, Wy, Wz = operators(mesh)
    c = np.asarray(c, dtype=float)
    M = vol / c ** 2
    H = boundary_diag(mesh.Nx, mesh.Ny, mesh.Nz, Wx, Wy, Wz, c)
    S = A - 1j * omega * sp.diags(H) - omega ** 2 * sp.diags(M)
    return S.tocsc(), A, M, H


def solve(mesh, c, omega, f, g=None):
    S, _, _, _ = system(mesh, c, omega)
    return spla.splu(S).solve(load(mesh, f, g))


def plane_wave(mesh, omega, c, d):
    """Plane wave u = exp(i k d.x) (constant c) and its impedance data
    g = i k (d.n - 1) u on each face."""
    k = omega / c
    X, Y, Z = node_coords(mesh)
    u = np.exp(1j * k * (d[0] * X + d[1] * Y + d[2] * Z))
    normals = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    parts = []
    for nodes, n in zip(face_nodes(mesh.Nx, mesh.Ny, mesh.Nz), normals):
        dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2]
        parts.append(1j * k * (dn - 1.0) * u[nodes])
    return u, np.concatenate(parts)
