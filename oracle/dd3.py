"""Non-overlapping domain decomposition of the box (paper Sec. III, the 3D
workload of Sec. VII-B): an sx x sy x sz grid of equal element blocks, every
subdomain with its own copies of its nodes, impedance (zeroth-order)
transmission on all six faces, the interface update of eq. (2) with the sign
read as in ``dd`` (g_r <- -g_l - 2 i (omega/c) u_l).

Subdomain l = (c * sy + b) * sx + a for block (a, b, c).  Interface data:
per subdomain the six faces in the order x0, x1, y0, y1, z0, z1, each in the
node order of ``sem3.face_nodes``; faces on the outer boundary carry physical
impedance data (zero here).  The sweep, glue and outer iteration have the
interface of ``dd.Decomposition``, so ``dd.solve_dd`` and ``waveholtz``
apply unchanged.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import sem3

OPPOSITE = {0: 1, 1: 0, 2: 3, 3: 2, 4: 5, 5: 4}
STEP = {0: (-1, 0, 0), 1: (1, 0, 0), 2: (0, -1, 0), 3: (0, 1, 0), 4: (0, 0, -1), 5: (0, 0, 1)}


@dataclass(frozen=True)
class Partition3:
    sx: int
    sy: int
    sz: int


class Decomposition3:
    def __init__(self, mesh, part, c, omega):
        if mesh.nx % part.sx or mesh.ny % part.sy or mesh.nz % part.sz:
            raise ValueError("partition must divide the element grid")
        self.mesh, self.part, self.omega, self.q = mesh, part, float(omega), 0.0
        self.c = np.asarray(c, dtype=float)
        self.mx, self.my, self.mz = mesh.nx // part.sx, mesh.ny // part.sy, mesh.nz // part.sz
        P = mesh.P
        self.nxl, self.nyl, self.nzl = self.mx * P + 1, self.my * P + 1, self.mz * P + 1
        self.L = part.sx * part.sy * part.sz
        nx, ny, nz = self.nxl, self.nyl, self.nzl
        self.face_len = [ny * nz, ny * nz, nx * nz, nx * nz, nx * ny, nx * ny]
        self.face_off = list(np.concatenate([[0], np.cumsum(self.face_len)[:-1]]))
        self.per_sub = int(sum(self.face_len))
        self.n_if = self.L * self.per_sub
        self.local_faces = sem3.face_nodes(nx, ny, nz)
        self.subs = [self._build(l) for l in range(self.L)]

    def block(self, l):
        p = self.part
        return l % p.sx, (l // p.sx) % p.sy, l // (p.sx * p.sy)

    def global_nodes(self, l):
        a, b, c = self.block(l)
        P, m = self.mesh.P, self.mesh
        i = a * self.mx * P + np.arange(self.nxl)
        j = b * self.my * P + np.arange(self.nyl)
        k = c * self.mz * P + np.arange(self.nzl)
        return (np.add.outer(np.add.outer(k * m.Ny, j) * m.Nx, i)).ravel()

    def sub_box(self, l):
        a, b, c = self.block(l)
        m = self.mesh
        return sem3.Box(self.mx, self.my, self.mz, m.P,
                        m.x0 + a * self.mx * m.hx, m.x0 + (a + 1) * self.mx * m.hx,
                        m.y0 + b * self.my * m.hy, m.y0 + (b + 1) * self.my * m.hy,
                        m.z0 + c * self.mz * m.hz, m.z0 + (c + 1) * self.mz * m.hz)

    def neighbour(self, l, s):
        a, b, c = self.block(l)
        da, db, dc = STEP[s]
        p = self.part
        a2, b2, c2 = a + da, b + db, c + dc
        if 0 <= a2 < p.sx and 0 <= b2 < p.sy and 0 <= c2 < p.sz:
            return (c2 * p.sy + b2) * p.sx + a2, OPPOSITE[s]
        return None

    def slot(self, l, s):
        o = l * self.per_sub + self.face_off[s]
        return slice(o, o + self.face_len[s])

    def _build(self, l):
        box = self.sub_box(l)
        A, vol, Wx, Wy, Wz = sem3.operators(box)
        cl = self.c[self.global_nodes(l)]
        M = vol / cl ** 2
        H = sem3.boundary_diag(self.nxl, self.nyl, self.nzl, Wx, Wy, Wz, cl)
        S = (A - 1j * self.omega * sp.diags(H) - self.omega ** 2 * sp.diags(M)).tocsc()
        return dict(rect=box, A=A, At=A, M=M, Mt=M, H=H, area=vol, c=cl,
                    face_w=sem3.face_weights(Wx, Wy, Wz), S=S, lu=None)

    def lu(self, l):
        sd = self.subs[l]
        if sd["lu"] is None:
            sd["lu"] = spla.splu(sd["S"])
        return sd["lu"]

    def embed_trace(self, g):
        if g is not None:
            raise NotImplementedError("boundary data in 3D: not needed by the workload")
        return np.zeros(self.n_if, dtype=complex)

    def interface_mask(self):
        m = np.zeros(self.n_if, dtype=bool)
        for l in range(self.L):
            for s in range(6):
                if self.neighbour(l, s) is not None:
                    m[self.slot(l, s)] = True
        return m

    def rhs(self, l, f, g_in, src):
        """b_l = src * (f, phi)_l + sum_faces W_face * g_{l,face}."""
        sd = self.subs[l]
        b = src * sd["area"] * np.asarray(f, dtype=complex)[self.global_nodes(l)]
        for s in range(6):
            b[self.local_faces[s]] += sd["face_w"][s] * g_in[self.slot(l, s)]
        return b

    def exchange(self, l, u, g_in, g_out):
        sd = self.subs[l]
        for s in range(6):
            nb = self.neighbour(l, s)
            if nb is None:
                continue
            r, s2 = nb
            nodes = self.local_faces[s]
            g_out[self.slot(r, s2)] = (-g_in[self.slot(l, s)]
                                       - 2j * (self.omega / sd["c"][nodes]) * u[nodes])

    def sweep(self, g_in, f, src, solver=None):
        g_in = np.asarray(g_in, dtype=complex)
        g_out = np.zeros(self.n_if, dtype=complex)
        us = []
        for l in range(self.L):
            b = self.rhs(l, f, g_in, src)
            u = self.lu(l).solve(b) if solver is None else solver(l, b)
            self.exchange(l, u, g_in, g_out)
            us.append(u)
        return g_out, us

    def glue(self, us):
        acc = np.zeros(self.mesh.N, dtype=complex)
        cnt = np.zeros(self.mesh.N)
        for l, u in enumerate(us):
            idx = self.global_nodes(l)
            np.add.at(acc, idx, u)
            np.add.at(cnt, idx, 1.0)
        return acc / cnt

    def restrict(self, u_global):
        return [np.asarray(u_global)[self.global_nodes(l)] for l in range(self.L)]
