"""Non-overlapping domain decomposition with impedance transmission
(paper Sec. III; Sec. IV for the subdomain discretisation).

Partition: an sx x sy grid of equal element blocks (every element in exactly
one subdomain, interface nodes duplicated).  Subdomain l = b * sx + a for block
column a, block row b.  Each subdomain assembles A_l, M_l, F_l from its own
elements only and H_l over all four of its sides, since outer and interface
sides carry the same impedance form (d_n - i k) (Sec. III, zeroth-order
transmission condition):
    S_l u_l = b_l,   b_l = src * (f, phi)_l + sum_sides W_side * g_{l,side}.

Interface data ("g") layout, shared with the HIP library by specification:
for l in 0..L-1, sides (left, right, bottom, top), each side ordered by
increasing coordinate; side length nyl (left/right) or nxl (bottom/top), where
nxl = mx*P + 1, nyl = my*P + 1.  One slot per side and subdomain; a slot on the
outer boundary holds physical impedance data.

Interface update (eq. (2) and the last step of Algorithm 1), with the sign
that makes the fixed point the global discrete solution: for an interface
side s of l facing side s' of r,
    g_{r,s'} <- -g_{l,s} - 2 i (omega / c) u_l   on the shared nodes.
(The paper prints +2ik; with +<g, phi> in b and outward normals the
consistency condition (d_{n_l} - ik)u + (d_{n_r} - ik)u = -2iku forces -2ik.)
Physical slots of the output are zero.

Second-order transmission condition (optional, q > 0).  The paper takes the
zeroth-order condition for simplicity and names optimized / higher-order
conditions as the natural replacement (Sec. III and the conclusion).  Reading
taken here: on interface sides
    B = d_n - i k - q (d_tt + k^2),   q >= 0 a real length,
i.e. the second-order term of the Taylor expansion of the transparent
condition with a real coefficient, so that it stays local in time.  Its weak
form adds q <d_t u, d_t phi> - q k^2 <u, phi> on the side: a 1D stiffness and
a 1D mass along the side.  They are lumped so that the subdomain operator
keeps its Kronecker form with the side's lumped 1D weights extended by q at
every interface end:
    Wx' = Wx + q (e_first [left is an interface] + e_last [right is one]),
    A' = Kx (x) Wy' + Wx' (x) Ky,   M' = Wx' (x) Wy' / c^2,
(H, the source weights and the weights of g in b stay unextended).  This is
the side terms q (K_side - omega^2 W_side / c^2) plus q^2 / c^2 at a corner
where two interface sides meet, which the update splits evenly between the
two sides:
    g_{r,s'} <- -g_{l,s} - 2 i (omega/c) u_l
                + 2 (q K_side u_l - omega^2 m u_l / c^2) / W_side,
    m = q W_side (+ q^2/2 at an end whose other side is an interface).
Summed over the subdomains that share a node, the extra terms cancel against
the interface data, so the fixed point is still the global solution.  Since
Wx' >= Wx, lambda_max(M'^-1 A') obeys the same time-step bound.  For a
Fourier mode e^{i xi t} along a straight interface the two-subdomain
convergence factor is |(s - lam)/(s + lam)|^2, s = -ik + q (xi^2 - k^2),
lam = sqrt(xi^2 - k^2): below 1 for evanescent modes (xi > k) when q > 0,
where the zeroth-order condition (q = 0) leaves it at exactly 1.

Outer iteration (Sec. III, last paragraph): the sweep is affine,
G' = T G + h with h = sweep(g_phys, src=1) and T G = sweep(G, src=0); the
fixed point solves (I - T) G = h.  The Krylov method is not named in the
paper; this oracle uses restarted GMRES(m) with modified Gram-Schmidt and
Givens rotations from G = 0, and plain fixed-point iteration as a baseline.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import sem

LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3
OPPOSITE = {LEFT: RIGHT, RIGHT: LEFT, BOTTOM: TOP, TOP: BOTTOM}


@dataclass(frozen=True)
class Partition:
    sx: int
    sy: int


class Decomposition:
    """Geometry and per-subdomain systems of a uniform block partition."""

    def __init__(self, mesh, part, c, omega, q=0.0):
        if mesh.nx % part.sx or mesh.ny % part.sy:
            raise ValueError("partition must divide the element grid")
        if not q >= 0.0:
            raise ValueError("q must be >= 0")
        self.mesh, self.part, self.omega, self.q = mesh, part, float(omega), float(q)
        self.c = np.asarray(c, dtype=float)
        self.mx, self.my = mesh.nx // part.sx, mesh.ny // part.sy
        P = mesh.P
        self.nxl, self.nyl = self.mx * P + 1, self.my * P + 1
        self.L = part.sx * part.sy
        self.side_len = [self.nyl, self.nyl, self.nxl, self.nxl]
        self.side_off = [0, self.nyl, 2 * self.nyl, 2 * self.nyl + self.nxl]
        self.per_sub = 2 * self.nyl + 2 * self.nxl
        self.n_if = self.L * self.per_sub
        self.local_sides = sem.side_nodes(self.nxl, self.nyl)
        self.subs = [self._build(l) for l in range(self.L)]

    # ---- geometry -------------------------------------------------------
    def block(self, l):
        return l % self.part.sx, l // self.part.sx

    def global_nodes(self, l):
        """Global flat node index of each local node (local row-major)."""
        a, b = self.block(l)
        P = self.mesh.P
        i = a * self.mx * P + np.arange(self.nxl)
        j = b * self.my * P + np.arange(self.nyl)
        return (j[:, None] * self.mesh.Nx + i[None, :]).ravel()

    def sub_rect(self, l):
        a, b = self.block(l)
        m = self.mesh
        return sem.Rect(self.mx, self.my, m.P,
                        m.x0 + a * self.mx * m.hx, m.x0 + (a + 1) * self.mx * m.hx,
                        m.y0 + b * self.my * m.hy, m.y0 + (b + 1) * self.my * m.hy)

    def neighbour(self, l, s):
        """(r, s') across side s of l, or None on the outer boundary."""
        a, b = self.block(l)
        da, db = {LEFT: (-1, 0), RIGHT: (1, 0), BOTTOM: (0, -1), TOP: (0, 1)}[s]
        a2, b2 = a + da, b + db
        if 0 <= a2 < self.part.sx and 0 <= b2 < self.part.sy:
            return b2 * self.part.sx + a2, OPPOSITE[s]
        return None

    def slot(self, l, s):
        o = l * self.per_sub + self.side_off[s]
        return slice(o, o + self.side_len[s])

    # ---- subdomain systems ---------------------------------------------
    def _build(self, l):
        rect = self.sub_rect(l)
        A, area, Wx, Wy = sem.operators(rect)
        cl = self.c[self.global_nodes(l)]
        M = area / cl ** 2
        H = sem.boundary_diag(self.nxl, self.nyl, Wx, Wy, cl)
        Kx, _ = sem.assemble_1d(rect.nx, rect.P, rect.hx)
        Ky, _ = sem.assemble_1d(rect.ny, rect.P, rect.hy)
        iface = [self.neighbour(l, s) is not None for s in range(4)]
        # second-order transmission terms: 1D weights extended at interface ends
        Wxt, Wyt = Wx.copy(), Wy.copy()
        Wxt[0] += self.q * iface[LEFT]
        Wxt[-1] += self.q * iface[RIGHT]
        Wyt[0] += self.q * iface[BOTTOM]
        Wyt[-1] += self.q * iface[TOP]
        At = (sp.kron(sp.diags(Wyt), Kx) + sp.kron(Ky, sp.diags(Wxt))).tocsr()
        Mt = np.kron(Wyt, Wxt) / cl ** 2
        S = (At - 1j * self.omega * sp.diags(H) - self.omega ** 2 * sp.diags(Mt)).tocsc()
        return dict(rect=rect, A=A, M=M, At=At, Mt=Mt, H=H, area=area, c=cl, iface=iface,
                    side_w=sem.side_weights(Wx, Wy), side_K=[Ky, Ky, Kx, Kx], S=S, lu=None)

    def lu(self, l):
        sd = self.subs[l]
        if sd["lu"] is None:
            sd["lu"] = spla.splu(sd["S"])
        return sd["lu"]

    # ---- data movement --------------------------------------------------
    def embed_trace(self, g):
        """Put a global boundary trace (left, right, bottom, top) into the
        physical slots of an interface-layout vector (interfaces zero)."""
        out = np.zeros(self.n_if, dtype=complex)
        if g is None:
            return out
        sides = sem.split_trace(g, self.mesh.Nx, self.mesh.Ny)
        P = self.mesh.P
        for l in range(self.L):
            a, b = self.block(l)
            for s in range(4):
                if self.neighbour(l, s) is not None:
                    continue
                if s in (LEFT, RIGHT):
                    o = b * self.my * P
                    out[self.slot(l, s)] = sides[s][o:o + self.nyl]
                else:
                    o = a * self.mx * P
                    out[self.slot(l, s)] = sides[s][o:o + self.nxl]
        return out

    def interface_mask(self):
        """True on slots that belong to an interface side."""
        m = np.zeros(self.n_if, dtype=bool)
        for l in range(self.L):
            for s in range(4):
                if self.neighbour(l, s) is not None:
                    m[self.slot(l, s)] = True
        return m

    def rhs(self, l, f, g_in, src):
        """b_l = src * (f, phi)_l + sum_sides W_side * g_{l,side}."""
        sd = self.subs[l]
        b = src * sd["area"] * np.asarray(f, dtype=complex)[self.global_nodes(l)]
        for s in range(4):
            b[self.local_sides[s]] += sd["side_w"][s] * g_in[self.slot(l, s)]
        return b

    def exchange(self, l, u, g_in, g_out):
        """Write -g_{l,s} - 2 i (omega/c) u_l (+ the second-order terms) into
        each neighbour's slot."""
        sd = self.subs[l]
        # the sides meeting side s at its first / last node
        ends = {LEFT: (BOTTOM, TOP), RIGHT: (BOTTOM, TOP), BOTTOM: (LEFT, RIGHT), TOP: (LEFT, RIGHT)}
        for s in range(4):
            nb = self.neighbour(l, s)
            if nb is None:
                continue
            r, s2 = nb
            nodes = self.local_sides[s]
            c = sd["c"][nodes]
            g = -g_in[self.slot(l, s)] - 2j * (self.omega / c) * u[nodes]
            if self.q > 0.0:
                W = sd["side_w"][s]
                m = self.q * W
                m[0] += 0.5 * self.q ** 2 * sd["iface"][ends[s][0]]
                m[-1] += 0.5 * self.q ** 2 * sd["iface"][ends[s][1]]
                g = g + 2.0 * (self.q * (sd["side_K"][s] @ u[nodes])
                               - self.omega ** 2 * m * u[nodes] / c ** 2) / W
            g_out[self.slot(r, s2)] = g

    # ---- sweeps -------------------------------------------------------------
    def sweep(self, g_in, f, src, solver=None):
        """One DD cycle on every subdomain.  ``solver(l, b)`` solves the
        subdomain system (default: sparse LU).  Returns (g_out, [u_l])."""
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
        """Global nodal vector: average of the subdomain copies of each node."""
        acc = np.zeros(self.mesh.N, dtype=complex)
        cnt = np.zeros(self.mesh.N)
        for l, u in enumerate(us):
            idx = self.global_nodes(l)
            np.add.at(acc, idx, u)
            np.add.at(cnt, idx, 1.0)
        return acc / cnt

    def restrict(self, u_global):
        """Stacked subdomain copies of a global nodal vector."""
        return [np.asarray(u_global)[self.global_nodes(l)] for l in range(self.L)]


def gmres(matvec, rhs, tol, restart=50, max_iter=1000):
    """Restarted GMRES(m) from x0 = 0 with modified Gram-Schmidt and complex
    Givens rotations.  Stops when the recursive residual |g_{j+1}| <=
    tol * ||rhs||.  Returns (x, iterations, recursive relative residual,
    history of relative residuals)."""
    rhs = np.asarray(rhs, dtype=complex)
    n = rhs.size
    x = np.zeros(n, dtype=complex)
    bnorm = np.linalg.norm(rhs)
    if bnorm == 0.0:
        return x, 0, 0.0, []
    its, hist = 0, []
    r = rhs.copy()
    rel = 1.0
    while True:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n), dtype=complex)
        Hm = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=complex)
        gv = np.zeros(restart + 1, dtype=complex)
        gv[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = matvec(V[j])
            its += 1
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0.0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -np.conj(sn[i]) * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            a, bb = Hm[j, j], Hm[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            Hm[j, j] = cs[j] * a + sn[j] * bb
            Hm[j + 1, j] = 0.0
            gv[j + 1] = -np.conj(sn[j]) * gv[j]
            gv[j] = cs[j] * gv[j]
            rel = abs(gv[j + 1]) / bnorm
            hist.append(rel)
            k = j + 1
            if rel <= tol or its >= max_iter:
                break
        y = np.zeros(k, dtype=complex)
        for i in range(k - 1, -1, -1):
            y[i] = (gv[i] - Hm[i, i + 1:k] @ y[i + 1:k]) / Hm[i, i]
        x = x + V[:k].T @ y
        if rel <= tol or its >= max_iter:
            return x, its, rel, hist
        r = rhs - matvec(x)


def solve_dd(dec, f, g=None, tol=1e-8, restart=50, max_iter=1000, method="gmres",
             solver=None, refine=4, reduction=None):
    """Outer DD iteration on the interface unknowns; returns (u_stacked,
    info).  ``solver`` replaces the exact subdomain LU (e.g. WaveHoltz).

    The paper accelerates the interface iteration by a Krylov method
    (Sec. III, last paragraph).  Here GMRES runs inside an
    iterative-refinement loop driven by the true interface residual
        r = h - (I - T) G,    G <- G + d,   (I - T) d = r  by GMRES,
    repeated (at most ``refine`` extra passes) until ||r|| <= tol ||h||.
    Pass k asks GMRES for the relative reduction tol ||h|| / ||r_k|| (what
    is left to reach tol), or for ``reduction`` if that is larger (a pass
    limited to a fixed reduction, as a correction computed with a less
    accurate operator would be).  When the first pass already meets the
    tolerance this is plain GMRES from G = 0 (info["passes"] == 1)."""
    g0 = dec.embed_trace(g)
    mask = dec.interface_mask()
    h, _ = dec.sweep(g0, f, 1.0, solver)
    hnorm = np.linalg.norm(h)

    def T(G):
        out, _ = dec.sweep(G, f, 0.0, solver)
        return out

    G = np.zeros(dec.n_if, dtype=complex)
    hist = []
    its = 0
    if method == "gmres":
        r = h.copy()
        rel = 1.0 if hnorm > 0 else 0.0
        passes = 0
        for _ in range(1 + refine):
            if rel <= tol or its >= max_iter:
                break
            rnorm = np.linalg.norm(r)
            want = tol * hnorm / rnorm
            if reduction is not None:
                want = max(want, reduction)
            d, k, rr, hh = gmres(lambda v: v - T(v), r, want, restart, max_iter - its)
            passes += 1
            its += k
            hist += [x * rnorm / hnorm for x in hh]
            G = G + d
            r = h - (G - T(G))
            rel = np.linalg.norm(r) / hnorm
    elif method == "fixed":
        passes = 0
        rel = 1.0
        while its < max_iter:
            Gn = T(G) + h
            rel = np.linalg.norm(Gn - G) / hnorm if hnorm > 0 else 0.0
            G = Gn
            its += 1
            hist.append(rel)
            if rel <= tol:
                break
    else:
        raise ValueError(method)
    G = np.where(mask, G, 0.0)
    g_fin, us = dec.sweep(G + g0, f, 1.0, solver)
    true_rel = np.linalg.norm(g_fin - G) / hnorm if hnorm > 0 else 0.0
    return us, dict(iters=its, rel=rel, true_rel=true_rel, hist=hist, G=G, passes=passes)
