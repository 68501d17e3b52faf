"""Seeded synthetic workload generators (inputs only, no method arithmetic).

Both the oracle and the GPU path read their inputs from here; nothing else is
shared between them.  A workload names a mesh (element grid, degree,
rectangle), a subdomain grid, omega, tolerances, and *callables* for the
wavespeed c(x, y) and the source f(x, y).  Each side samples those callables
at the node coordinates it computes itself.

The paper benchmarks on synthetic problems only (constant c on [-1,1]^d,
uniform meshes, random input vectors; a Y-shaped waveguide with 3x contrast
and an off-centre point source for its illustration).  The generators below
follow those shapes:

* ``c1``  unit square, 16x16 elements, P=2, c=1, omega=10, Gaussian source
          (sigma 0.05) at (0.3, 0.6), 2x2 subdomains, impedance outer boundary.
* ``c2``  unit square, 256x256 elements, P=3, 16x16 subdomains of 16x16
          elements, Y-waveguide with a slow core c=1/3 in background c=1,
          omega for 10 points per wavelength in the core, off-centre source.
* ``c2_t1`` the ``c2`` problem on 32x32 subdomains of 8x8 elements (625 nodes,
          one node per thread fits a workgroup).
* ``c3``  512x512 elements, P=3, 8x8 subdomains of 64x64 elements, same
          physical problem as ``c2``.
* ``c4``  a seeded batch of independent problems whose subdomains (8..64
          elements per side, P in 1..4) total 400, log-normal smooth
          wavespeed with contrast up to 3, omega=40.
* ``c5``  a seeded Poisson-arrival stream of independent solves.

Box (3D) workloads, the paper's second benchmark family (constant c on
[-1,1]^3, uniform hexahedra, 16^3 to 128^3 elements, degree up to 3):

* ``c6``     64^3 elements, P=3, 32^3 subdomains of 2^3 elements (343 nodes),
             c=1, omega for 10 points per wavelength, Gaussian source.
* ``c6_p1``  128^3 elements, P=1, 16^3 subdomains of 8^3 elements (729 nodes).
* ``c6_small`` 8^3 elements, P=3, 4^3 subdomains of 2^3 elements: the ``c6``
             subdomain shape at a size the oracle finishes in seconds.
* ``c6_tiny`` 4^3 elements, P=2, 2^3 subdomains (the smoke check).
"""
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    P: int
    sx: int
    sy: int
    omega: float
    c: Callable
    f: Callable
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    g: Optional[Callable] = None   # boundary trace generator, None = 0
    tol: float = 1e-8
    tau_in: float = 1e-12
    meta: dict = field(default_factory=dict)


def gaussian(x0, y0, sigma, amp=1.0):
    """Unit-amplitude Gaussian point source exp(-|x - x0|^2 / (2 sigma^2))."""
    def f(X, Y):
        return amp * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2.0 * sigma ** 2))
    return f


def constant(val):
    def c(X, Y):
        return np.full(np.broadcast(X, Y).shape, float(val))
    return c


def _seg_dist(X, Y, a, b):
    ax, ay = a
    bx, by = b
    dx, dy = bx - ax, by - ay
    t = np.clip(((X - ax) * dx + (Y - ay) * dy) / (dx * dx + dy * dy), 0.0, 1.0)
    return np.hypot(X - (ax + t * dx), Y - (ay + t * dy))


def y_waveguide(seed=2, c_bg=1.0, c_core=1.0 / 3.0, width=0.03, delta=1.0 / 256):
    """Y-shaped waveguide: a stem from (0.5, 0) to a junction near (0.5, 0.4)
    and two arms to near (0.2, 1) and (0.8, 1); tanh-smoothed edges so the
    pointwise value at any node is well defined.  The seed jitters the
    junction height and the arm end points by U(-0.05, 0.05)."""
    rng = np.random.default_rng(seed)
    jy = 0.4 + rng.uniform(-0.05, 0.05)
    lx = 0.2 + rng.uniform(-0.05, 0.05)
    rx = 0.8 + rng.uniform(-0.05, 0.05)
    segs = [((0.5, 0.0), (0.5, jy)), ((0.5, jy), (lx, 1.0)), ((0.5, jy), (rx, 1.0))]

    def c(X, Y):
        d = np.minimum.reduce([_seg_dist(X, Y, a, b) for a, b in segs])
        return c_bg + (c_core - c_bg) * 0.5 * (1.0 - np.tanh((d - width) / delta))
    c.segments = segs
    return c


def lognormal_field(seed, n_modes=32, kmax=4, contrast=3.0):
    """Smooth 1-periodic random wavespeed: log c = (ln contrast / 2) G / max|G|,
    G = sum_j a_j cos(2 pi k_j . x + phi_j), integer k_j with
    1 <= |k_j|_inf <= kmax, a_j ~ N(0, 1/|k_j|^2), phi_j ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=2)
        if np.abs(k).max() >= 1:
            ks.append(k)
    ks = np.array(ks, dtype=float)
    amp = rng.normal(0.0, 1.0, n_modes) / np.linalg.norm(ks, axis=1)
    ph = rng.uniform(0.0, 2 * np.pi, n_modes)

    def G(X, Y):
        X = np.asarray(X, dtype=float)
        Y = np.asarray(Y, dtype=float)
        out = np.zeros(np.broadcast(X, Y).shape)
        for (kx, ky), a, p in zip(ks, amp, ph):
            out += a * np.cos(2 * np.pi * (kx * X + ky * Y) + p)
        return out
    # max |G| on a 257^2 grid, computed when the field is first sampled (a
    # request stream draws many fields and samples few of them)
    scale = []

    def c(X, Y):
        if not scale:
            g = np.linspace(0.0, 1.0, 257)
            GX, GY = np.meshgrid(g, g)
            scale.append(0.5 * np.log(contrast) / np.abs(G(GX, GY)).max())
        return np.exp(scale[0] * G(X, Y))
    c.cmin = float(np.exp(-0.5 * np.log(contrast)))
    return c


def _omega_ppw(P, h, c_min, ppw):
    """omega giving ``ppw`` nodes per wavelength at speed c_min."""
    return 2 * np.pi * c_min * P / (ppw * h)


def c1():
    return Workload("c1", 16, 16, 2, 2, 2, 10.0, constant(1.0), gaussian(0.3, 0.6, 0.05),
                    tol=1e-8, tau_in=1e-12)


def c2(seed=2):
    om = _omega_ppw(3, 1.0 / 256, 1.0 / 3.0, 10.0)
    return Workload("c2", 256, 256, 3, 16, 16, om, y_waveguide(seed),
                    gaussian(0.51, 0.15, 0.01), tol=1e-8, tau_in=1e-12)


def c2_small(seed=2):
    """The c2 problem scaled to 64x64 elements (4x4 subdomains of 16x16):
    same wavespeed and source functions, omega for 10 points per wavelength
    in the core at this resolution.  Sized so the oracle finishes in
    seconds while keeping c2's subdomain shape."""
    om = _omega_ppw(3, 1.0 / 64, 1.0 / 3.0, 10.0)
    return Workload("c2_small", 64, 64, 3, 4, 4, om, y_waveguide(seed),
                    gaussian(0.51, 0.15, 0.01), tol=1e-8, tau_in=1e-12)


def c2_t1(seed=2):
    """The c2 problem partitioned into 32x32 subdomains of 8x8 elements
    (625 nodes each), small enough for one node per thread."""
    wl = c2(seed)
    wl.name, wl.sx, wl.sy = "c2_t1", 32, 32
    return wl


def c3(seed=2):
    om = _omega_ppw(3, 1.0 / 256, 1.0 / 3.0, 10.0)
    return Workload("c3", 512, 512, 3, 8, 8, om, y_waveguide(seed),
                    gaussian(0.51, 0.15, 0.01), tol=1e-8, tau_in=1e-12)


def c4(seed=4, total=400):
    """Independent conforming problems sharing one wavespeed field, drawn
    until their subdomains total ``total``; the last grid is truncated."""
    rng = np.random.default_rng(seed)
    c = lognormal_field(seed)
    omega = 40.0
    probs, count = [], 0
    while count < total:
        P = int(rng.integers(1, 5))
        s = int(rng.integers(8, 65))
        gx, gy = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        if count + gx * gy > total:
            gx, gy = min(total - count, 4), 1
        h = P * 2 * np.pi * c.cmin / (10.0 * omega)
        ox, oy = rng.uniform(0.0, 1.0, 2)
        W, H = gx * s * h, gy * s * h
        sxp, syp = ox + rng.uniform(0.2, 0.8) * W, oy + rng.uniform(0.2, 0.8) * H
        probs.append(Workload(f"c4_{len(probs)}", gx * s, gy * s, P, gx, gy, omega, c,
                              gaussian(sxp, syp, 3 * h), ox, ox + W, oy, oy + H,
                              tol=1e-6, tau_in=1e-5))
        count += gx * gy
    return probs


def c5(seed=5, n_requests=2000):
    """Independent requests on the unit square with their own meshes,
    frequencies, wavespeeds (log-normal field times 0-2 waveguides) and 1-4
    Gaussian sources; (n, P) resampled until >= 8 points per wavelength at
    the slowest speed."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_requests):
        omega = float(rng.uniform(10.0, 80.0))
        base = lognormal_field(int(rng.integers(1 << 30)))
        n_guides = int(rng.integers(0, 3))
        cores = []
        for _ in range(n_guides):
            cores.append(float(rng.uniform(1.0 / 3.0, 0.5)))
        guides = [y_waveguide(int(rng.integers(1 << 30)), c_bg=1.0, c_core=cg) for cg in cores]
        cmin = base.cmin * (min(cores) if cores else 1.0)
        for _ in range(1000):
            P = int(rng.integers(2, 5))
            s = int(rng.choice(np.arange(16, 65, 8)))
            g = int(rng.integers(-(-64 // s), 512 // s + 1))
            n = s * g
            if 2 * np.pi * cmin / omega * n * P >= 8.0:
                break
        nsrc = int(rng.integers(1, 5))
        h = 1.0 / n
        srcs = [gaussian(*rng.uniform(0.1, 0.9, 2), max(0.01, 3 * h)) for _ in range(nsrc)]

        def c_fn(X, Y, base=base, guides=guides):
            out = base(X, Y)
            for gd in guides:
                out = out * gd(X, Y)
            return out

        def f_fn(X, Y, srcs=srcs):
            return sum(s_(X, Y) for s_ in srcs)
        reqs.append(Workload(f"c5_{r}", n, n, P, g, g, omega, c_fn, f_fn, tol=1e-6,
                             tau_in=1e-5))
    return reqs


CONFIGS = {"c1": c1, "c2": c2, "c2_small": c2_small, "c2_t1": c2_t1, "c3": c3}


@dataclass
class Workload3:
    name: str
    nx: int
    ny: int
    nz: int
    P: int
    sx: int
    sy: int
    sz: int
    omega: float
    c: Callable            # c(X, Y, Z)
    f: Callable            # f(X, Y, Z)
    box: tuple = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def constant3(val):
    def c(X, Y, Z):
        return np.full(np.shape(X), float(val))
    return c


def gaussian3(x0, y0, z0, sigma):
    def f(X, Y, Z):
        return np.exp(-((X - x0) ** 2 + (Y - y0) ** 2 + (Z - z0) ** 2) / (2 * sigma ** 2))
    return f


def _box(name, n, P, sub):
    om = _omega_ppw(P, 2.0 / n, 1.0, 10.0)
    return Workload3(name, n, n, n, P, n // sub, n // sub, n // sub, om, constant3(1.0),
                     gaussian3(0.1, -0.2, 0.15, 0.1))


def c6():
    return _box("c6", 64, 3, 2)


def c6_p1():
    return _box("c6_p1", 128, 1, 8)


def c6_small():
    return _box("c6_small", 8, 3, 2)


def c6_tiny():
    """4^3 elements, P=2, 2^3 subdomains of 2^3 elements: a box problem whose
    global LU takes milliseconds."""
    return _box("c6_tiny", 4, 2, 2)


CONFIGS3 = {"c6": c6, "c6_p1": c6_p1, "c6_small": c6_small, "c6_tiny": c6_tiny}
