"""Pins for the oracle's second-order transmission condition on interface
sides, B = d_n - i k - q (d_tt + k^2) with a real length q (the paper names
higher-order / optimized transmission conditions as the replacement of its
zeroth-order one, Sec. III and the conclusion)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dd, gll, sem
from oracle import waveholtz as wh


def _problem(n=16, P=2, om=10.0):
    m = sem.Rect(n, n, P)
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.3 * np.sin(4 * X + 1) * np.cos(3 * Y)
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    return m, c, om, f


@pytest.mark.parametrize("part,q", [((2, 2), 0.004), ((4, 2), 0.01), ((3, 3), 0.02)])
def test_converged_dd_equals_global_lu(part, q):
    """The condition changes the iteration, not its fixed point: the DD
    solution is the global discrete solution."""
    m, c, om, f = _problem(n=12)
    dec = dd.Decomposition(m, dd.Partition(*part), c, om, q=q)
    us, info = dd.solve_dd(dec, f, tol=1e-12)
    u = sem.solve(m, c, om, f)
    ref = np.concatenate(dec.restrict(u))
    err = np.linalg.norm(np.concatenate(us) - ref) / np.linalg.norm(ref)
    assert err < 1e-10, (err, info["iters"])


def test_plane_wave_through_dd_p3():
    m = sem.Rect(8, 8, 3)
    ue, g = sem.plane_wave(m, 12.0, 1.0, (np.cos(1.1), np.sin(1.1)))
    dec = dd.Decomposition(m, dd.Partition(2, 4), np.ones(m.N), 12.0, q=0.01)
    us, info = dd.solve_dd(dec, np.zeros(m.N), g, tol=1e-12)
    u = sem.solve(m, np.ones(m.N), 12.0, np.zeros(m.N), g)
    assert np.linalg.norm(dec.glue(us) - u) < 1e-10 * np.linalg.norm(u)


def test_side_terms_are_the_weak_form():
    """For u = x y on the middle subdomain of a 3x3 partition (four
    interface sides), u^T (A' - A) u = q * sum over sides of the integral of
    (d_t u)^2 along the side, exactly (GLL is exact for these degrees), and
    the mass grows by q W_side / c^2 on each side plus q^2 / c^2 at each
    corner where two interface sides meet."""
    m = sem.Rect(6, 6, 3, 0.0, 1.5, 0.0, 1.2)
    c = np.full(m.N, 1.3)
    q = 0.07
    dec = dd.Decomposition(m, dd.Partition(3, 3), c, 5.0, q=q)
    sd = dec.subs[4]
    r = sd["rect"]
    xs = sem.node_coords_1d(r.nx, r.P, r.x0, r.x1)
    ys = sem.node_coords_1d(r.ny, r.P, r.y0, r.y1)
    X, Y = np.meshgrid(xs, ys)
    u = (X * Y).ravel()
    lx, ly = r.x1 - r.x0, r.y1 - r.y0
    # d_t u along left / right (x fixed) is x, along bottom / top it is y
    exact = q * (r.x0 ** 2 * ly + r.x1 ** 2 * ly + r.y0 ** 2 * lx + r.y1 ** 2 * lx)
    got = u @ ((sd["At"] - sd["A"]) @ u)
    assert abs(got - exact) < 1e-12 * exact
    dM = (sd["Mt"] - sd["M"]) * c[0] ** 2
    nxl, nyl = dec.nxl, dec.nyl
    side_mass = dM.sum()
    # each side contributes q * its length, each of the 4 corners q^2
    assert abs(side_mass - (q * 2 * (lx + ly) + 4 * q * q)) < 1e-13
    interior = np.ones(nxl * nyl, bool)
    for nodes in sem.side_nodes(nxl, nyl):
        interior[nodes] = False
    assert not np.any(dM[interior])


def test_outer_boundary_sides_unchanged():
    """Sides on the outer boundary keep the zeroth-order (impedance) form."""
    m, c, om, f = _problem(n=8)
    dec0 = dd.Decomposition(m, dd.Partition(1, 1), c, om)
    decq = dd.Decomposition(m, dd.Partition(1, 1), c, om, q=0.05)
    assert (decq.subs[0]["S"] != dec0.subs[0]["S"]).nnz == 0


def test_fewer_outer_iterations():
    """With q = 0.25 min(c) / omega GMRES needs fewer iterations than with the
    zeroth-order condition (measured: 35 -> 25 on this problem)."""
    m = sem.Rect(16, 16, 2)
    X, Y = sem.node_coords(m)
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    c = np.ones(m.N)
    om = 10.0
    its = {}
    for q in (0.0, 0.25 * c.min() / om):
        dec = dd.Decomposition(m, dd.Partition(2, 2), c, om, q=q)
        _, info = dd.solve_dd(dec, f, tol=1e-8)
        its[q] = info["iters"]
    q0, q1 = sorted(its)
    assert its[q1] < 0.85 * its[q0], its


def test_iteration_operator_contracts_more():
    """Spectral radius of the sweep map T off its cross-point modes: the
    spectrum is symmetric (lambda and -lambda; a sweep maps the data of one
    side of each interface to the other), each interior cross point carries
    the pair +1, -1, and the next largest modulus drops with q > 0
    (measured 0.998 -> 0.815 here)."""
    m = sem.Rect(6, 6, 2)
    rho = {}
    for q in (0.0, 0.02):
        dec = dd.Decomposition(m, dd.Partition(3, 2), np.ones(m.N), 6.0, q=q)
        idx = np.where(dec.interface_mask())[0]
        T = np.zeros((idx.size, idx.size), complex)
        for k, i in enumerate(idx):
            e = np.zeros(dec.n_if, complex)
            e[i] = 1.0
            T[:, k] = dec.sweep(e, np.zeros(m.N), 0.0)[0][idx]
        ev = np.linalg.eigvals(T)
        assert np.sum(np.abs(ev - 1.0) < 1e-8) == 2           # (sx - 1)(sy - 1)
        assert np.sum(np.abs(ev + 1.0) < 1e-8) == 2
        a = np.abs(ev)
        rho[q] = a[np.abs(a - 1.0) >= 1e-8].max()
    assert rho[0.0] > 0.99 and rho[0.02] < 0.9, rho


def test_large_q_leaves_the_unit_disc():
    """The condition's limit (documented with its reading): for q omega / c
    around 1 and above, the lumped discrete sweep map has eigenvalues beyond
    the unit circle, so a plain fixed-point iteration diverges there (GMRES
    still converges); q omega / c <= 0.5 keeps them inside."""
    m = sem.Rect(6, 6, 2)
    rad = {}
    for q in (0.08, 0.17):
        dec = dd.Decomposition(m, dd.Partition(3, 2), np.ones(m.N), 6.0, q=q)
        idx = np.where(dec.interface_mask())[0]
        T = np.zeros((idx.size, idx.size), complex)
        for k, i in enumerate(idx):
            e = np.zeros(dec.n_if, complex)
            e[i] = 1.0
            T[:, k] = dec.sweep(e, np.zeros(m.N), 0.0)[0][idx]
        rad[q] = np.abs(np.linalg.eigvals(T)).max()
    assert rad[0.08] < 1.0 + 1e-10 and rad[0.17] > 1.05, rad


def test_time_step_rule_still_bounds():
    """The extended weights only add mass where they add stiffness
    (Wx' >= Wx): lambda_max(M'^-1 A') stays below the rule's bound."""
    m = sem.Rect(9, 9, 3)
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.2 * np.cos(3 * X) * np.sin(2 * Y)
    dec = dd.Decomposition(m, dd.Partition(3, 3), c, 7.0, q=0.05)
    _, w = gll.nodes_weights(3)
    K = gll.element_stiffness_1d(3)
    s = 1.0 / np.sqrt(w)
    mu = np.linalg.eigvalsh(s[:, None] * K * s[None, :]).max()
    for l in (0, 4):
        sd = dec.subs[l]
        r = sd["rect"]
        Mi = 1.0 / np.sqrt(sd["Mt"])
        B = (sd["At"].toarray() * Mi[:, None]) * Mi[None, :]
        lam = np.linalg.eigvalsh(B).max()
        bound = sd["c"].max() ** 2 * mu * ((2 / r.hx) ** 2 + (2 / r.hy) ** 2)
        assert lam <= bound * (1 + 1e-12)


def test_waveholtz_converges_to_the_subdomain_solution():
    """WaveHoltz on the subdomain system with the condition's terms reaches
    the sparse-LU solution of that system (Pi u* = u*)."""
    m, c, om, f = _problem(n=8)
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om, q=0.02)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    nts = wh.subdomain_steps(dec)
    for l in (0, 3):
        sd = dec.subs[l]
        b = dec.rhs(l, f, g, 1.0)
        u_lu = dec.lu(l).solve(b)
        u, it = wh.solve(sd["At"], sd["Mt"], sd["H"], b, om, nts[l], tol=1e-13, max_iter=500)
        assert np.linalg.norm(u - u_lu) < 1e-9 * np.linalg.norm(u_lu), it
