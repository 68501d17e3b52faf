"""Pins for the oracle's domain decomposition (paper Sec. III, eq. (2),
Algorithm 1's interface update) and outer GMRES."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dd, sem
from oracle import waveholtz as wh


def _c1():
    m = sem.Rect(16, 16, 2)
    X, Y = sem.node_coords(m)
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    return m, np.ones(m.N), 10.0, f


def test_single_subdomain_is_global_solve():
    m, c, om, f = _c1()
    dec = dd.Decomposition(m, dd.Partition(1, 1), c, om)
    assert not dec.interface_mask().any()
    _, us = dec.sweep(np.zeros(dec.n_if, complex), f, 1.0)
    u = sem.solve(m, c, om, f)
    assert np.linalg.norm(us[0] - u) < 1e-13 * np.linalg.norm(u)


def test_single_subdomain_with_boundary_data():
    m = sem.Rect(6, 5, 3)
    ue, g = sem.plane_wave(m, 8.0, 1.0, (0.6, 0.8))
    dec = dd.Decomposition(m, dd.Partition(1, 1), np.ones(m.N), 8.0)
    _, us = dec.sweep(dec.embed_trace(g), np.zeros(m.N), 1.0)
    u = sem.solve(m, np.ones(m.N), 8.0, np.zeros(m.N), g)
    assert np.linalg.norm(us[0] - u) < 1e-12 * np.linalg.norm(u)


@pytest.mark.parametrize("part", [(2, 2), (4, 2), (1, 4)])
def test_converged_dd_equals_global_lu(part):
    m, _, om, f = _c1()
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.3 * np.sin(4 * X + 1) * np.cos(3 * Y)
    dec = dd.Decomposition(m, dd.Partition(*part), c, om)
    us, info = dd.solve_dd(dec, f, tol=1e-12)
    u = sem.solve(m, c, om, f)
    ref = dec.restrict(u)
    err = np.linalg.norm(np.concatenate(us) - np.concatenate(ref)) / np.linalg.norm(np.concatenate(ref))
    assert err < 1e-10, (err, info["iters"])
    assert info["true_rel"] < 1e-10
    assert info["passes"] == 1   # plain GMRES from G = 0


def test_plane_wave_through_dd():
    m = sem.Rect(8, 8, 3)
    ue, g = sem.plane_wave(m, 12.0, 1.0, (np.cos(1.1), np.sin(1.1)))
    dec = dd.Decomposition(m, dd.Partition(2, 4), np.ones(m.N), 12.0)
    us, info = dd.solve_dd(dec, np.zeros(m.N), g, tol=1e-12)
    u = sem.solve(m, np.ones(m.N), 12.0, np.zeros(m.N), g)
    assert np.linalg.norm(dec.glue(us) - u) < 1e-10 * np.linalg.norm(u)
    assert np.linalg.norm(dec.glue(us) - ue) < 1e-3 * np.linalg.norm(ue)


def test_interface_sign_reading():
    """The printed +2ik update converges to a different problem; the -2ik
    reading converges to the global discrete solution (plant the printed
    sign in a copy of the oracle's exchange)."""
    m, c, om, f = _c1()

    class PrintedSign(dd.Decomposition):
        def exchange(self, l, u, g_in, g_out):
            sd = self.subs[l]
            for s in range(4):
                nb = self.neighbour(l, s)
                if nb is None:
                    continue
                r, s2 = nb
                nodes = self.local_sides[s]
                g_out[self.slot(r, s2)] = (-g_in[self.slot(l, s)]
                                           + 2j * (self.omega / sd["c"][nodes]) * u[nodes])

    u = sem.solve(m, c, om, f)
    bad = PrintedSign(m, dd.Partition(2, 2), c, om)
    us_bad, info = dd.solve_dd(bad, f, tol=1e-10, max_iter=400)
    err_bad = np.linalg.norm(bad.glue(us_bad) - u) / np.linalg.norm(u)
    assert err_bad > 1e-3


@pytest.mark.parametrize("n,P,sx,sy", [(4, 1, 2, 2), (6, 1, 3, 2), (6, 2, 3, 3)])
def test_null_modes_equal_interior_cross_points(n, P, sx, sy):
    """I - T is singular with one circulating mode per interior cross point:
    lambda is not unique, u is."""
    m = sem.Rect(n, n, P)
    dec = dd.Decomposition(m, dd.Partition(sx, sy), np.ones(m.N), 3.0)
    idx = np.where(dec.interface_mask())[0]
    T = np.zeros((idx.size, idx.size), complex)
    for k, i in enumerate(idx):
        e = np.zeros(dec.n_if, complex)
        e[i] = 1.0
        T[:, k] = dec.sweep(e, np.zeros(m.N), 0.0)[0][idx]
    ev = np.linalg.eigvals(T)
    assert np.sum(np.abs(ev - 1.0) < 1e-8) == (sx - 1) * (sy - 1)
    assert np.abs(ev).max() < 1.0 + 1e-10


def test_gmres_history_matches_scipy():
    """GMRES's residual after k steps is the minimum over the Krylov space,
    so the history must match scipy's GMRES on the same operator."""
    m, c, om, f = _c1()
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om)
    g0 = dec.embed_trace(None)
    h, _ = dec.sweep(g0, f, 1.0)

    def mv(v):
        return v - dec.sweep(v, f, 0.0)[0]
    x, its, rel, hist = dd.gmres(mv, h, 1e-10, restart=20, max_iter=200)
    op = spla.LinearOperator((dec.n_if, dec.n_if), matvec=mv, dtype=complex)
    sc = []
    xs, infoc = spla.gmres(op, h, rtol=1e-10, atol=0.0, restart=20, maxiter=20,
                           callback=lambda r: sc.append(r), callback_type="pr_norm")
    k = min(len(hist), len(sc), 25)
    assert np.allclose(hist[:k], sc[:k], rtol=1e-6, atol=1e-13)
    assert np.linalg.norm(mv(x) - h) <= 2e-10 * np.linalg.norm(h)


def test_fixed_point_outer_mode_decreases():
    m, c, om, f = _c1()
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om)
    us, info = dd.solve_dd(dec, f, tol=1e-8, method="fixed", max_iter=300)
    h = info["hist"]
    assert h[-1] < 0.05 * h[0]


def test_waveholtz_inner_dd_matches_exact_dd():
    m, c, om, f = _c1()
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om)
    us_ex, info_ex = dd.solve_dd(dec, f, tol=1e-8)
    us_wh, info_wh = dd.solve_dd(dec, f, tol=1e-8, solver=wh.make_solver(dec, tol=1e-12))
    a, b = np.concatenate(us_wh), np.concatenate(us_ex)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-9
    assert info_ex["iters"] == info_wh["iters"]


@pytest.mark.parametrize("reduction", [1e-2, 1e-3])
def test_refinement_passes_reach_global_lu(reduction):
    """The refinement loop of the outer iteration (Krylov acceleration of
    the interface iteration, Sec. III): passes limited to a fixed reduction
    must chain through the true residual r = h - (I - T) G and the rescaled
    tolerance to the global discrete solution.  A sign or scaling slip in
    either stalls the passes or converges elsewhere."""
    m, _, om, f = _c1()
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.3 * np.sin(4 * X + 1) * np.cos(3 * Y)
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om)
    us, info = dd.solve_dd(dec, f, tol=1e-12, refine=12, reduction=reduction)
    u = sem.solve(m, c, om, f)
    ref = np.concatenate(dec.restrict(u))
    err = np.linalg.norm(np.concatenate(us) - ref) / np.linalg.norm(ref)
    # each pass buys at least the fixed reduction, and not many times more
    need = int(np.ceil(np.log(1e-12) / np.log(reduction)))
    assert need <= info["passes"] <= need + 2, info["passes"]
    assert info["true_rel"] <= 1e-12
    assert err < 1e-10, err
    # the history is stated relative to ||h|| across passes; the last pass
    # asks for exactly what is left (tol ||h|| / ||r||), so it stops at the
    # first iterate below tol: an over- or under-scaled request would stop
    # later or earlier
    assert info["hist"][-1] <= 1e-12 < info["hist"][-2]


def test_refinement_first_pass_is_plain_gmres():
    """With no reduction limit the loop is one GMRES pass from G = 0: the
    same iterates and iteration count as calling GMRES directly."""
    m, c, om, f = _c1()
    dec = dd.Decomposition(m, dd.Partition(2, 2), c, om)
    us, info = dd.solve_dd(dec, f, tol=1e-10)
    h, _ = dec.sweep(dec.embed_trace(None), f, 1.0)
    G, its, _, _ = dd.gmres(lambda v: v - dec.sweep(v, f, 0.0)[0], h, 1e-10)
    assert info["passes"] == 1 and info["iters"] == its
    assert np.array_equal(info["G"], np.where(dec.interface_mask(), G, 0.0))


def test_pool_sweep_equals_serial_sweep():
    """The process-pool sweep assembles each output slot from the one
    subdomain that writes it: bit for bit the serial sweep, and the same
    outer solve."""
    from oracle import pool
    m, _, om, f = _c1()
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.3 * np.sin(4 * X + 1) * np.cos(3 * Y)
    part = dd.Partition(4, 2)
    dec = dd.Decomposition(m, part, c, om)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    with pool.ParallelDecomposition(m, part, c, om, workers=3) as pdec:
        a, ua = pdec.sweep(g, f, 1.0)
        b, ub = dec.sweep(g, f, 1.0)
        assert np.array_equal(a, b)
        assert all(np.array_equal(x, y) for x, y in zip(ua, ub))
        us1, i1 = dd.solve_dd(pdec, f, tol=1e-10)
        us2, i2 = dd.solve_dd(dec, f, tol=1e-10)
    assert i1["iters"] == i2["iters"]
    assert all(np.array_equal(x, y) for x, y in zip(us1, us2))
