"""Pins for the 3D oracle (the paper's hexahedral workload, Sec. VII-B):
assembly, conservation sums, the global solve, the decomposition and
WaveHoltz on a box."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dd, dd3, gll, sem3
from oracle import waveholtz as wh


def test_p1_is_seven_point_laplacian():
    """Cube elements of side h at P = 1: A = h (T (x) I (x) I + I (x) T (x) I
    + I (x) I (x) T) with T = tridiag(-1, 2, -1) (end rows halved) and
    I = diag(1/2, 1, ..., 1, 1/2) (trapezoidal weights)."""
    n = 4
    m = sem3.Box(n, n, n, 1, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
    A, _, _, _, _ = sem3.operators(m)
    T = sp.diags([-np.ones(n), 2 * np.ones(n + 1), -np.ones(n)], [-1, 0, 1]).tolil()
    T[0, 0] = T[n, n] = 1.0
    I = sp.diags(np.r_[0.5, np.ones(n - 1), 0.5])
    ref = (sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I)))
    assert abs(A - ref / n).max() < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3])
def test_constants_and_sums(P):
    """A annihilates constants and is symmetric; the lumped mass sums to the
    volume over c^2 and the boundary mass to the surface area over c."""
    m = sem3.Box(2, 3, 2, P, -1.0, 1.0, 0.0, 0.5, 0.2, 1.0)
    c = np.full(m.N, 1.7)
    S, A, M, H = sem3.system(m, c, 3.0)
    assert np.abs(A @ np.ones(m.N)).max() < 1e-12
    assert abs(A - A.T).max() < 1e-13
    lx, ly, lz = 2.0, 0.5, 0.8
    assert abs(M.sum() - lx * ly * lz / 1.7 ** 2) < 1e-13
    assert abs(H.sum() - 2 * (lx * ly + lx * lz + ly * lz) / 1.7) < 1e-13


def test_gradient_energy_exact():
    """u^T A u is the exact integral of |grad u|^2 for a polynomial of degree
    <= P per direction (GLL integrates the products exactly)."""
    m = sem3.Box(2, 2, 3, 2, 0.0, 1.0, 0.0, 2.0, 0.0, 1.5)
    X, Y, Z = sem3.node_coords(m)
    u = X * Y + Z ** 2
    A, _, _, _, _ = sem3.operators(m)
    # grad u = (y, x, 2z): integral over [0,1]x[0,2]x[0,1.5]
    exact = (8.0 / 3.0) * 1.5 + (1.0 / 3.0) * 2.0 * 1.5 + 4.0 * (1.5 ** 3 / 3.0) * 2.0
    assert abs(u @ (A @ u) - exact) < 1e-11 * exact


def test_plane_wave_converges():
    """Global solve with plane-wave impedance data: the nodal error drops
    under refinement at fixed omega (P = 2)."""
    om = 4.0
    d = np.array([0.48, 0.6, 0.64])
    errs = []
    for n in (2, 4, 8):
        m = sem3.Box(n, n, n, 2, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0)
        ue, g = sem3.plane_wave(m, om, 1.0, d)
        u = sem3.solve(m, np.ones(m.N), om, np.zeros(m.N), g)
        errs.append(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4, errs


@pytest.mark.parametrize("part", [(2, 2, 2), (3, 1, 2)])
def test_converged_dd_equals_global_lu(part):
    m = sem3.Box(6, 4, 4, 2)
    X, Y, Z = sem3.node_coords(m)
    c = 1.0 + 0.2 * np.sin(2 * X) * np.cos(Y + Z)
    f = np.exp(-((X - 0.2) ** 2 + (Y + 0.3) ** 2 + Z ** 2) / 0.1)
    dec = dd3.Decomposition3(m, dd3.Partition3(*part), c, 5.0)
    us, info = dd.solve_dd(dec, f, tol=1e-12)
    u = sem3.solve(m, c, 5.0, f)
    ref = np.concatenate(dec.restrict(u))
    err = np.linalg.norm(np.concatenate(us) - ref) / np.linalg.norm(ref)
    assert err < 1e-10, (err, info["iters"])


def test_waveholtz_on_a_box_subdomain():
    """WaveHoltz (with the box's time-step rule) reaches the sparse-LU
    solution of a subdomain system (Pi u* = u*)."""
    m = sem3.Box(4, 4, 2, 2)
    X, Y, Z = sem3.node_coords(m)
    c = 1.0 + 0.1 * X * Y
    dec = dd3.Decomposition3(m, dd3.Partition3(2, 2, 1), c, 4.0)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    f = np.exp(-(X ** 2 + Y ** 2 + Z ** 2))
    nts = wh.subdomain_steps(dec)
    sd = dec.subs[1]
    b = dec.rhs(1, f, g, 1.0)
    u, it = wh.solve(sd["A"], sd["M"], sd["H"], b, 4.0, nts[1], tol=1e-13, max_iter=500)
    u_lu = dec.lu(1).solve(b)
    assert np.linalg.norm(u - u_lu) < 1e-9 * np.linalg.norm(u_lu), it


def test_time_step_rule_bounds_the_box_spectrum():
    m = sem3.Box(2, 2, 2, 3, 0.0, 1.0, 0.0, 0.8, 0.0, 1.2)
    X, Y, Z = sem3.node_coords(m)
    c = 1.0 + 0.3 * np.cos(3 * X) * Y
    S, A, M, H = sem3.system(m, c, 5.0)
    Mi = 1.0 / np.sqrt(M)
    lam = np.linalg.eigvalsh((A.toarray() * Mi[:, None]) * Mi[None, :]).max()
    _, w = gll.nodes_weights(3)
    K = gll.element_stiffness_1d(3)
    s = 1.0 / np.sqrt(w)
    mu = np.linalg.eigvalsh(s[:, None] * K * s[None, :]).max()
    bound = c.max() ** 2 * mu * ((2 / m.hx) ** 2 + (2 / m.hy) ** 2 + (2 / m.hz) ** 2)
    assert lam <= bound * (1 + 1e-12)
    nt = wh.time_steps3(3, m.hx, m.hy, m.hz, c.max(), 5.0)
    sigma = np.sin(np.pi / nt) / 2.5
    assert sigma ** 2 * lam < 4.0
