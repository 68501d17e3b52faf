"""Pins for the oracle's WaveHoltz solver (paper Sec. V): filter identities,
the exactness claim of the modified leapfrog, the fixed point, the sign and
scale readings of eq. (7) against Algorithm 1, and the time-step rule."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dd, sem
from oracle import waveholtz as wh


@pytest.mark.parametrize("N", [3, 4, 5, 7, 16, 68, 101])
def test_filter_identities(N):
    """(2/N) sum kappa_nu cos(2 pi nu/N) = 1 and sum kappa_nu sin = 0, on the
    integer and the half-integer grids: the filter passes the omega mode."""
    kap, kaph, cs, sn = wh.filter_tables(N)
    nu = np.arange(N)
    assert abs(2.0 / N * np.dot(kap, cs) - 1.0) < 1e-13
    assert abs(np.dot(kap, sn)) < 1e-12
    ch = np.cos(2 * np.pi * (nu + 0.5) / N)
    shh = np.sin(2 * np.pi * (nu + 0.5) / N)
    assert abs(2.0 / N * np.dot(kaph, ch) - 1.0) < 1e-13
    assert abs(np.dot(kaph, shh)) < 1e-12


def _subproblem(P=2, n=6, omega=9.0, seed=0):
    m = sem.Rect(n, n, P)
    rng = np.random.default_rng(seed)
    X, Y = sem.node_coords(m)
    c = 1.0 + 0.4 * np.sin(3 * X) * np.cos(2 * Y)
    S, A, M, H = sem.system(m, c, omega)
    b = rng.standard_normal(m.N) + 1j * rng.standard_normal(m.N)
    u = spla.splu(S).solve(b)
    Nt = wh.time_steps(P, m.hx, m.hy, c.max(), omega)
    return A, M, H, b, u, Nt, omega


def test_leapfrog_trajectory_is_exact():
    """Started from the discrete solution, p^nu = Re{u e^{-2 pi i nu/N_t}}
    at every step (the exactness claim after the leapfrog scheme)."""
    A, M, H, b, u, Nt, om = _subproblem()
    traj = wh.trajectory(A, M, H, b, om, Nt, u)
    nu = np.arange(Nt)
    ref = (u[None, :] * np.exp(-2j * np.pi * nu / Nt)[:, None]).real
    assert np.abs(traj - ref).max() < 1e-11 * np.abs(u).max()


def test_fixed_point_is_the_helmholtz_solution():
    A, M, H, b, u, Nt, om = _subproblem()
    pu = wh.iterate(A, M, H, b, om, Nt, u)
    assert np.linalg.norm(pu - u) / np.linalg.norm(u) < 1e-13
    # independent of the number of steps
    pu2 = wh.iterate(A, M, H, b, om, Nt + 3, u)
    assert np.linalg.norm(pu2 - u) / np.linalg.norm(u) < 1e-13


def test_sign_and_scale_readings():
    """Algorithm 1's sign of the pdot term maps u* to conj-like garbage and
    its missing 2/N_t rescales the iterate; eq. (7) as read here does not."""
    A, M, H, b, u, Nt, om = _subproblem()
    kap, kaph, cs, sn = wh.filter_tables(Nt)
    sigma, alpha, beta = wh.leapfrog_coeffs(M, H, om, Nt)
    p = u.real.copy()
    pd = (-1j * om * u * np.exp(-1j * np.pi / Nt)).real
    v = kap[0] * p + kaph[0] * pd / (1j * om)      # Algorithm 1's sign
    for nu in range(1, Nt):
        p = p + sigma * pd
        pd = alpha * pd + beta * (-(A @ p) + b.real * cs[nu] + b.imag * sn[nu])
        v = v + kap[nu] * p + kaph[nu] * pd / (1j * om)
    assert np.linalg.norm(2.0 / Nt * v - np.conj(u)) / np.linalg.norm(u) < 1e-12
    assert np.linalg.norm(v - u) / np.linalg.norm(u) > 0.5


def test_iteration_converges_to_lu():
    A, M, H, b, u, Nt, om = _subproblem()
    uw, it = wh.solve(A, M, H, b, om, Nt, tol=1e-12, max_iter=200)
    assert it < 200
    assert np.linalg.norm(uw - u) / np.linalg.norm(u) < 1e-9


def test_time_step_rule_bound_is_sharp():
    """lambda_max(M^-1 A) equals c^2 (mu_x + mu_y) for constant c, so the
    rule sits exactly at the leapfrog stability limit (times the safety)."""
    for P in (1, 2, 3, 4):
        m = sem.Rect(3, 2, P, 0.0, 0.6, 0.0, 0.5)
        c = np.full(m.N, 1.7)
        _, A, M, _ = sem.system(m, c, 1.0)
        lam = np.linalg.eigvals(np.diag(1 / M) @ A.toarray()).real.max()
        # N_t with safety 1 is the smallest N with sin(pi/N) < omega/sqrt(lam)
        om = 3.0
        N = wh.time_steps(P, m.hx, m.hy, 1.7, om, safety=1.0)
        assert np.sin(np.pi / N) <= om / np.sqrt(lam) * (1 + 1e-12)
        assert N == 4 or np.sin(np.pi / (N - 1)) > om / np.sqrt(lam) * (1 - 1e-12)


def test_time_step_rule_is_stable_and_tight():
    """Undamped scheme (H = 0): bounded over many periods at the rule's N_t,
    exponential growth 10% beyond the limit."""
    P, n, om = 3, 4, 5.0
    m = sem.Rect(n, n, P)
    c = np.ones(m.N)
    _, A, M, _ = sem.system(m, c, om)
    H = np.zeros(m.N)
    rng = np.random.default_rng(0)

    def run(Nt, periods=30):
        sigma, alpha, beta = wh.leapfrog_coeffs(M, H, om, Nt)
        p = rng.standard_normal(m.N)
        pd = np.zeros(m.N)
        n0 = np.linalg.norm(p)
        for _ in range(periods * Nt):
            pd = alpha * pd - beta * (A @ p)
            p = p + sigma * pd
        return np.linalg.norm(p) / n0

    Nt = wh.time_steps(P, m.hx, m.hy, 1.0, om)
    assert run(Nt) < 10.0
    # a step 10% over the stability limit blows up
    lam = np.linalg.eigvals(np.diag(1 / M) @ A.toarray()).real.max()
    Nbad = int(np.floor(np.pi / np.arcsin(min(1.0, 1.1 * om / np.sqrt(lam)))))
    with np.errstate(over="ignore", invalid="ignore"):
        grow = run(Nbad)
    assert not np.isfinite(grow) or grow > 1e6


def test_subdomain_wave_holtz_counts_c1():
    """C1's subdomains converge to 1e-12 in well under the 100-iteration cap
    (the paper reports five to twenty at its sizes)."""
    m = sem.Rect(16, 16, 2)
    X, Y = sem.node_coords(m)
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    dec = dd.Decomposition(m, dd.Partition(2, 2), np.ones(m.N), 10.0)
    counts = []
    solver = wh.make_solver(dec, tol=1e-12, max_iter=100, counts=counts)
    g, us = dec.sweep(np.zeros(dec.n_if, complex), f, 1.0, solver)
    g2, us2 = dec.sweep(np.zeros(dec.n_if, complex), f, 1.0)
    assert max(counts) < 100
    for a, b_ in zip(us, us2):
        assert np.linalg.norm(a - b_) <= 1e-9 * np.linalg.norm(b_) + 1e-30
