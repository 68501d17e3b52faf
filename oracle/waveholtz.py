"""WaveHoltz subdomain solver (paper Sec. V, eqs. (6)-(7), the modified
leapfrog scheme, and the WaveHoltz loop of Algorithm 1).

Given the lumped system (A - i omega H - omega^2 M) u = b, WaveHoltz evolves
the real wave equation  M p'' + H p' + A p = Re{b e^{-i omega t}}  (eq. (6))
over one period T = 2 pi / omega with N_t steps and replaces u by the filtered
time average (eq. (7)):
    u <- (2/N_t) sum_{nu=0}^{N_t-1} ( kappa_nu p^nu
                                       + (i/omega) kappa_{nu+1/2} pdot^{nu+1/2} ),
    kappa_s = cos(2 pi s / N_t) - 1/4 + 1/4 tan^2(pi / N_t),  s in {nu, nu+1/2}.
Readings:
* the pdot term enters with +i/omega = -1/(i omega), the sign of eq. (7)
  (Algorithm 1 prints the opposite sign, which converges to conj(u));
* the factor 2/N_t of eq. (7) is applied when the new iterate is formed
  (Algorithm 1 omits it);
* time levels are t_nu = nu * dt with dt = 2 pi / (omega N_t), so
  omega t_nu = 2 pi nu / N_t (consistent with the forcing phase of the
  leapfrog scheme and the initial half step);
* the same kappa formula is evaluated at half-integer arguments.
Leapfrog (per component j), theta = tan(omega dt/2)/omega,
sigma = sin(omega dt/2)/(omega/2):
    pdot^{nu+1/2} = alpha_j pdot^{nu-1/2} + beta_j (-(A p^nu)_j + Re{b_j e^{-2 pi i nu/N_t}}),
    p^{nu+1}      = p^nu + sigma pdot^{nu+1/2},
    alpha_j = (M_jj - theta H_jj)/(M_jj + theta H_jj),  beta_j = sigma/(M_jj + theta H_jj).
Initial state of each iteration: p^0 = Re u, pdot^{1/2} = Re{-i omega u e^{-i pi/N_t}}.
"""
import numpy as np

from . import gll


def time_steps(P, hx, hy, cmax, omega, safety=0.9):
    """Number of leapfrog steps per period.

    The scheme is leapfrog with step sigma; undamped it reads
    p^{n+1} - 2 p^n + p^{n-1} = -sigma^2 M^-1 A p^n, stable iff
    sigma^2 lambda_max(M^-1 A) < 4.  With sigma = 2 sin(pi/N_t)/omega this is
    sin(pi/N_t) < omega / sqrt(lambda_max).  For the Kronecker-sum stiffness
    lambda_max(M^-1 A) <= cmax^2 (mu_x + mu_y), mu = (2/h)^2 mu_hat where
    mu_hat is the largest eigenvalue of the reference element pencil
    (D^T W D, W) (equality for constant c).  The paper's rule
    dt <= 2h/(P^2 c_max) is looser than this bound, so the bound is used:
        N_t = max(4, ceil(pi / arcsin(safety * omega / sqrt(lambda_bar)))).
    """
    _, w = gll.nodes_weights(P)
    K = gll.element_stiffness_1d(P)
    s = 1.0 / np.sqrt(w)
    mu_hat = np.linalg.eigvalsh(s[:, None] * K * s[None, :]).max()
    lam = cmax ** 2 * mu_hat * ((2.0 / hx) ** 2 + (2.0 / hy) ** 2)
    arg = safety * omega / np.sqrt(lam)
    if arg >= 1.0:
        return 4
    return max(4, int(np.ceil(np.pi / np.arcsin(arg))))


def filter_tables(Nt):
    """kappa at integer and half-integer steps, and cos/sin of the forcing
    phase 2 pi nu / N_t, for nu = 0..N_t-1 (eq. (7) and the leapfrog forcing).
    The tan^2 constant does not change the fixed point (its sums against
    cos and sin vanish); it is parity-unpinned except through iterate
    agreement."""
    nu = np.arange(Nt, dtype=float)
    k0 = -0.25 + 0.25 * np.tan(np.pi / Nt) ** 2
    kap = np.cos(2 * np.pi * nu / Nt) + k0
    kaph = np.cos(2 * np.pi * (nu + 0.5) / Nt) + k0
    return kap, kaph, np.cos(2 * np.pi * nu / Nt), np.sin(2 * np.pi * nu / Nt)


def leapfrog_coeffs(M, H, omega, Nt):
    dt = 2 * np.pi / (omega * Nt)
    theta = np.tan(omega * dt / 2) / omega
    sigma = np.sin(omega * dt / 2) / (omega / 2)
    alpha = (M - theta * H) / (M + theta * H)
    beta = sigma / (M + theta * H)
    return sigma, alpha, beta


def iterate(A, M, H, b, omega, Nt, u):
    """One application of the WaveHoltz map Pi (eq. (7)) to u."""
    kap, kaph, cs, sn = filter_tables(Nt)
    sigma, alpha, beta = leapfrog_coeffs(M, H, omega, Nt)
    br, bi = b.real, b.imag
    p = u.real.copy()
    # pdot^{1/2} = Re{-i omega u e^{-i pi/N_t}}
    pd = (-1j * omega * u * np.exp(-1j * np.pi / Nt)).real
    v = kap[0] * p + (1j / omega) * kaph[0] * pd
    for nu in range(1, Nt):
        p = p + sigma * pd
        q = A @ p
        pd = alpha * pd + beta * (-q + br * cs[nu] + bi * sn[nu])
        v = v + kap[nu] * p + (1j / omega) * kaph[nu] * pd
    return (2.0 / Nt) * v


def solve(A, M, H, b, omega, Nt, tol=1e-12, max_iter=100, fixed_iters=None, u0=None):
    """WaveHoltz fixed-point iteration from u0 (default 0, Algorithm 1).

    Stops when ||u_new - u||_2 <= tol ||u_new||_2 or after max_iter, or runs
    exactly ``fixed_iters`` iterations.  Returns (u, iterations)."""
    b = np.asarray(b, dtype=complex)
    u = np.zeros(b.size, dtype=complex) if u0 is None else np.asarray(u0, dtype=complex)
    n = fixed_iters if fixed_iters is not None else max_iter
    it = 0
    for it in range(1, n + 1):
        un = iterate(A, M, H, b, omega, Nt, u)
        if fixed_iters is None:
            d = np.linalg.norm(un - u)
            if d <= tol * np.linalg.norm(un):
                return un, it
        u = un
    return u, it


def trajectory(A, M, H, b, omega, Nt, u):
    """p^nu for nu = 0..N_t-1 of one WaveHoltz period started from u
    (used to check the exactness claim of the modified leapfrog)."""
    _, _, cs, sn = filter_tables(Nt)
    sigma, alpha, beta = leapfrog_coeffs(M, H, omega, Nt)
    p = u.real.copy()
    pd = (-1j * omega * u * np.exp(-1j * np.pi / Nt)).real
    out = [p.copy()]
    for nu in range(1, Nt):
        p = p + sigma * pd
        pd = alpha * pd + beta * (-(A @ p) + b.real * cs[nu] + b.imag * sn[nu])
        out.append(p.copy())
    return np.array(out)


def time_steps3(P, hx, hy, hz, cmax, omega, safety=0.9):
    """``time_steps`` for the box: lambda_bar gains the third direction,
    lambda_bar = cmax^2 mu_hat ((2/hx)^2 + (2/hy)^2 + (2/hz)^2)."""
    _, w = gll.nodes_weights(P)
    K = gll.element_stiffness_1d(P)
    s = 1.0 / np.sqrt(w)
    mu_hat = np.linalg.eigvalsh(s[:, None] * K * s[None, :]).max()
    lam = cmax ** 2 * mu_hat * ((2.0 / hx) ** 2 + (2.0 / hy) ** 2 + (2.0 / hz) ** 2)
    arg = safety * omega / np.sqrt(lam)
    if arg >= 1.0:
        return 4
    return max(4, int(np.ceil(np.pi / np.arcsin(arg))))


def subdomain_steps(dec, safety=0.9):
    """N_t of every subdomain of a Decomposition (c_max over its nodes); 2D
    rectangles or 3D boxes."""
    out = []
    for l in range(dec.L):
        sd = dec.subs[l]
        r = sd["rect"]
        if hasattr(r, "nz"):
            out.append(time_steps3(r.P, r.hx, r.hy, r.hz, sd["c"].max(), dec.omega, safety))
        else:
            out.append(time_steps(r.P, r.hx, r.hy, sd["c"].max(), dec.omega, safety))
    return out


def make_solver(dec, tol=1e-12, max_iter=100, fixed_iters=None, safety=0.9, counts=None):
    """Subdomain solver for ``Decomposition.sweep`` that runs WaveHoltz."""
    nts = subdomain_steps(dec, safety)

    def solver(l, b):
        sd = dec.subs[l]
        u, it = solve(sd["At"], sd["Mt"], sd["H"], b, dec.omega, nts[l], tol, max_iter, fixed_iters)
        if counts is not None:
            counts.append(it)
        return u
    return solver
