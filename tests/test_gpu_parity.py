"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (relative l2 over the stacked subdomain copies):
* stiffness apply, FP64: 1e-13; FP32: 2e-6 (single rounding per term).
* fixed-count WaveHoltz sweep iterates, FP64: 1e-11 (the GPU sums the
  stiffness in a different order; the error after m periods of N_t steps stays
  within a few hundred ulps of the solution); FP32: 1e-4 (bounded by
  N_t * m * eps_32 * amplification).
* converged sweep vs sparse LU, FP64: 1e-9 (inner tolerance 1e-12 times the
  WaveHoltz contraction constant).
* full solve vs the oracle DD at the same outer tolerance: 1e-10 in FP64;
  FP32 subdomain sweeps: 1e-6.
"""
import numpy as np
import pytest

from oracle import dd, sem
from oracle import waveholtz as wh

pytestmark = pytest.mark.gpu


def _setup(W, nx, ny, P, sx, sy, omega, cfun, box=(0.0, 1.0, 0.0, 1.0), **opt):
    o = W.dd_default_options(**opt)
    N = (nx * P + 1) * (ny * P + 1)
    probe = W.dd_setup(nx, ny, P, np.ones(N), omega, sx, sy, *box, options=o)
    X, Y = W.dd_node_coords(probe)
    W.dd_destroy(probe)
    h = W.dd_setup(nx, ny, P, cfun(X, Y), omega, sx, sy, *box, options=o)
    return h, X, Y


def _oracle(nx, ny, P, sx, sy, omega, cfun, box=(0.0, 1.0, 0.0, 1.0)):
    mesh = sem.Rect(nx, ny, P, *box)
    X, Y = sem.node_coords(mesh)
    dec = dd.Decomposition(mesh, dd.Partition(sx, sy), cfun(X, Y), omega)
    return dec, X, Y


def _cwave(X, Y):
    return 1.0 + 0.35 * np.sin(5 * X + 0.3) * np.cos(4 * Y - 0.2)


def _rel(a, b):
    a, b = np.concatenate([np.ravel(x) for x in a]), np.concatenate([np.ravel(x) for x in b])
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SHAPES = [(6, 4, 3, 2, 2), (8, 8, 2, 2, 2), (4, 6, 1, 2, 3), (4, 4, 4, 2, 1), (3, 5, 3, 1, 1),
          (4, 3, 3, 4, 3)]  # last: one element per subdomain
LAYOUTS = [1, 2, 3, 4]  # DD_LAYOUT_NODE, _PATCH, _PATCH_XCHG, _STREAM


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [0, 1])
def test_stiffness_apply(gpu_lib, shape, layout, prec):
    W = gpu_lib
    nx, ny, P, sx, sy = shape
    h, _, _ = _setup(W, nx, ny, P, sx, sy, 7.0, _cwave, precision=prec, layout=layout)
    dec, _, _ = _oracle(nx, ny, P, sx, sy, 7.0, _cwave)
    print(f"stiffness shape={shape} layout={layout} prec={prec}", flush=True)
    rng = np.random.default_rng(sum(shape) + 10 * layout)
    p = rng.standard_normal(dec.L * dec.nxl * dec.nyl)
    q = W.dd_apply_stiffness(h, p)
    n = dec.nxl * dec.nyl
    ref = [dec.subs[l]["A"] @ p[l * n:(l + 1) * n] for l in range(dec.L)]
    W.dd_destroy(h)
    assert _rel([q], ref) < (1e-13 if prec == 0 else 2e-6)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_stiffness_unit_vectors(gpu_lib, layout):
    """A applied to every unit vector of a one-subdomain mesh equals the
    oracle's assembled matrix entry by entry."""
    W = gpu_lib
    h, _, _ = _setup(W, 3, 2, 3, 1, 1, 5.0, _cwave, layout=layout)
    dec, _, _ = _oracle(3, 2, 3, 1, 1, 5.0, _cwave)
    A = dec.subs[0]["A"].toarray()
    n = A.shape[0]
    cols = np.array([W.dd_apply_stiffness(h, np.eye(n)[k]) for k in range(n)]).T
    W.dd_destroy(h)
    assert np.abs(cols - A).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_time_steps_match_oracle(gpu_lib, shape):
    W = gpu_lib
    nx, ny, P, sx, sy = shape
    for om in (3.0, 11.0, 40.0):
        h, _, _ = _setup(W, nx, ny, P, sx, sy, om, _cwave)
        dec, _, _ = _oracle(nx, ny, P, sx, sy, om, _cwave)
        nt = W.dd_time_steps(h)
        W.dd_destroy(h)
        assert list(nt) == wh.subdomain_steps(dec), (shape, om)


def _random_g(dec, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_fixed_iterations(gpu_lib, shape, layout, prec):
    """One DD cycle with exactly m WaveHoltz iterations from u = 0: iterates
    and interface output against the oracle's WaveHoltz (Algorithm 1)."""
    W = gpu_lib
    nx, ny, P, sx, sy = shape
    om, m = 9.0, 3
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, precision=prec, layout=layout,
                       tau_in=0.0, max_wh=m)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, om, _cwave)
    print(f"sweep shape={shape} layout={layout} prec={prec}", flush=True)
    g = _random_g(dec, sum(shape))
    f = np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.02)
    fl = np.exp(-((Xl - 0.4) ** 2 + (Yl - 0.55) ** 2) / 0.02)
    g_gpu, u_gpu, its = W.dd_sweep(h, g, fl, 1.0)
    W.dd_destroy(h)
    g_ref, u_ref = dec.sweep(g, f, 1.0, wh.make_solver(dec, fixed_iters=m))
    assert (its == m).all()
    tol = 1e-11 if prec == 0 else 1e-4
    assert _rel([u_gpu], u_ref) < tol
    assert _rel([g_gpu], [g_ref]) < tol


@pytest.mark.parametrize("shape", [(6, 4, 3, 2, 2), (6, 6, 2, 3, 2), (4, 3, 3, 4, 3)])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_second_order_condition(gpu_lib, shape, layout, prec):
    """Second-order transmission condition (tc2 > 0): one DD cycle of exactly
    m WaveHoltz iterations against the oracle's sweep with the same
    q = tc2 * min(c) / omega (extended 1D weights in the coefficients, the
    tangential terms in the interface update)."""
    W = gpu_lib
    nx, ny, P, sx, sy = shape
    om, m, tc2 = 9.0, 3, 0.3
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, precision=prec, layout=layout,
                       tau_in=0.0, max_wh=m, tc2=tc2)
    mesh = sem.Rect(nx, ny, P)
    X, Y = sem.node_coords(mesh)
    q = tc2 * _cwave(Xl, Yl).min() / om
    dec = dd.Decomposition(mesh, dd.Partition(sx, sy), _cwave(X, Y), om, q=q)
    print(f"sweep tc2 shape={shape} layout={layout} prec={prec}", flush=True)
    g = _random_g(dec, sum(shape) + 1)
    f = np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.02)
    fl = np.exp(-((Xl - 0.4) ** 2 + (Yl - 0.55) ** 2) / 0.02)
    nt = W.dd_time_steps(h)
    g_gpu, u_gpu, its = W.dd_sweep(h, g, fl, 1.0)
    W.dd_destroy(h)
    assert list(nt) == wh.subdomain_steps(dec)
    g_ref, u_ref = dec.sweep(g, f, 1.0, wh.make_solver(dec, fixed_iters=m))
    tol = 1e-11 if prec == 0 else 1e-4
    assert _rel([u_gpu], u_ref) < tol
    assert _rel([g_gpu], [g_ref]) < tol


@pytest.mark.parametrize("layout", LAYOUTS)
def test_sweep_converged_matches_lu(gpu_lib, layout):
    W = gpu_lib
    nx, ny, P, sx, sy = 8, 8, 2, 2, 2
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, 10.0, _cwave, layout=layout, tau_in=1e-12)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, 10.0, _cwave)
    g = _random_g(dec, 5)
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    fl = np.exp(-((Xl - 0.3) ** 2 + (Yl - 0.6) ** 2) / (2 * 0.05 ** 2))
    g_gpu, u_gpu, its = W.dd_sweep(h, g, fl, 1.0)
    W.dd_destroy(h)
    g_ref, u_ref = dec.sweep(g, f, 1.0)
    assert _rel([u_gpu], u_ref) < 1e-9
    assert _rel([g_gpu], [g_ref]) < 1e-9
    # the stop rule (Sec. V): each subdomain stops after as many WaveHoltz
    # iterations as the oracle's WaveHoltz under the same rule, and the
    # iterates agree
    counts = []
    g_wh, u_wh = dec.sweep(g, f, 1.0, wh.make_solver(dec, tol=1e-12, max_iter=1000,
                                                       counts=counts))
    print(f"layout {layout}: GPU WaveHoltz counts {its.tolist()}, oracle {counts}", flush=True)
    assert its.tolist() == counts
    assert _rel([u_gpu], u_wh) < 1e-11


@pytest.mark.parametrize("layout", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_full_workgroup_subdomains(gpu_lib, layout, prec):
    """Subdomains of 16x16 elements at P = 3 (2401 nodes, the shape of the
    256x256 waveguide's subdomains): all 256 threads of the patch layouts
    own an element and 97 of them an edge node.  A 2x2 grid of them, a
    source, random interface data, exactly 2 WaveHoltz iterations against
    the oracle's WaveHoltz."""
    W = gpu_lib
    nx, ny, P, sx, sy = 32, 32, 3, 2, 2
    om, m = 60.0, 2
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, precision=prec, layout=layout,
                       tau_in=0.0, max_wh=m)
    assert W.dd_layout(h) == (layout, 256)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, om, _cwave)
    print(f"sweep 16x16-element subdomains layout={layout} prec={prec}", flush=True)
    g = _random_g(dec, 17)
    f = np.exp(-((X - 0.45) ** 2 + (Y - 0.6) ** 2) / 0.01)
    fl = np.exp(-((Xl - 0.45) ** 2 + (Yl - 0.6) ** 2) / 0.01)
    g_gpu, u_gpu, its = W.dd_sweep(h, g, fl, 1.0)
    W.dd_destroy(h)
    g_ref, u_ref = dec.sweep(g, f, 1.0, wh.make_solver(dec, fixed_iters=m))
    assert (its == m).all()
    tol = 1e-11 if prec == 0 else 1e-4
    assert _rel([u_gpu], u_ref) < tol
    assert _rel([g_gpu], [g_ref]) < tol


def test_autotuned_layout_is_a_fitting_layout(gpu_lib):
    W = gpu_lib
    h, _, _ = _setup(W, 8, 8, 2, 2, 2, 10.0, _cwave)  # auto
    lay, wg = W.dd_layout(h)
    W.dd_destroy(h)
    assert lay in (1, 2, 3) and wg % 64 == 0   # on-chip layouts when they fit


@pytest.mark.parametrize("prec", [0, 1])
def test_stream_matches_node_bitwise(gpu_lib, prec):
    """STREAM performs the NODE layout's per-node arithmetic in the same
    order (and, with one node per thread, the same stop-test sums): the
    sweeps agree bit for bit."""
    W = gpu_lib
    nx, ny, P, sx, sy = 6, 4, 3, 2, 2
    dec, X, Y = _oracle(nx, ny, P, sx, sy, 9.0, _cwave)
    g = _random_g(dec, 3)
    out = []
    for lay in (1, 4):
        h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, 9.0, _cwave, precision=prec, layout=lay,
                           tau_in=1e-9 if prec == 0 else 1e-5)
        fl = np.exp(-((Xl - 0.4) ** 2 + (Yl - 0.55) ** 2) / 0.02)
        out.append(W.dd_sweep(h, g, fl, 1.0))
        W.dd_destroy(h)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_stream_solve_large_subdomains_matches_oracle_dd(gpu_lib):
    """2x2 subdomains of 24x24 elements at P=3 (5329 nodes each, more than
    the on-chip layouts hold): auto picks STREAM; the FP64 solve follows
    the oracle DD's GMRES path."""
    W = gpu_lib
    nx = ny = 48
    P, sx, sy, om = 3, 2, 2, 25.0
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, tau_in=1e-12)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, om, _cwave)
    lay, wg = W.dd_layout(h)
    print(f"stream layout threads per subdomain {wg}", flush=True)
    assert lay == 4 and wg in (256, 512, 1024, 2048)

    def src(X, Y):
        return np.exp(-((X - 0.37) ** 2 + (Y - 0.58) ** 2) / (2 * 0.04 ** 2))
    u, st, _ = W.dd_solve(h, src(Xl, Yl), None, 1e-8)
    W.dd_destroy(h)
    us_ref, info = dd.solve_dd(dec, src(X, Y), tol=1e-8)
    assert info["passes"] == 1
    print(f"stream solve gpu iters={st['outer_iters']} oracle={info['iters']}", flush=True)
    assert st["outer_iters"] == info["iters"]
    assert _rel([u], [dec.glue(us_ref)]) < 1e-10


@pytest.mark.parametrize("prec", [0, 1])
def test_c3_full_size_sweep_sampled(gpu_lib, prec):
    """The 512x512-element P=3 waveguide with 8x8 subdomains (193x193 nodes
    each, STREAM) at full size: one sweep of two fixed WaveHoltz iterations
    from random interface data, in the launch configuration of a solve.
    Sampled subdomains (corner, edge, interior) are recomputed one by one by
    the oracle's WaveHoltz on that subdomain alone."""
    import workloads
    W = gpu_lib
    wl = workloads.c3()
    m = 2
    h, Xl, Yl = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, precision=prec,
                       tau_in=0.0, max_wh=m)
    lay, _ = W.dd_layout(h)
    assert lay == 4
    sizes = W.dd_sizes(h)
    L, nloc, n_if = sizes["n_sub"], sizes["n_local"], sizes["n_iface"]
    rng = np.random.default_rng(33)
    g = rng.standard_normal(n_if) + 1j * rng.standard_normal(n_if)
    print(f"c3 sweep prec={prec} L={L} nloc={nloc}", flush=True)
    g_gpu, u_gpu, its = W.dd_sweep(h, g, wl.f(Xl, Yl), 1.0)
    W.dd_destroy(h)
    assert (its == m).all()
    mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    mx, my = wl.nx // wl.sx, wl.ny // wl.sy
    nxl, nyl = mx * wl.P + 1, my * wl.P + 1
    per = 2 * nxl + 2 * nyl
    X, Y = sem.node_coords(mesh)
    c, f = wl.c(X, Y), wl.f(X, Y)
    tol = 1e-11 if prec == 0 else 1e-4
    for l in (0, 13, 63):
        a, b = l % wl.sx, l // wl.sx
        x0, y0 = wl.x0 + a * mx * mesh.hx, wl.y0 + b * my * mesh.hy
        sub = sem.Rect(mx, my, wl.P, x0, x0 + mx * mesh.hx, y0, y0 + my * mesh.hy)
        i = a * mx * wl.P + np.arange(nxl)
        j = b * my * wl.P + np.arange(nyl)
        gl = (j[:, None] * mesh.Nx + i[None, :]).ravel()
        one = dd.Decomposition(sub, dd.Partition(1, 1), c[gl], wl.omega)
        fl = np.zeros(sub.N)
        fl[:] = f[gl]
        b_l = one.rhs(0, fl, g[l * per:(l + 1) * per], 1.0)
        sd = one.subs[0]
        nt = wh.subdomain_steps(one)[0]
        u_ref, it = wh.solve(sd["A"], sd["M"], sd["H"], b_l, wl.omega, nt, fixed_iters=m)
        assert _rel([u_gpu[l * nloc:(l + 1) * nloc]], [u_ref]) < tol, l


def test_sweep_is_deterministic(gpu_lib):
    W = gpu_lib
    h, Xl, Yl = _setup(W, 8, 8, 3, 2, 2, 12.0, _cwave, tau_in=1e-10)
    dec, _, _ = _oracle(8, 8, 3, 2, 2, 12.0, _cwave)
    g = _random_g(dec, 9)
    a = W.dd_sweep(h, g, None, 0.0)
    b = W.dd_sweep(h, g, None, 0.0)
    W.dd_destroy(h)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _c1_pair(W, **opt):
    import workloads
    wl = workloads.c1()
    h, Xl, Yl = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, **opt)
    dec, X, Y = _oracle(wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c)
    return wl, h, Xl, Yl, dec, X, Y


@pytest.mark.parametrize("layout", LAYOUTS)
def test_solve_c1_fp64_matches_oracle_dd(gpu_lib, layout):
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W, layout=layout, tau_in=1e-12)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol)
    us_ref, info = dd.solve_dd(dec, wl.f(X, Y), tol=wl.tol)
    assert info["passes"] == 1
    W.dd_destroy(h)
    print(f"c1 gpu iters={st['outer_iters']} oracle iters={info['iters']}", flush=True)
    assert st["outer_iters"] == info["iters"]
    assert _rel([u], [dec.glue(us_ref)]) < 1e-10
    assert st["true_rel_residual"] < 2 * wl.tol


def test_solve_c1_tight_matches_global_lu(gpu_lib):
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W, tau_in=1e-14)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, 1e-12)
    u_lu = sem.solve(dec.mesh, wl.c(X, Y), wl.omega, wl.f(X, Y))
    rel_res = W.dd_residual(h, u, wl.f(Xl, Yl))
    W.dd_destroy(h)
    assert _rel([u], [u_lu]) < 1e-10
    assert rel_res < 1e-10


@pytest.mark.parametrize("layout", [0] + LAYOUTS)
def test_solve_c1_fp32_refined(gpu_lib, layout):
    """FP32 sweeps with FP64 residual refinement reach the FP64 answer (FP32
    and FP64 sweeps alternate on one handle: for STREAM they must not share
    workspace bytes)."""
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W, precision=1, tau_in=1e-6, layout=layout)
    u, st, rc = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol)
    W.dd_destroy(h)
    u_lu = sem.solve(dec.mesh, wl.c(X, Y), wl.omega, wl.f(X, Y))
    err = _rel([u], [u_lu])
    print(f"c1 fp32+refine err={err:.3e} iters={st['outer_iters']} refine={st['refine_steps']} "
          f"true_res={st['true_rel_residual']:.2e}")
    assert st["true_rel_residual"] <= wl.tol
    assert err < 1e-6


def _c2_small_pair(W, **opt):
    import workloads
    wl = workloads.c2_small()
    h, Xl, Yl = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, **opt)
    dec, X, Y = _oracle(wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c)
    return wl, h, Xl, Yl, dec, X, Y


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_c2_small_matches_oracle_dd(gpu_lib, prec):
    """The waveguide at 64x64 elements with the benchmark's subdomain shape
    (4x4 subdomains of 16x16 elements, P = 3): the full GMRES solve against
    the oracle DD (splu subdomain solves, same GMRES) at the same outer
    tolerance.  FP64 with tau_in = 1e-12: 1e-10 and the same iteration count;
    FP32 sweeps (tau_in = 1e-5) with FP64 refinement: 1e-6.  The WaveHoltz
    cap is 1000: the waveguide-junction subdomains need up to ~160 periods
    to reach 1e-12 (the default cap of 100 stops them near 1e-8)."""
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c2_small_pair(W, precision=prec, max_wh=1000,
                                              tau_in=1e-12 if prec == 0 else 1e-5)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol, max_iter=2000)
    W.dd_destroy(h)
    us_ref, info = dd.solve_dd(dec, wl.f(X, Y), tol=wl.tol)
    assert info["passes"] == 1
    err = _rel([u], [dec.glue(us_ref)])
    print(f"c2_small prec={prec} gpu iters={st['outer_iters']} oracle iters={info['iters']} "
          f"wh_max={st['wh_iters_max']} err={err:.2e}", flush=True)
    assert info["passes"] == 1   # the oracle is plain GMRES from G = 0
    assert st["true_rel_residual"] <= wl.tol
    if prec == 0:
        assert st["outer_iters"] == info["iters"]
        assert err < 1e-10
    else:
        assert err < 1e-6


def test_solve_c2_small_capped_at_100(gpu_lib):
    """With the WaveHoltz cap at 100 the junction subdomains stop before
    tau_in = 1e-12; the solve still meets the outer tolerance and stays
    within 1e-6 of the oracle DD (the library's default cap is 1000)."""
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c2_small_pair(W, tau_in=1e-12, max_wh=100)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol, max_iter=2000)
    W.dd_destroy(h)
    us_ref, _ = dd.solve_dd(dec, wl.f(X, Y), tol=wl.tol)
    assert st["wh_iters_max"] == 100
    assert st["true_rel_residual"] <= wl.tol
    assert _rel([u], [dec.glue(us_ref)]) < 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_zero_data_gives_zero(gpu_lib, prec):
    """No source and no boundary data: the solution is exactly zero, found
    without an outer iteration."""
    W = gpu_lib
    h, Xl, Yl = _setup(W, 6, 4, 3, 2, 2, 9.0, _cwave, precision=prec)
    u, st, rc = W.dd_solve(h, None, None, 1e-8)
    W.dd_destroy(h)
    assert rc == W.DD_OK and st["outer_iters"] == 0
    assert not np.any(u)


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_second_order_condition_matches_oracle_dd(gpu_lib, prec):
    """c1 with the second-order condition (tc2 = 0.25): FP64 against the oracle
    DD with the same q (1e-10, same iteration count), FP32 sweeps with FP64
    refinement against the global solution (1e-6); fewer outer iterations
    than the zeroth-order condition."""
    W = gpu_lib
    tc2 = 0.25
    tau = 1e-12 if prec == 0 else 1e-6
    wl, h, Xl, Yl, dec0, X, Y = _c1_pair(W, precision=prec, tau_in=tau, tc2=tc2)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol)
    W.dd_destroy(h)
    h0, _, _ = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, precision=prec,
                      tau_in=tau)
    _, st0, _ = W.dd_solve(h0, wl.f(Xl, Yl), None, wl.tol)
    W.dd_destroy(h0)
    q = tc2 * wl.c(Xl, Yl).min() / wl.omega
    dec = dd.Decomposition(dec0.mesh, dec0.part, wl.c(X, Y), wl.omega, q=q)
    us_ref, info = dd.solve_dd(dec, wl.f(X, Y), tol=wl.tol)
    assert info["passes"] == 1
    print(f"c1 tc2 prec={prec} gpu iters={st['outer_iters']} oracle iters={info['iters']} "
          f"zeroth-order iters={st0['outer_iters']}", flush=True)
    assert st["true_rel_residual"] <= wl.tol
    assert st["outer_iters"] < st0["outer_iters"]
    if prec == 0:
        assert st["outer_iters"] == info["iters"]
        assert _rel([u], [dec.glue(us_ref)]) < 1e-10
    else:
        u_lu = sem.solve(dec.mesh, wl.c(X, Y), wl.omega, wl.f(X, Y))
        assert _rel([u], [u_lu]) < 1e-6


def test_solve_c2_small_second_order_condition(gpu_lib):
    """The benchmark's subdomain shape with the second-order condition
    (tc2 = 0.25, cap 1000): FP64 solve against the oracle DD with the same q."""
    W = gpu_lib
    wl, h, Xl, Yl, dec0, X, Y = _c2_small_pair(W, max_wh=1000, tau_in=1e-12, tc2=0.25)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol, max_iter=2000)
    W.dd_destroy(h)
    q = 0.25 * wl.c(Xl, Yl).min() / wl.omega
    dec = dd.Decomposition(dec0.mesh, dec0.part, wl.c(X, Y), wl.omega, q=q)
    us_ref, info = dd.solve_dd(dec, wl.f(X, Y), tol=wl.tol)
    assert info["passes"] == 1
    err = _rel([u], [dec.glue(us_ref)])
    print(f"c2_small tc2 gpu iters={st['outer_iters']} oracle iters={info['iters']} err={err:.2e}",
          flush=True)
    assert st["outer_iters"] == info["iters"]
    assert err < 1e-10


def test_solve_c1_fp32_plain(gpu_lib):
    """FP32 sweeps and FP32-accurate outer residuals only (refine = 0: one
    GMRES pass, asked for the whole outer tolerance): the error floor is
    the FP32 sweep's."""
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W, precision=1, tau_in=1e-6, refine=0)
    u, st, rc = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol, allow_notconv=True)
    W.dd_destroy(h)
    u_lu = sem.solve(dec.mesh, wl.c(X, Y), wl.omega, wl.f(X, Y))
    err = _rel([u], [u_lu])
    print(f"c1 fp32 plain err={err:.3e} true_res={st['true_rel_residual']:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_c1_relaxed_inner_tolerance(gpu_lib, prec):
    """Variable inner tolerance: the matvecs loosen as the outer residual
    falls; the answer still meets the outer tolerance (true residual)."""
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W, precision=prec, tau_in=1e-12 if prec == 0 else 1e-6,
                                        relax=0.1)
    u, st, rc = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol)
    W.dd_destroy(h)
    u_lu = sem.solve(dec.mesh, wl.c(X, Y), wl.omega, wl.f(X, Y))
    err = _rel([u], [u_lu])
    print(f"c1 relaxed prec={prec} err={err:.3e} true_res={st['true_rel_residual']:.2e} "
          f"wh_total={st['wh_iters_total']}")
    assert st["true_rel_residual"] <= 2 * wl.tol
    assert err < 1e-6


def test_plane_wave_boundary_data(gpu_lib):
    """Outer impedance data g = i k (d.n - 1) u of an exact plane wave."""
    W = gpu_lib
    nx, P, om = 8, 3, 12.0
    h, Xl, Yl = _setup(W, nx, nx, P, 2, 4, om, lambda X, Y: np.ones_like(X), tau_in=1e-14)
    mesh = sem.Rect(nx, nx, P)
    ue, g = sem.plane_wave(mesh, om, 1.0, (np.cos(1.1), np.sin(1.1)))
    u, st, _ = W.dd_solve(h, None, g, 1e-12)
    u_lu = sem.solve(mesh, np.ones(mesh.N), om, np.zeros(mesh.N), g)
    W.dd_destroy(h)
    assert _rel([u], [u_lu]) < 1e-9
    assert _rel([u], [ue]) < 1e-3


def test_single_subdomain_is_one_sweep(gpu_lib):
    W = gpu_lib
    h, Xl, Yl = _setup(W, 6, 6, 2, 1, 1, 8.0, _cwave)
    dec, X, Y = _oracle(6, 6, 2, 1, 1, 8.0, _cwave)
    f = np.cos(3 * X) * Y
    u, st, _ = W.dd_solve(h, np.cos(3 * Xl) * Yl, None, 1e-10)
    W.dd_destroy(h)
    assert st["outer_iters"] == 0
    assert _rel([u], [sem.solve(dec.mesh, dec.c, 8.0, f)]) < 1e-9


def test_max_iter_reports_not_converged(gpu_lib):
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W)
    u, st, rc = W.dd_solve(h, wl.f(Xl, Yl), None, 1e-12, max_iter=2, allow_notconv=True)
    W.dd_destroy(h)
    assert rc == W.DD_ENOTCONV
    assert st["outer_iters"] == 2 and np.isfinite(u).all()


@pytest.mark.parametrize("nx,ny,P", [(5, 7, 3), (40, 30, 2), (9, 70, 1), (12, 11, 4),
                                     (100, 12, 3)])
def test_operator_and_residual_kernels(gpu_lib, nx, ny, P):
    """Whole-domain S x and the global residual against the oracle's
    assembled S, on grids spanning several row segments and column blocks
    of the operator kernel."""
    import torch
    W = gpu_lib
    h, Xl, Yl = _setup(W, nx, ny, P, 1, 1, 6.0, _cwave)
    mesh = sem.Rect(nx, ny, P)
    X, Y = sem.node_coords(mesh)
    S, _, _, _ = sem.system(mesh, _cwave(X, Y), 6.0)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(mesh.N) + 1j * rng.standard_normal(mesh.N)
    xt = torch.from_numpy(np.stack([x.real, x.imag], 1).ravel()).cuda()
    yt = torch.empty_like(xt)
    W.dd_apply_operator_device(h, xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    y = y[0::2] + 1j * y[1::2]
    ref = S @ x
    f = rng.standard_normal(mesh.N)
    rel = W.dd_residual(h, x, f)
    b = sem.load(mesh, f)
    W.dd_destroy(h)
    assert np.linalg.norm(y - ref) < 1e-13 * np.linalg.norm(ref)
    assert abs(rel - np.linalg.norm(b - ref) / np.linalg.norm(b)) < 1e-12 * rel


def test_state_roundtrip(gpu_lib):
    W = gpu_lib
    wl, h, Xl, Yl, dec, X, Y = _c1_pair(W)
    u, st, _ = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol)
    G = W.dd_get_state(h)
    W.dd_set_state(h, G)
    assert np.array_equal(W.dd_get_state(h), G)
    W.dd_destroy(h)


@pytest.mark.parametrize("layout", [0, 4])
def test_fixed_point_warm_start(gpu_lib, layout):
    """Fixed-point outer iteration, cold and warm-started WaveHoltz, on a
    strip partition (no interior cross points, so I - T has no null mode and
    the fixed point converges): the cold run follows the oracle's fixed-point
    iteration; both reach the global LU solution to the outer tolerance's
    accuracy; warm starts need far fewer WaveHoltz iterations."""
    W = gpu_lib
    nx, ny, P, sx, sy, om, tol = 8, 8, 1, 2, 1, 6.0, 1e-8   # converges in ~480 iterations

    def src(X, Y):
        return np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * 0.05 ** 2))
    out = {}
    for warm in (0, 1):
        h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, outer=W.DD_OUTER_FIXED, warm=warm,
                           tau_in=1e-12, layout=layout)
        u, st, rc = W.dd_solve(h, src(Xl, Yl), None, tol, max_iter=5000)
        W.dd_destroy(h)
        out[warm] = (u, st)
        print(f"fixed point warm={warm} iters={st['outer_iters']} "
              f"wh_total={st['wh_iters_total']}", flush=True)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, om, _cwave)
    us_ref, info = dd.solve_dd(dec, src(X, Y), tol=tol, method="fixed", max_iter=5000)
    u_lu = sem.solve(dec.mesh, _cwave(X, Y), om, src(X, Y))
    assert abs(out[0][1]["outer_iters"] - info["iters"]) <= 1
    for warm in (0, 1):
        assert _rel([out[warm][0]], [u_lu]) < 1e-6
        assert out[warm][1]["true_rel_residual"] <= 2 * tol
    assert out[1][1]["wh_iters_total"] < 0.5 * out[0][1]["wh_iters_total"]


def _oracle_sub(wl, mesh, l, c, f, g_l, nxl, nyl, mx, my):
    """The oracle's system for subdomain l of a workload alone (a 1x1
    decomposition of its rectangle) and its right-hand side."""
    a, b = l % wl.sx, l // wl.sx
    x0, y0 = wl.x0 + a * mx * mesh.hx, wl.y0 + b * my * mesh.hy
    sub = sem.Rect(mx, my, wl.P, x0, x0 + mx * mesh.hx, y0, y0 + my * mesh.hy)
    i = a * mx * wl.P + np.arange(nxl)
    j = b * my * wl.P + np.arange(nyl)
    gl = (j[:, None] * mesh.Nx + i[None, :]).ravel()
    one = dd.Decomposition(sub, dd.Partition(1, 1), c[gl], wl.omega)
    b_l = one.rhs(0, np.asarray(f[gl], dtype=float), g_l, 1.0)
    return one, b_l


@pytest.mark.parametrize("prec", [0, 1])
def test_c2_full_size_sweep_sampled(gpu_lib, prec):
    """The 256x256-element P=3 waveguide with 16x16 subdomains at full size,
    in the autotuned layout the benchmark uses: one sweep of three fixed
    WaveHoltz iterations from random interface data; sampled subdomains
    (corner, edge, waveguide, interior) recomputed one by one by the
    oracle's WaveHoltz."""
    import workloads
    W = gpu_lib
    wl = workloads.c2()
    m = 3
    h, Xl, Yl = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, precision=prec,
                       tau_in=0.0, max_wh=m)
    sizes = W.dd_sizes(h)
    nloc, n_if = sizes["n_local"], sizes["n_iface"]
    rng = np.random.default_rng(22)
    g = rng.standard_normal(n_if) + 1j * rng.standard_normal(n_if)
    print(f"c2 sweep prec={prec} layout={W.dd_layout(h)}", flush=True)
    g_gpu, u_gpu, its = W.dd_sweep(h, g, wl.f(Xl, Yl), 1.0)
    W.dd_destroy(h)
    assert (its == m).all()
    mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    mx, my = wl.nx // wl.sx, wl.ny // wl.sy
    nxl, nyl = mx * wl.P + 1, my * wl.P + 1
    per = 2 * nxl + 2 * nyl
    X, Y = sem.node_coords(mesh)
    c, f = wl.c(X, Y), wl.f(X, Y)
    tol = 1e-11 if prec == 0 else 1e-4
    for l in (0, 7, 8 + 16 * 2, 8 + 16 * 9, 255):
        one, b_l = _oracle_sub(wl, mesh, l, c, f, g[l * per:(l + 1) * per], nxl, nyl, mx, my)
        sd = one.subs[0]
        nt = wh.subdomain_steps(one)[0]
        u_ref, _ = wh.solve(sd["A"], sd["M"], sd["H"], b_l, wl.omega, nt, fixed_iters=m)
        assert _rel([u_gpu[l * nloc:(l + 1) * nloc]], [u_ref]) < tol, l


@pytest.fixture(scope="module")
def c2_oracle_dd():
    """The oracle DD (exact sparse-LU subdomain solves, GMRES(50) from
    G = 0) of the 256x256-element waveguide at its outer tolerance, computed
    once on a pool of host processes."""
    import workloads
    from oracle import pool
    wl = workloads.c2()
    mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    X, Y = sem.node_coords(mesh)
    c, f = wl.c(X, Y), wl.f(X, Y)
    with pool.ParallelDecomposition(mesh, dd.Partition(wl.sx, wl.sy), c, wl.omega) as pdec:
        us, info = dd.solve_dd(pdec, f, tol=wl.tol)
        u = pdec.glue(us)
    print(f"oracle DD c2: {info['iters']} outer iterations on {pdec.workers} workers", flush=True)
    return wl, mesh, c, f, u, info


@pytest.mark.parametrize("variant", ["fp64", "fp32_refined"])
def test_c2_full_size_solve_matches_oracle_dd(gpu_lib, c2_oracle_dd, variant):
    """The benchmark's solve at full size (256x256 elements, P = 3, 16x16
    subdomains, tol 1e-8) with the benchmark's options: the glued GPU
    solution against the oracle DD at the same outer tolerance.  FP64
    (WaveHoltz to 1e-12): 1e-10 and the same outer iteration count; FP32
    sweeps with FP64 refinement: 1e-6.  The FP64 run also meets the global
    residual measured with the oracle's assembled operator."""
    from bench import VARIANTS
    W = gpu_lib
    wl, mesh, c, f, u_ref, info = c2_oracle_dd
    assert info["passes"] == 1
    if variant == "fp64":
        opt = dict(precision=0, tau_in=wl.tau_in)
    else:
        pname, tau, relax, tc2 = VARIANTS[variant]
        assert (pname, relax, tc2) == ("fp32", 0.0, 0.0)
        opt = dict(precision=1, tau_in=tau)
    h, Xl, Yl = _setup(W, wl.nx, wl.ny, wl.P, wl.sx, wl.sy, wl.omega, wl.c, max_wh=1000, **opt)
    print(f"c2 full-size solve {variant}, layout {W.dd_layout(h)}", flush=True)
    u, st, rc = W.dd_solve(h, wl.f(Xl, Yl), None, wl.tol, max_iter=2000)
    W.dd_destroy(h)
    err = _rel([u], [u_ref])
    print(f"c2 {variant}: gpu iters={st['outer_iters']} oracle iters={info['iters']} "
          f"wh_max={st['wh_iters_max']} rel_l2_vs_oracle={err:.2e}", flush=True)
    assert rc == 0 and st["true_rel_residual"] <= wl.tol
    if variant == "fp64":
        assert st["wh_iters_max"] < 1000   # every subdomain reached tau_in
        assert st["outer_iters"] == info["iters"]
        assert err < 1e-10
        S, _, _, _ = sem.system(mesh, c, wl.omega)
        b = sem.load(mesh, f)
        res = np.linalg.norm(b - S @ u) / np.linalg.norm(b)
        print(f"c2 global residual {res:.2e}", flush=True)
        assert res < 5 * wl.tol
    else:
        assert err < 1e-6


@pytest.mark.parametrize("shape", [(128, 3, 2, 60.0), (128, 2, 4, 19.7), (96, 2, 3, 30.0)])
def test_stream_shared_subdomains_match_single_workgroup(gpu_lib, shape):
    """Large STREAM subdomains of an FP64 problem with few of them: the
    autotuner may give each subdomain several workgroups (synchronised
    through L2 every step).  With a fixed WaveHoltz count the per-node
    arithmetic is the same as with one workgroup per subdomain, so the
    sweeps agree bit for bit (also with short row segments: 4x4 subdomains
    of 65x65 nodes split over 32 waves).  FP32 sweeps keep one workgroup per
    subdomain."""
    W = gpu_lib
    nx, P, s_, om = shape
    ny, sx, sy, prec = nx, s_, s_, 0
    rng = np.random.default_rng(31)
    res = {}
    for lay in (0, 4):   # autotuned, STREAM with one workgroup per subdomain
        h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, precision=prec, layout=lay,
                           tau_in=0.0, max_wh=3)
        n_if = W.dd_sizes(h)["n_iface"]
        g = rng.standard_normal(n_if) + 1j * rng.standard_normal(n_if)
        rng = np.random.default_rng(31)
        f = np.cos(3 * Xl) * Yl
        res[lay] = (W.dd_layout(h), W.dd_sweep(h, g, f, 1.0))
        W.dd_destroy(h)
    (lay_a, (ga, ua, ia)), (lay_s, (gs, us, is_)) = res[0], res[4]
    print(f"autotuned {lay_a}, single-workgroup {lay_s}", flush=True)
    assert lay_a[0] == 4 and lay_s == (4, 512)
    assert (ia == 3).all() and (is_ == 3).all()
    assert np.array_equal(ga, gs) and np.array_equal(ua, us)


def test_stream_shared_subdomains_solve_matches_oracle_dd(gpu_lib):
    W = gpu_lib
    nx = ny = 96
    P, sx, sy, om = 3, 2, 2, 40.0
    h, Xl, Yl = _setup(W, nx, ny, P, sx, sy, om, _cwave, tau_in=1e-12, max_wh=1000)
    lay = W.dd_layout(h)
    dec, X, Y = _oracle(nx, ny, P, sx, sy, om, _cwave)

    def src(X, Y):
        return np.exp(-((X - 0.41) ** 2 + (Y - 0.63) ** 2) / (2 * 0.05 ** 2))
    u, st, _ = W.dd_solve(h, src(Xl, Yl), None, 1e-8)
    W.dd_destroy(h)
    us_ref, info = dd.solve_dd(dec, src(X, Y), tol=1e-8)
    assert info["passes"] == 1
    err = _rel([u], [dec.glue(us_ref)])
    print(f"layout {lay}: gpu iters={st['outer_iters']} oracle={info['iters']} err={err:.2e}",
          flush=True)
    assert st["outer_iters"] == info["iters"]
    assert err < 1e-10
