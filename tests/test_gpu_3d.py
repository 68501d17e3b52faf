"""GPU parity of the box (hexahedral) path against the FP64 CPU oracle
(``oracle.dd3`` / ``oracle.sem3``) on the same seeded inputs.

Tolerances, as for the 2D sweep (relative l2 over the stacked subdomain
copies): fixed-count WaveHoltz sweep FP64 1e-11, FP32 1e-4; converged sweep
vs sparse LU 1e-9; whole-box operator 1e-13.
"""
import numpy as np
import pytest

from oracle import dd3, sem3
from oracle import waveholtz as wh

pytestmark = pytest.mark.gpu

BOX = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)


def _c3(X, Y, Z):
    return 1.0 + 0.3 * np.sin(2 * X + 0.3) * np.cos(1.5 * Y) * np.cos(Z - 0.2)


def _setup(W, shape, omega, cfun=_c3, **opt):
    nx, ny, nz, P, sx, sy, sz = shape
    X, Y, Z = W.dd3_mesh_coords(nx, ny, nz, P, *BOX)
    o = W.dd_default_options(**opt)
    h = W.dd3_setup(nx, ny, nz, P, cfun(X, Y, Z), omega, sx, sy, sz, *BOX, options=o)
    return h, X, Y, Z


def _oracle(shape, omega, cfun=_c3):
    nx, ny, nz, P, sx, sy, sz = shape
    mesh = sem3.Box(nx, ny, nz, P, *BOX)
    X, Y, Z = sem3.node_coords(mesh)
    dec = dd3.Decomposition3(mesh, dd3.Partition3(sx, sy, sz), cfun(X, Y, Z), omega)
    return dec, X, Y, Z


def _rel(a, b):
    a, b = np.concatenate([np.ravel(x) for x in a]), np.concatenate([np.ravel(x) for x in b])
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _src(X, Y, Z):
    return np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2 + (Z - 0.3) ** 2) / 0.1)


# (nx, ny, nz, P, sx, sy, sz): several subdomains per direction, anisotropic
# blocks, one subdomain, P = 4, a 1000-node subdomain (10^3, close to the
# 1024-thread limit), P = 1 with 9^3 nodes, one element per subdomain.
SHAPES = [(4, 4, 4, 2, 2, 2, 2), (3, 2, 4, 3, 3, 1, 2), (2, 2, 2, 1, 1, 1, 1),
          (4, 4, 2, 4, 2, 2, 1), (6, 3, 3, 3, 2, 1, 1), (16, 8, 8, 1, 2, 1, 1),
          (3, 3, 3, 2, 3, 3, 3)]


@pytest.mark.parametrize("shape", SHAPES)
def test_time_steps_match_oracle(gpu_lib, shape):
    W = gpu_lib
    h, _, _, _ = _setup(W, shape, 6.0)
    nt = W.dd3_time_steps(h)
    W.dd3_destroy(h)
    dec, _, _, _ = _oracle(shape, 6.0)
    assert list(nt) == wh.subdomain_steps(dec)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_fixed_iterations(gpu_lib, shape, prec):
    """One DD cycle with exactly m WaveHoltz iterations from u = 0 on every
    box subdomain: iterates and interface output against the oracle."""
    W = gpu_lib
    om, m = 6.0, 3
    print(f"3d sweep shape={shape} prec={prec}", flush=True)
    h, Xl, Yl, Zl = _setup(W, shape, om, precision=prec, tau_in=0.0, max_wh=m)
    dec, X, Y, Z = _oracle(shape, om)
    rng = np.random.default_rng(sum(shape) + 7 * prec)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    g_gpu, u_gpu, its = W.dd3_sweep(h, g, _src(Xl, Yl, Zl), 1.0)
    W.dd3_destroy(h)
    g_ref, u_ref = dec.sweep(g, _src(X, Y, Z), 1.0, wh.make_solver(dec, fixed_iters=m))
    assert (its == m).all()
    tol = 1e-11 if prec == 0 else 1e-4
    assert _rel([u_gpu], u_ref) < tol
    assert _rel([g_gpu], [g_ref]) < tol
    # outer faces carry physical data: the sweep writes zeros there
    outer = ~dec.interface_mask()
    assert np.all(g_gpu[outer] == 0)


def test_sweep_complex_source_and_src_scale(gpu_lib):
    """Complex f with src = -0.5: b = src (f, phi) enters linearly."""
    W = gpu_lib
    shape, om, m = (4, 4, 4, 2, 2, 2, 2), 6.0, 2
    h, Xl, Yl, Zl = _setup(W, shape, om, tau_in=0.0, max_wh=m)
    dec, X, Y, Z = _oracle(shape, om)
    f = _src(X, Y, Z) * (1.0 - 0.7j)
    fl = _src(Xl, Yl, Zl) * (1.0 - 0.7j)
    g_gpu, u_gpu, _ = W.dd3_sweep(h, None, fl, -0.5)
    W.dd3_destroy(h)
    g_ref, u_ref = dec.sweep(np.zeros(dec.n_if), f, -0.5, wh.make_solver(dec, fixed_iters=m))
    assert _rel([u_gpu], u_ref) < 1e-11
    assert _rel([g_gpu], [g_ref]) < 1e-11


def test_sweep_zero_data_gives_zero(gpu_lib):
    W = gpu_lib
    h, _, _, _ = _setup(W, (4, 4, 4, 2, 2, 2, 2), 6.0, tau_in=0.0, max_wh=2)
    g, u, _ = W.dd3_sweep(h, None, None, 1.0)
    W.dd3_destroy(h)
    assert np.all(g == 0) and np.all(u == 0)


def test_sweep_converged_matches_lu(gpu_lib):
    """With the inner tolerance 1e-12, every subdomain's WaveHoltz result is
    its impedance problem's solution (oracle sparse LU)."""
    W = gpu_lib
    shape, om = (4, 4, 4, 2, 2, 2, 2), 6.0
    h, Xl, Yl, Zl = _setup(W, shape, om, tau_in=1e-12, max_wh=200)
    dec, X, Y, Z = _oracle(shape, om)
    rng = np.random.default_rng(11)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    g_gpu, u_gpu, its = W.dd3_sweep(h, g, _src(Xl, Yl, Zl), 1.0)
    W.dd3_destroy(h)
    g_ref, u_ref = dec.sweep(g, _src(X, Y, Z), 1.0)
    assert _rel([u_gpu], u_ref) < 1e-9
    assert _rel([g_gpu], [g_ref]) < 1e-9
    # the stop rule (Sec. V): the same WaveHoltz iteration count per
    # subdomain as the oracle's WaveHoltz under the same rule
    counts = []
    _, u_wh = dec.sweep(g, _src(X, Y, Z), 1.0, wh.make_solver(dec, tol=1e-12, max_iter=200,
                                                               counts=counts))
    print(f"box WaveHoltz counts GPU {its.tolist()}, oracle {counts}", flush=True)
    assert its.tolist() == counts
    assert _rel([u_gpu], u_wh) < 1e-11


def test_sweep_is_deterministic(gpu_lib):
    W = gpu_lib
    shape = (6, 3, 3, 3, 2, 1, 1)
    h, Xl, Yl, Zl = _setup(W, shape, 6.0, tau_in=1e-10, max_wh=50)
    rng = np.random.default_rng(2)
    n_if = W.dd3_sizes(h)["n_iface"]
    g = rng.standard_normal(n_if) + 1j * rng.standard_normal(n_if)
    a = W.dd3_sweep(h, g, _src(Xl, Yl, Zl), 1.0)
    b = W.dd3_sweep(h, g, _src(Xl, Yl, Zl), 1.0)
    W.dd3_destroy(h)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("nx,ny,nz,P", [(3, 4, 5, 3), (20, 6, 3, 2), (70, 3, 2, 1),
                                        (4, 3, 3, 4), (20, 4, 40, 3)])
def test_operator(gpu_lib, nx, ny, nz, P):
    """Whole-box S x against the oracle's assembled S: ragged 64 x 4 column
    tiles, several z chunks (the last shape: 40 workgroups, so the XCD tile
    numbering is active)."""
    import torch
    W = gpu_lib
    X, Y, Z = W.dd3_mesh_coords(nx, ny, nz, P, *BOX)
    o = W.dd_default_options()
    # one subdomain may exceed the sweep's 1024-node limit: set up with a
    # partition into single-element blocks (the operator is global)
    h = W.dd3_setup(nx, ny, nz, P, _c3(X, Y, Z), 5.0, nx, ny, nz, *BOX, options=o)
    mesh = sem3.Box(nx, ny, nz, P, *BOX)
    Xo, Yo, Zo = sem3.node_coords(mesh)
    S, _, _, _ = sem3.system(mesh, _c3(Xo, Yo, Zo), 5.0)
    rng = np.random.default_rng(nx + ny + nz + P)
    x = rng.standard_normal(mesh.N) + 1j * rng.standard_normal(mesh.N)
    xt = torch.from_numpy(np.stack([x.real, x.imag], 1).ravel()).cuda()
    yt = torch.empty_like(xt)
    W.dd3_apply_operator_device(h, xt, yt)
    torch.cuda.synchronize()
    W.dd3_destroy(h)
    y = yt.cpu().numpy()
    y = y[0::2] + 1j * y[1::2]
    ref = S @ x
    assert np.linalg.norm(y - ref) < 1e-13 * np.linalg.norm(ref)


def test_time_sweep_reports_dof_updates(gpu_lib):
    W = gpu_lib
    shape = (8, 8, 8, 2, 4, 4, 4)
    h, _, _, _ = _setup(W, shape, 6.0)
    ms, du = W.dd3_time_sweep(h, reps=3, fixed_iters=5)
    nt = W.dd3_time_steps(h)
    s = W.dd3_sizes(h)
    W.dd3_destroy(h)
    assert ms > 0
    assert du == pytest.approx(float(np.sum(s["n_local"] * (nt - 1) * 5)))


def _box_workload_setup(W, wl, prec, m):
    X, Y, Z = W.dd3_mesh_coords(wl.nx, wl.ny, wl.nz, wl.P, *wl.box)
    o = W.dd_default_options(precision=prec, tau_in=0.0, max_wh=m)
    h = W.dd3_setup(wl.nx, wl.ny, wl.nz, wl.P, wl.c(X, Y, Z), wl.omega, wl.sx, wl.sy, wl.sz,
                    *wl.box, options=o)
    return h, X, Y, Z


@pytest.mark.parametrize("prec", [0, 1])
def test_c6_small_protocol_sweep(gpu_lib, prec):
    """The c6 subdomain shape (2^3 elements, P=3, 343 nodes) at 8^3 elements:
    one DD cycle of the paper's 5 WaveHoltz iterations against the oracle."""
    import workloads
    W = gpu_lib
    wl = workloads.c6_small()
    h, Xl, Yl, Zl = _box_workload_setup(W, wl, prec, 5)
    mesh = sem3.Box(wl.nx, wl.ny, wl.nz, wl.P, *wl.box)
    X, Y, Z = sem3.node_coords(mesh)
    dec = dd3.Decomposition3(mesh, dd3.Partition3(wl.sx, wl.sy, wl.sz), wl.c(X, Y, Z), wl.omega)
    rng = np.random.default_rng(6)
    g = rng.standard_normal(dec.n_if) + 1j * rng.standard_normal(dec.n_if)
    g_gpu, u_gpu, its = W.dd3_sweep(h, g, wl.f(Xl, Yl, Zl), 1.0)
    W.dd3_destroy(h)
    g_ref, u_ref = dec.sweep(g, wl.f(X, Y, Z), 1.0, wh.make_solver(dec, fixed_iters=5))
    assert (its == 5).all()
    tol = 1e-11 if prec == 0 else 1e-4
    assert _rel([u_gpu], u_ref) < tol
    assert _rel([g_gpu], [g_ref]) < tol


@pytest.mark.parametrize("name", ["c6", "c6_p1"])
@pytest.mark.parametrize("prec", [0, 1])
def test_c6_full_size_sweep_sampled(gpu_lib, prec, name):
    """The full box launches of the bench (c6: 64^3 elements, P=3, 32768
    subdomains; c6_p1: 128^3 elements, P=1, 4096 subdomains) checked on
    sampled subdomains: each sampled subdomain's WaveHoltz iterate equals
    the oracle's on that subdomain alone (a one-subdomain decomposition of
    its box with its slice of g), and the interface data it sends to every
    neighbour equals -g - 2i(omega/c)u."""
    import workloads
    W = gpu_lib
    wl = workloads.CONFIGS3[name]()
    h, Xl, Yl, Zl = _box_workload_setup(W, wl, prec, 5)
    s = W.dd3_sizes(h)
    rng = np.random.default_rng(66)
    g = rng.standard_normal(s["n_iface"]) + 1j * rng.standard_normal(s["n_iface"])
    print(f"{name} full-size sweep prec={prec}", flush=True)
    g_gpu, u_gpu, its = W.dd3_sweep(h, g, wl.f(Xl, Yl, Zl), 1.0)
    W.dd3_destroy(h)
    assert (its == 5).all()
    P, L, nloc, per = wl.P, s["n_sub"], s["n_local"], s["n_iface"] // s["n_sub"]
    mx, my, mz = wl.nx // wl.sx, wl.ny // wl.sy, wl.nz // wl.sz
    hx = (wl.box[1] - wl.box[0]) / wl.nx
    hy = (wl.box[3] - wl.box[2]) / wl.ny
    hz = (wl.box[5] - wl.box[4]) / wl.nz
    tol = 1e-11 if prec == 0 else 1e-4
    for l in (0, L // 2 + 17 * wl.sx + 5, L - 1):
        a, b, c = l % wl.sx, (l // wl.sx) % wl.sy, l // (wl.sx * wl.sy)
        x0, y0, z0 = wl.box[0] + a * mx * hx, wl.box[2] + b * my * hy, wl.box[4] + c * mz * hz
        sub = sem3.Box(mx, my, mz, P, x0, x0 + mx * hx, y0, y0 + my * hy, z0, z0 + mz * hz)
        X, Y, Z = sem3.node_coords(sub)
        one = dd3.Decomposition3(sub, dd3.Partition3(1, 1, 1), wl.c(X, Y, Z), wl.omega)
        gl = g[l * per:(l + 1) * per]
        b_l = one.rhs(0, wl.f(X, Y, Z), gl, 1.0)
        u_ref = wh.make_solver(one, fixed_iters=5)(0, b_l)
        u_l = u_gpu[l * nloc:(l + 1) * nloc]
        assert _rel([u_l], [u_ref]) < tol, l
        for face in range(6):
            step = dd3.STEP[face]
            a2, b2, c2 = a + step[0], b + step[1], c + step[2]
            if not (0 <= a2 < wl.sx and 0 <= b2 < wl.sy and 0 <= c2 < wl.sz):
                continue
            r = (c2 * wl.sy + b2) * wl.sx + a2
            o2 = one.face_off[dd3.OPPOSITE[face]]
            nodes = one.local_faces[face]
            sent = g_gpu[r * per + o2:r * per + o2 + one.face_len[face]]
            want = (-gl[one.face_off[face]:one.face_off[face] + one.face_len[face]]
                    - 2j * (wl.omega / one.subs[0]["c"][nodes]) * u_ref[nodes])
            assert _rel([sent], [want]) < tol, (l, face)


def test_solve_matches_oracle_dd(gpu_lib):
    """Outer FP64 GMRES over box sweeps (WaveHoltz to 1e-12) against the
    oracle's DD with exact subdomain solves at the same outer tolerance."""
    from oracle import dd
    W = gpu_lib
    shape, om, tol = (4, 4, 4, 2, 2, 2, 2), 6.0, 1e-8
    h, Xl, Yl, Zl = _setup(W, shape, om, tau_in=1e-12, max_wh=1000)
    dec, X, Y, Z = _oracle(shape, om)
    u, st, _ = W.dd3_solve(h, _src(Xl, Yl, Zl), tol)
    rel_res = W.dd3_residual(h, u, _src(Xl, Yl, Zl))
    W.dd3_destroy(h)
    us_ref, info = dd.solve_dd(dec, _src(X, Y, Z), tol=tol)
    err = _rel([u], [dec.glue(us_ref)])
    print(f"box solve gpu iters={st['outer_iters']} oracle iters={info['iters']} "
          f"wh_max={st['wh_iters_max']} err={err:.2e}", flush=True)
    assert info["passes"] == 1
    assert st["outer_iters"] == info["iters"]
    assert err < 1e-10
    assert st["true_rel_residual"] < 2 * tol
    S, _, _, _ = sem3.system(dec.mesh, _c3(X, Y, Z), om)
    b = sem3.load(dec.mesh, _src(X, Y, Z))
    assert rel_res == pytest.approx(np.linalg.norm(b - S @ u) / np.linalg.norm(b), rel=1e-9)


def test_solve_tight_matches_global_lu(gpu_lib):
    W = gpu_lib
    shape, om = (3, 2, 4, 3, 3, 1, 2), 6.0
    h, Xl, Yl, Zl = _setup(W, shape, om, tau_in=1e-14, max_wh=1000)
    mesh = sem3.Box(*shape[:4], *BOX)
    X, Y, Z = sem3.node_coords(mesh)
    u, st, _ = W.dd3_solve(h, _src(Xl, Yl, Zl) * (1 + 0.5j), 1e-12)
    rel_res = W.dd3_residual(h, u, _src(Xl, Yl, Zl) * (1 + 0.5j))
    W.dd3_destroy(h)
    u_lu = sem3.solve(mesh, _c3(X, Y, Z), om, _src(X, Y, Z) * (1 + 0.5j))
    assert _rel([u], [u_lu]) < 1e-10
    assert rel_res < 1e-10


def test_solve_fp32_sweeps_plain(gpu_lib):
    """FP32 box sweeps under the FP64 outer GMRES without refinement reach
    the answer to the FP32 sweep accuracy."""
    W = gpu_lib
    shape, om = (4, 4, 4, 2, 2, 2, 2), 6.0
    h, Xl, Yl, Zl = _setup(W, shape, om, precision=1, tau_in=1e-6, max_wh=400, refine=0)
    mesh = sem3.Box(*shape[:4], *BOX)
    X, Y, Z = sem3.node_coords(mesh)
    u, st, rc = W.dd3_solve(h, _src(Xl, Yl, Zl), 1e-5, allow_notconv=True)
    W.dd3_destroy(h)
    u_lu = sem3.solve(mesh, _c3(X, Y, Z), om, _src(X, Y, Z))
    print(f"box fp32 rc={rc} iters={st['outer_iters']} err={_rel([u], [u_lu]):.2e}", flush=True)
    assert _rel([u], [u_lu]) < 1e-4


def test_c6_small_solve_matches_oracle_dd(gpu_lib):
    """The c6 subdomain shape at 8^3 elements: box solve on the GPU against the
    oracle DD (exact subdomain solves)."""
    import workloads
    from oracle import dd
    W = gpu_lib
    wl = workloads.c6_small()
    X, Y, Z = W.dd3_mesh_coords(wl.nx, wl.ny, wl.nz, wl.P, *wl.box)
    o = W.dd_default_options(tau_in=1e-12, max_wh=1000)
    h = W.dd3_setup(wl.nx, wl.ny, wl.nz, wl.P, wl.c(X, Y, Z), wl.omega, wl.sx, wl.sy, wl.sz,
                    *wl.box, options=o)
    u, st, _ = W.dd3_solve(h, wl.f(X, Y, Z), 1e-8)
    W.dd3_destroy(h)
    mesh = sem3.Box(wl.nx, wl.ny, wl.nz, wl.P, *wl.box)
    Xo, Yo, Zo = sem3.node_coords(mesh)
    dec = dd3.Decomposition3(mesh, dd3.Partition3(wl.sx, wl.sy, wl.sz), wl.c(Xo, Yo, Zo), wl.omega)
    us_ref, info = dd.solve_dd(dec, wl.f(Xo, Yo, Zo), tol=1e-8)
    err = _rel([u], [dec.glue(us_ref)])
    print(f"c6_small solve gpu iters={st['outer_iters']} oracle iters={info['iters']} "
          f"wh_max={st['wh_iters_max']} err={err:.2e}", flush=True)
    assert info["passes"] == 1
    assert st["outer_iters"] == info["iters"]
    assert err < 1e-10


def test_solve_zero_source_and_bad_arguments(gpu_lib):
    """No source: u = 0 without outer iterations; bad tolerances, iteration
    counts and non-finite sources are rejected before any device work."""
    W = gpu_lib
    h, _, _, _ = _setup(W, (4, 4, 4, 2, 2, 2, 2), 6.0)
    u, st, rc = W.dd3_solve(h, None, 1e-8)
    assert rc == 0 and st["outer_iters"] == 0 and np.all(u == 0)
    for tol, it in ((0.0, 10), (1e-8, 0)):
        with pytest.raises(W.WaveddError) as ei:
            W.dd3_solve(h, None, tol, it)
        assert ei.value.code == W.DD_EINVAL
    n = W.dd3_sizes(h)["n_global"]
    f = np.ones(n)
    f[3] = np.nan
    with pytest.raises(W.WaveddError) as ei:
        W.dd3_solve(h, f, 1e-8)
    assert ei.value.code == W.DD_ENAN
    W.dd3_destroy(h)


@pytest.mark.parametrize("shape", [(4, 4, 4, 2, 2, 2, 2), (3, 2, 4, 3, 3, 1, 2)])
def test_solve_fp32_refined_matches_fp64(gpu_lib, shape):
    """FP32 box sweeps with FP64 iterative refinement: the same outer
    tolerance as the FP64 oracle DD, and the answer within 1e-6 of it."""
    from oracle import dd
    W = gpu_lib
    om, tol = 6.0, 1e-8
    h, Xl, Yl, Zl = _setup(W, shape, om, precision=1, tau_in=1e-6, max_wh=400)
    u, st, rc = W.dd3_solve(h, _src(Xl, Yl, Zl), tol)
    W.dd3_destroy(h)
    dec, X, Y, Z = _oracle(shape, om)
    us_ref, info = dd.solve_dd(dec, _src(X, Y, Z), tol=tol)
    err = _rel([u], [dec.glue(us_ref)])
    print(f"box fp32 refined rc={rc} iters={st['outer_iters']} refine={st['refine_steps']} "
          f"true={st['true_rel_residual']:.2e} err={err:.2e}", flush=True)
    assert rc == 0 and st["true_rel_residual"] <= tol
    assert st["refine_steps"] >= 2
    assert err < 1e-6



@pytest.mark.parametrize("prec", [0, 1])
def test_solve_relaxed_inner_tolerance(gpu_lib, prec):
    """Variable inner tolerance (relax = 0.1) with FP64 refinement: the same
    answer as the strict FP64 solve at the outer tolerance, with fewer
    WaveHoltz iterations."""
    W = gpu_lib
    shape, om, tol = (4, 4, 4, 2, 2, 2, 2), 6.0, 1e-8
    h, Xl, Yl, Zl = _setup(W, shape, om, tau_in=1e-12, max_wh=400)
    u0, st0, _ = W.dd3_solve(h, _src(Xl, Yl, Zl), tol)
    W.dd3_destroy(h)
    tau = 1e-12 if prec == 0 else 1e-5
    h, Xl, Yl, Zl = _setup(W, shape, om, precision=prec, tau_in=tau, max_wh=400, relax=0.1)
    u, st, rc = W.dd3_solve(h, _src(Xl, Yl, Zl), tol)
    W.dd3_destroy(h)
    print(f"box relax prec={prec} rc={rc} iters={st['outer_iters']} refine={st['refine_steps']} "
          f"wh={st['wh_iters_total']} vs strict {st0['wh_iters_total']} diff={_rel([u], [u0]):.2e}",
          flush=True)
    assert rc == 0 and st["true_rel_residual"] <= tol
    assert _rel([u], [u0]) < 1e-6
    if prec == 0:
        assert st["wh_iters_total"] < st0["wh_iters_total"]
