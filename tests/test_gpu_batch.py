"""GPU: batched launches (the subdomains of several problems in one launch)
and the serving engine, through the C ABI, against single-problem solves of
the same problems and against the oracle.

A batched launch runs each subdomain's work item exactly as a launch of its
own problem does (same kernel, same data, same per-item WaveHoltz
tolerance), and every problem keeps its own outer iteration, so with the
same layout the batched solution equals the single-problem solution bit
for bit; the oracle bar is the single-solve bar (FP64 1e-10 at equal outer
tolerance)."""
import numpy as np
import pytest

from oracle import dd, sem

pytestmark = pytest.mark.gpu

# nx, ny, P, sx, sy, omega, box: mixed degrees, shapes and layouts; the last
# has 24x24-element subdomains (5329 nodes), which only STREAM holds
SPECS = [
    (8, 8, 2, 2, 2, 10.0, (0.0, 1.0, 0.0, 1.0)),
    (6, 4, 3, 2, 2, 9.0, (0.0, 1.5, 0.0, 1.0)),
    (4, 6, 1, 2, 3, 6.0, (0.0, 1.0, 0.0, 1.0)),
    (4, 4, 4, 2, 1, 8.0, (0.2, 1.2, 0.0, 1.0)),
    (48, 24, 3, 2, 1, 20.0, (0.0, 2.0, 0.0, 1.0)),
]


def _c(X, Y):
    return 1.0 + 0.3 * np.sin(4 * X + 0.5) * np.cos(3 * Y - 0.1)


def _f(X, Y, k):
    x0, y0 = X.min() + 0.37 * (X.max() - X.min()), Y.min() + (0.3 + 0.1 * k) * (Y.max() - Y.min())
    return np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * 0.06 ** 2))


def _spec(W, k):
    nx, ny, P, sx, sy, om, box = SPECS[k]
    X, Y = W.dd_mesh_coords(nx, ny, P, *box)
    return dict(nx=nx, ny=ny, P=P, x0=box[0], x1=box[1], y0=box[2], y1=box[3], sx=sx, sy=sy,
                omega=om, c=_c(X, Y), f=_f(X, Y, k), X=X, Y=Y)


def _single(W, s, tol, **opt):
    o = W.dd_default_options(**opt)
    h = W.dd_setup(s["nx"], s["ny"], s["P"], s["c"], s["omega"], s["sx"], s["sy"], s["x0"],
                   s["x1"], s["y0"], s["y1"], o)
    u, st, _ = W.dd_solve(h, s["f"], None, tol)
    W.dd_destroy(h)
    return u, st


@pytest.mark.parametrize("tc2", [0.0, 0.1])
def test_batch_matches_single_solves(gpu_lib, tc2):
    """Batched solves equal single-problem solves bit for bit, with the
    paper's transmission condition and with the second-order one."""
    W = gpu_lib
    specs = [_spec(W, k) for k in range(len(SPECS))]
    o = W.dd_default_options(tau_in=1e-12, tc2=tc2)
    b = W.dd_batch_setup(specs, o)
    try:
        lays = [W.dd_layout(W.dd_batch_handle(b, i))[0] for i in range(len(specs))]
        print(f"batch layouts {lays}", flush=True)
        assert lays[-1] == W.DD_LAYOUT_STREAM
        us, sts, rcs, rc = W.dd_batch_solve(b, [s["f"] for s in specs], 1e-8)
        launches = W.dd_batch_launches(b)
    finally:
        W.dd_batch_destroy(b)
    assert rc == W.DD_OK and all(r == W.DD_OK for r in rcs)
    # a launch carries at most one sweep of each problem and may carry several
    # problems' sweeps
    assert max(st["sweeps"] for st in sts) <= launches <= sum(st["sweeps"] for st in sts)
    for i, s in enumerate(specs):
        u1, st1 = _single(W, s, 1e-8, tau_in=1e-12, layout=lays[i], tc2=tc2)
        print(f"problem {i}: batch iters {sts[i]['outer_iters']} single {st1['outer_iters']}",
              flush=True)
        assert sts[i]["outer_iters"] == st1["outer_iters"]
        assert np.array_equal(us[i], u1), i


@pytest.mark.parametrize("k", [0, 3, 4])
def test_batch_matches_oracle(gpu_lib, k):
    W = gpu_lib
    specs = [_spec(W, i) for i in range(len(SPECS))]
    b = W.dd_batch_setup(specs, W.dd_default_options(tau_in=1e-12))
    try:
        us, sts, rcs, rc = W.dd_batch_solve(b, [s["f"] for s in specs], 1e-8)
    finally:
        W.dd_batch_destroy(b)
    s = specs[k]
    mesh = sem.Rect(s["nx"], s["ny"], s["P"], s["x0"], s["x1"], s["y0"], s["y1"])
    X, Y = sem.node_coords(mesh)
    dec = dd.Decomposition(mesh, dd.Partition(s["sx"], s["sy"]), _c(X, Y), s["omega"])
    us_ref, info = dd.solve_dd(dec, _f(X, Y, k), tol=1e-8)
    assert sts[k]["outer_iters"] == info["iters"]
    u_ref = dec.glue(us_ref)
    assert np.linalg.norm(us[k] - u_ref) / np.linalg.norm(u_ref) < 1e-10


def test_batch_fp32_relaxed_reaches_tolerance(gpu_lib):
    W = gpu_lib
    specs = [_spec(W, i) for i in range(len(SPECS))]
    b = W.dd_batch_setup(specs, W.dd_default_options(precision=W.DD_FP32, tau_in=1e-6, relax=0.1))
    try:
        us, sts, rcs, rc = W.dd_batch_solve(b, [s["f"] for s in specs], 1e-8)
        res = [W.dd_residual(W.dd_batch_handle(b, i), us[i], specs[i]["f"])
               for i in range(len(specs))]
    finally:
        W.dd_batch_destroy(b)
    assert rc == W.DD_OK
    for i, s in enumerate(specs):
        u64, _ = _single(W, s, 1e-8, tau_in=1e-12)
        assert np.linalg.norm(us[i] - u64) / np.linalg.norm(u64) < 1e-6, i
        assert sts[i]["true_rel_residual"] <= 1e-8
        assert res[i] < 1e-6


def test_batch_time_sweep_counts_dof_updates(gpu_lib):
    W = gpu_lib
    specs = [_spec(W, i) for i in range(len(SPECS))]
    b = W.dd_batch_setup(specs)
    try:
        expect = 0.0
        for i in range(len(specs)):
            h = W.dd_batch_handle(b, i)
            nt = W.dd_time_steps(h)
            expect += W.dd_sizes(h)["n_local"] * float((nt - 1).sum()) * 3
        ms, dof, launches = W.dd_batch_time_sweep(b, reps=2, fixed_iters=3)
    finally:
        W.dd_batch_destroy(b)
    assert ms > 0 and launches >= 1
    assert dof == expect


def _engine_run(W, specs, order, budget=4 << 30, max_active=3, **opt):
    e = W.dd_engine_create(budget, max_active, W.dd_default_options(**opt))
    try:
        ids = [W.dd_engine_submit(e, specs[k], specs[k]["f"], 1e-8) for k in order]
        out = [W.dd_engine_wait(e, rid, specs[k]["c"].size) for rid, k in zip(ids, order)]
        info = W.dd_engine_get_info(e)
    finally:
        W.dd_engine_destroy(e)
    return out, info


def test_engine_mix_matches_alone_and_single(gpu_lib):
    """Each request's answer is the same in a mix of concurrent requests, in
    the engine alone, and from a plain dd_solve (layout fixed to STREAM so
    all three launch identical work items)."""
    W = gpu_lib
    specs = [_spec(W, i) for i in range(len(SPECS))]
    order = [4, 0, 1, 2, 3, 1, 0]
    mix, info = _engine_run(W, specs, order, tau_in=1e-12, layout=W.DD_LAYOUT_STREAM)
    print(f"engine info {info}", flush=True)
    assert info["done"] == len(order) and info["peak_running"] <= 3
    assert all(rc == W.DD_OK for *_, rc in mix)
    alone, _ = _engine_run(W, specs, [1], tau_in=1e-12, layout=W.DD_LAYOUT_STREAM)
    assert np.array_equal(alone[0][0], mix[2][0]) and np.array_equal(mix[2][0], mix[5][0])
    for (u, st, times, rc), k in zip(mix, order):
        u1, st1 = _single(W, specs[k], 1e-8, tau_in=1e-12, layout=W.DD_LAYOUT_STREAM)
        assert st["outer_iters"] == st1["outer_iters"], k
        assert np.array_equal(u, u1), k
        assert times[0] <= times[1] <= times[2]


def test_engine_wait_any_returns_each_request_once(gpu_lib):
    """wait_any hands out every finished request once; with none left that
    it has not returned (or none outstanding) it fails instead of blocking."""
    W = gpu_lib
    specs = [_spec(W, i) for i in range(2)]
    e = W.dd_engine_create(1 << 30, 2, W.dd_default_options(tau_in=1e-10))
    try:
        ids = [W.dd_engine_submit(e, specs[k], specs[k]["f"], 1e-8) for k in (0, 1)]
        got = sorted(W.dd_engine_wait_any(e) for _ in ids)
        assert got == sorted(ids)
        with pytest.raises(W.WaveddError):
            W.dd_engine_wait_any(e)
        for rid, k in zip(ids, (0, 1)):
            *_, rc = W.dd_engine_wait(e, rid, specs[k]["c"].size)
            assert rc == W.DD_OK
        with pytest.raises(W.WaveddError):
            W.dd_engine_wait_any(e)
    finally:
        W.dd_engine_destroy(e)


def test_engine_admission_under_a_small_budget(gpu_lib):
    """A 64 MiB engine admits requests as memory frees up and rejects one
    larger than all it holds."""
    W = gpu_lib
    specs = [_spec(W, i) for i in range(4)]
    out, info = _engine_run(W, specs, [0, 1, 2, 3, 0, 1], budget=64 << 20, max_active=8,
                            tau_in=1e-12)
    assert info["done"] == 6 and all(rc == W.DD_OK for *_, rc in out)
    e = W.dd_engine_create(64 << 20, 2)
    try:
        nx = ny = 400
        X, Y = W.dd_mesh_coords(nx, ny, 2)
        big = dict(nx=nx, ny=ny, P=2, x0=0.0, x1=1.0, y0=0.0, y1=1.0, sx=8, sy=8, omega=10.0,
                   c=np.ones(X.size))
        with pytest.raises(W.WaveddError) as ei:
            W.dd_engine_submit(e, big, None, 1e-6)
        assert ei.value.code == W.DD_ENOMEM
    finally:
        W.dd_engine_destroy(e)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_batch_sampled(gpu_lib, prec):
    """The 400-subdomain batch (58 problems, P 1..4, 8..64 elements per
    subdomain side) set up as the benchmark does, one layout per shape from
    the autotuner: for one problem of each layout in use, one sweep of two
    fixed WaveHoltz iterations from random interface data, a corner and the
    last subdomain recomputed by the oracle's WaveHoltz."""
    import workloads
    from oracle import waveholtz as wh
    W = gpu_lib
    wls = workloads.c4()
    specs = [W.workload_spec(wl) for wl in wls]
    m = 2
    b = W.dd_batch_setup(specs, W.dd_default_options(precision=prec, tau_in=0.0, max_wh=m))
    try:
        lays = [W.dd_layout(W.dd_batch_handle(b, i))[0] for i in range(len(wls))]
        picks = sorted({lay: i for i, lay in reversed(list(enumerate(lays)))}.values())
        print(f"layouts {sorted(set(lays))} picks {picks}", flush=True)
        for i in picks:
            wl, s = wls[i], specs[i]
            h = W.dd_batch_handle(b, i)
            sz = W.dd_sizes(h)
            rng = np.random.default_rng(100 + i)
            g = rng.standard_normal(sz["n_iface"]) + 1j * rng.standard_normal(sz["n_iface"])
            g_gpu, u_gpu, its = W.dd_sweep(h, g, s["f"], 1.0)
            assert (its == m).all()
            mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
            X, Y = sem.node_coords(mesh)
            c, f = wl.c(X, Y), wl.f(X, Y)
            mx, my = wl.nx // wl.sx, wl.ny // wl.sy
            nxl, nyl = mx * wl.P + 1, my * wl.P + 1
            per, nloc = 2 * nxl + 2 * nyl, sz["n_local"]
            for l in sorted({0, wl.sx * wl.sy - 1}):
                a_, b_ = l % wl.sx, l // wl.sx
                x0, y0 = wl.x0 + a_ * mx * mesh.hx, wl.y0 + b_ * my * mesh.hy
                sub = sem.Rect(mx, my, wl.P, x0, x0 + mx * mesh.hx, y0, y0 + my * mesh.hy)
                ii = a_ * mx * wl.P + np.arange(nxl)
                jj = b_ * my * wl.P + np.arange(nyl)
                gl = (jj[:, None] * mesh.Nx + ii[None, :]).ravel()
                one = dd.Decomposition(sub, dd.Partition(1, 1), c[gl], wl.omega)
                rhs = one.rhs(0, np.asarray(f[gl], dtype=float), g[l * per:(l + 1) * per], 1.0)
                sd = one.subs[0]
                nt = wh.subdomain_steps(one)[0]
                u_ref, _ = wh.solve(sd["A"], sd["M"], sd["H"], rhs, wl.omega, nt, fixed_iters=m)
                err = np.linalg.norm(u_gpu[l * nloc:(l + 1) * nloc] - u_ref) / np.linalg.norm(u_ref)
                assert err < (1e-11 if prec == 0 else 1e-4), (i, l, lays[i], err)
    finally:
        W.dd_batch_destroy(b)


def _oracle_dd(s, f, tol):
    """The oracle DD of a problem dict (wavespeed and source sampled at the
    oracle's own node coordinates by the given callables)."""
    mesh = sem.Rect(s["nx"], s["ny"], s["P"], s["x0"], s["x1"], s["y0"], s["y1"])
    X, Y = sem.node_coords(mesh)
    dec = dd.Decomposition(mesh, dd.Partition(s["sx"], s["sy"]), s["cfun"](X, Y), s["omega"])
    us, info = dd.solve_dd(dec, f(X, Y), tol=tol)
    # plain GMRES from G = 0: one pass (none for a single subdomain, which
    # has no interface unknowns)
    assert info["passes"] == (1 if s["sx"] * s["sy"] > 1 else 0)
    return dec.glue(us), info


def test_engine_mix_matches_oracle_fp64(gpu_lib):
    """Served FP64 results of a mixed stream (five shapes, P = 1..4, one of
    them STREAM-sized, two submitted twice) against the oracle DD at the
    same outer tolerance: 1e-10 and the same outer iteration count."""
    W = gpu_lib
    specs = [_spec(W, i) for i in range(len(SPECS))]
    order = [4, 0, 1, 2, 3, 1, 0]
    mix, info = _engine_run(W, specs, order, tau_in=1e-12, max_active=4)
    assert info["done"] == len(order)
    refs = {}
    for (u, st, _, rc), k in zip(mix, order):
        if k not in refs:
            s = dict(specs[k], cfun=_c)
            refs[k] = _oracle_dd(s, lambda X, Y, k=k: _f(X, Y, k), 1e-8)
        u_ref, info_ref = refs[k]
        err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
        print(f"served problem {k}: iters {st['outer_iters']} oracle {info_ref['iters']} "
              f"err {err:.2e}", flush=True)
        assert rc == W.DD_OK
        assert st["outer_iters"] == info_ref["iters"], k
        assert err < 1e-10, k


def test_engine_c5_requests_alone_and_mixed_match_oracle(gpu_lib):
    """Twenty requests drawn (seeded) from the serving stream among those of
    at most 60,000 global nodes and 5,000 nodes per subdomain, FP32 sweeps
    with FP64 refinement, served
    together and each alone: every result within 1e-6 of the FP64 oracle DD
    at the same outer tolerance (1e-8 here, so that the bar is tighter than
    the FP32 sweep accuracy), and the mixed result equal to the alone result
    to the same bar (bitwise where both runs chose the same layout)."""
    import workloads
    W = gpu_lib
    cand = [wl for wl in workloads.c5(n_requests=2000)
            if (wl.nx * wl.P + 1) * (wl.ny * wl.P + 1) <= 60000
            and ((wl.nx // wl.sx) * wl.P + 1) * ((wl.ny // wl.sy) * wl.P + 1) <= 5000]
    rng = np.random.default_rng(55)
    pick = [cand[i] for i in sorted(rng.choice(len(cand), 20, replace=False))]
    specs = [W.workload_spec(wl) for wl in pick]
    tol = 1e-8
    opt = dict(precision=W.DD_FP32, tau_in=1e-5, max_wh=1000)
    e = W.dd_engine_create(8 << 30, 8, W.dd_default_options(**opt))
    try:
        ids = [W.dd_engine_submit(e, s, s["f"], tol, 3000) for s in specs]
        mix = [W.dd_engine_wait(e, rid, s["c"].size) for rid, s in zip(ids, specs)]
        info = W.dd_engine_get_info(e)
    finally:
        W.dd_engine_destroy(e)
    print(f"c5 sample: {len(specs)} requests, nodes {[s['c'].size for s in specs]}, "
          f"peak running {info['peak_running']}", flush=True)
    for k, (s, wl) in enumerate(zip(specs, pick)):
        e = W.dd_engine_create(8 << 30, 1, W.dd_default_options(**opt))
        try:
            rid = W.dd_engine_submit(e, s, s["f"], tol, 3000)
            alone = W.dd_engine_wait(e, rid, s["c"].size)
        finally:
            W.dd_engine_destroy(e)
        u_ref, _ = _oracle_dd(dict(s, cfun=wl.c), wl.f, tol)
        u_mix, u_alone = mix[k][0], alone[0]
        e_mix = np.linalg.norm(u_mix - u_ref) / np.linalg.norm(u_ref)
        e_alone = np.linalg.norm(u_alone - u_ref) / np.linalg.norm(u_ref)
        d = np.linalg.norm(u_mix - u_alone) / np.linalg.norm(u_alone)
        print(f"request {wl.name}: n={wl.nx} P={wl.P} {wl.sx}x{wl.sy} subdomains, "
              f"omega={wl.omega:.1f}: mix vs oracle {e_mix:.2e}, alone vs oracle {e_alone:.2e}, "
              f"mix vs alone {d:.2e}", flush=True)
        assert mix[k][3] == W.DD_OK and alone[3] == W.DD_OK
        assert e_mix < 1e-6 and e_alone < 1e-6 and d < 1e-6, k
