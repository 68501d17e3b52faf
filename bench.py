"""Benchmark: full DD solves of the 256x256-element, P=3 Y-waveguide problem
(16x16 subdomains of 16x16 elements, FP64, outer tolerance 1e-8) on one
MI355X.

A step is one dd_solve (outer GMRES over sweep launches, every subdomain's
WaveHoltz solve in each launch) with inputs resident in HBM.  Prints one JSON
line: WaveHoltz DOF-updates/s (value), solves/s and p50/p99 latency, the
roofline of the sweep kernel (algorithmic FLOP per launch / average launch
time measured with HIP events on the library's stream) and the oracle timed
on the host CPU on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2|c3|c1]
                    [--precision fp64|fp32] [--no-cpu]
    python bench.py --config c4      batched solves of 400 subdomains
    python bench.py --serve          serving engine on a Poisson request stream
    python bench.py --config c6      box (3D) DD cycle of 5 WaveHoltz iterations
                                     against the whole-box operator
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}   # MI355X vector ALU peaks

# HBM bytes per sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled by
# a 256 MiB copy: fetch x2.000, write x1.000), keyed by the hash of the
# kernel's code (its layout section plus the shared helpers, comments
# ignored) and the run; reported as null once that code changes.
MEASURED_TRAFFIC = {
    ("7b4a3859ee1e88a9", "solve", "c2", "fp64"): round((15405.7 * 2.0 + 15651.4) * 1024),
    ("6a3c53d4b8a9ebae", "protocol", "c3", "fp64"): round((40715903.3 * 2.0 + 50894355.0) * 1024),
}

# HBM bytes per launch of the box (3D) sweep kernel, same counters and scale,
# keyed by the hash of the box kernel source (comments ignored).
MEASURED_TRAFFIC3 = {
    ("92c1ab59dbfb4a70", "c6", "fp64"): round((473142.4 * 2.0 + 437807.2) * 1024),
}

# section markers of each layout in the kernel source
_SECTIONS = {1: ("// NODE layout (one DOF per thread)", "// STREAM layout"),
             2: ("// PATCH layout, one barrier per step", "// NODE layout (one DOF per thread)"),
             3: ("// PATCH layout\n", "// PATCH layout, one barrier per step"),
             4: ("// STREAM layout", "}  // namespace\n")}
LAYOUT_NAMES = {1: "node", 2: "patch", 3: "patch_xchg", 4: "stream"}
LAYOUT_IDS = {"auto": 0, **{v: k for k, v in LAYOUT_NAMES.items()}}


def kernel_name(lay, wg):
    """Kernel a layout runs; a STREAM subdomain of more than one workgroup
    (threads per subdomain above 1024) runs the cooperative build."""
    if lay == 4 and wg > 1024:
        return "sweep_stream_coop_kernel"
    return KERNEL_NAMES[lay]
KERNEL_NAMES = {1: "sweep_node_kernel", 2: "sweep_patch1_kernel", 3: "sweep_patch_kernel",
                4: "sweep_stream_kernel"}


def kernel_hash(layout, src=None):
    """Hash of the code (comments and blank lines dropped) of the shared
    device helpers plus the given layout's section."""
    import hashlib
    import re
    if src is None:
        src = open(os.path.join(ROOT, "paper_2606_21695_amd", "csrc", "sweep_kernels.hip")).read()
    head = src[:src.index("// PATCH layout\n")]
    a, b = _SECTIONS[layout]
    i = src.index(a)
    body = src[i:src.index(b, i + len(a))]
    code = [re.sub(r"//.*$", "", line).rstrip() for line in (head + body).splitlines()]
    return hashlib.sha256("\n".join(x for x in code if x).encode()).hexdigest()[:16]


def kernel3_hash():
    """Hash of the box sweep kernel source (comments and blank lines dropped)."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_2606_21695_amd", "csrc", "sweep3_kernels.hip")).read()
    code = [re.sub(r"//.*$", "", line).rstrip() for line in src.splitlines()]
    return hashlib.sha256("\n".join(x for x in code if x).encode()).hexdigest()[:16]


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(msg, file=sys.stderr, flush=True)


def flops_per_update(P):
    """Algorithmic FLOP of one DOF-update (one leapfrog step of one node):
    stiffness 4(P+2) + 3, p update 2, velocity update 7, filter 4."""
    return 4 * (P + 2) + 16


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, the CPUs this
    process may use, memory."""
    info = {"cpu_model": None, "nproc": os.cpu_count(), "ram_gib": None}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity_cpus"] = os.cpu_count()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    info["ram_gib"] = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return info


def oracle_setup(wl):
    """The oracle's mesh, node coordinates, wavespeed and source of a 2D
    workload (sampled at the oracle's own node coordinates)."""
    from oracle import sem
    mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    X, Y = sem.node_coords(mesh)
    return mesh, wl.c(X, Y), wl.f(X, Y)


def cpu_baseline_dd(wl, tol, workers=None):
    """The oracle DD (exact sparse-LU subdomain solves, the same restarted
    GMRES from G = 0, the same outer tolerance) on a pool of host processes,
    one BLAS thread each: subdomain factorisation time, then one full solve
    timed.  Returns (baseline dict, glued oracle solution)."""
    from oracle import dd, pool
    mesh, c, f = oracle_setup(wl)
    t0 = time.perf_counter()
    pdec = pool.ParallelDecomposition(mesh, dd.Partition(wl.sx, wl.sy), c, wl.omega,
                                      workers=workers)
    try:
        pdec.factor()
        setup_s = time.perf_counter() - t0
        t1 = time.perf_counter()
        us, info = dd.solve_dd(pdec, f, tol=tol)
        solve_s = time.perf_counter() - t1
        u = pdec.glue(us)
        n = pdec.workers
    finally:
        pdec.close()
    base = {"value": 1.0 / solve_s, "unit": "solves/s", "cores": n, "kind": "oracle",
            "sample": f"one oracle-DD solve of the same workload ({wl.sx * wl.sy} sparse-LU "
                      f"subdomain solves per sweep on {n} worker processes, one BLAS thread "
                      f"each, restarted GMRES(50) from G = 0 to tol {tol}): {solve_s:.1f} s, "
                      f"{info['iters']} outer iterations; subdomain factorisation "
                      f"{setup_s:.1f} s not counted",
            "solve_s": solve_s, "factor_s": setup_s, "outer_iters": info["iters"],
            "true_rel_residual_interface": info["true_rel"], **host_info()}
    return base, u


def cpu_global_lu(wl):
    """Global sparse LU of S = A - i omega H - omega^2 M (SuperLU, one
    thread): factorisation and solve times and the solution."""
    import scipy.sparse.linalg as spla
    from oracle import sem
    mesh, c, f = oracle_setup(wl)
    S, _, _, _ = sem.system(mesh, c, wl.omega)
    b = sem.load(mesh, f)
    t0 = time.perf_counter()
    lu = spla.splu(S)
    t1 = time.perf_counter()
    u = lu.solve(b)
    t2 = time.perf_counter()
    return {"n": int(S.shape[0]), "factor_s": t1 - t0, "solve_s": t2 - t1}, u


def cpu_baseline(wl, seconds=12.0):
    """The oracle's WaveHoltz (vectorised numpy, FP64) on this workload's
    subdomains, one WaveHoltz iteration per subdomain, subdomains taken in
    order until ~`seconds` of CPU time; DOF-updates/s on one host thread."""
    from oracle import dd, sem
    from oracle import waveholtz as wh
    mesh = sem.Rect(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    X, Y = sem.node_coords(mesh)
    t_setup = time.perf_counter()
    dec = dd.Decomposition(mesh, dd.Partition(wl.sx, wl.sy), wl.c(X, Y), wl.omega)
    nts = wh.subdomain_steps(dec)
    f = wl.f(X, Y)
    g0 = np.zeros(dec.n_if, dtype=complex)
    setup_s = time.perf_counter() - t_setup
    updates, n_it = 0.0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for l in range(dec.L):
            sd = dec.subs[l]
            b = dec.rhs(l, f, g0, 1.0)
            wh.iterate(sd["A"], sd["M"], sd["H"], b, dec.omega, nts[l],
                       np.zeros(b.size, complex))
            updates += b.size * (nts[l] - 1)
            n_it += 1
            if time.perf_counter() - t0 > seconds:
                break
    el = time.perf_counter() - t0
    return {"value": updates / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_it} subdomain WaveHoltz iterations (N_t-1 leapfrog steps each) "
                      f"over the {dec.L} subdomains of the same workload, numpy/scipy FP64, "
                      f"one thread ({el:.1f} s; oracle setup {setup_s:.1f} s not counted)"}


def cpu_baseline3(wl, seconds=12.0, n_sub=8):
    """The oracle's WaveHoltz (vectorised numpy, FP64) on subdomains of a
    box workload: the first `n_sub` subdomains are each set up on their own
    box (the problem the sweep solves there, given its interface data), then
    WaveHoltz iterations over them in turn until ~`seconds`; DOF-updates/s
    on one host thread."""
    from oracle import dd3, sem3
    from oracle import waveholtz as wh
    mx, my, mz = wl.nx // wl.sx, wl.ny // wl.sy, wl.nz // wl.sz
    hx = (wl.box[1] - wl.box[0]) / wl.nx
    hy = (wl.box[3] - wl.box[2]) / wl.ny
    hz = (wl.box[5] - wl.box[4]) / wl.nz
    L = wl.sx * wl.sy * wl.sz
    subs = []
    for l in range(min(n_sub, L)):
        a, b, c = l % wl.sx, (l // wl.sx) % wl.sy, l // (wl.sx * wl.sy)
        x0, y0, z0 = wl.box[0] + a * mx * hx, wl.box[2] + b * my * hy, wl.box[4] + c * mz * hz
        sub = sem3.Box(mx, my, mz, wl.P, x0, x0 + mx * hx, y0, y0 + my * hy, z0, z0 + mz * hz)
        X, Y, Z = sem3.node_coords(sub)
        one = dd3.Decomposition3(sub, dd3.Partition3(1, 1, 1), wl.c(X, Y, Z), wl.omega)
        rhs = one.rhs(0, wl.f(X, Y, Z), np.zeros(one.n_if, dtype=complex), 1.0)
        subs.append((one.subs[0], rhs, wh.subdomain_steps(one)[0]))
    updates, n_it = 0.0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sd, rhs, nt = subs[n_it % len(subs)]
        wh.iterate(sd["A"], sd["M"], sd["H"], rhs, wl.omega, nt, np.zeros(rhs.size, complex))
        updates += rhs.size * (nt - 1)
        n_it += 1
    el = time.perf_counter() - t0
    return {"value": updates / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_it} subdomain WaveHoltz iterations (N_t-1 leapfrog steps each) over "
                      f"the first {len(subs)} of the {L} subdomains of the same workload, "
                      f"numpy/scipy FP64, one thread ({el:.1f} s)"}


# name: (sweep precision, inner tolerance (None: the workload's), relax, tc2).
# FP32 WaveHoltz stagnates near 1e-6, so FP32 sweeps stop at 1e-5 and the
# FP64 refinement sweeps (the workload's tolerance) carry the accuracy.
VARIANTS = {"fp32_refined": ("fp32", 1e-5, 0.0, 0.0), "fp64_relaxed": ("fp64", None, 0.1, 0.0),
            "fp32_refined_relaxed": ("fp32", 1e-5, 0.1, 0.0),
            "fp64_tc2": ("fp64", None, 0.0, 0.1),
            "fp32_refined_relaxed_tc2": ("fp32", 1e-5, 0.1, 0.1)}


def rel_l2(u, ref):
    """Relative l2 difference of glued nodal vectors."""
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))


def timed_solves(W, prob, tol, steps, warmup=1, max_iter=2000):
    """`warmup` untimed then `steps` timed dd_solve_device calls with the
    source resident in HBM; a solve that does not converge raises.  Returns
    (per-solve seconds, stats of each, solution of the last)."""
    import torch
    dev = torch.device("cuda:0")
    N = prob.f.size
    f_re = torch.from_numpy(prob.f).to(dev)
    u_re = torch.empty(N, dtype=torch.float64, device=dev)
    u_im = torch.empty(N, dtype=torch.float64, device=dev)
    for _ in range(warmup):
        W.dd_solve_device(prob.h, f_re, None, None, None, tol, max_iter, u_re, u_im)
    torch.cuda.synchronize()
    lat, stats = [], []
    for _ in range(steps):
        t1 = time.perf_counter()
        st, _ = W.dd_solve_device(prob.h, f_re, None, None, None, tol, max_iter, u_re, u_im)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
        stats.append(st)
    u = u_re.cpu().numpy() + 1j * u_im.cpu().numpy()
    return lat, stats, u


def variants(W, wl, names, max_wh, progress=0, steps=2):
    """FP32 sweeps (with FP64 refinement), relaxed inner tolerance and the
    second-order transmission condition on the same workload: solves/s,
    latency, DOF-updates/s; returns the results and each variant's
    solution (compared with the oracle by the caller)."""
    out, sols = {}, {}
    for name in names:
        pname, tau, relax, tc2 = VARIANTS[name]
        prec = W.DD_FP64 if pname == "fp64" else W.DD_FP32
        tau = wl.tau_in if tau is None else tau
        prob = W.Problem(wl, precision=prec, tau_in=tau, relax=relax, max_wh=max_wh, tc2=tc2)
        if progress:
            W.dd_set_progress(prob.h, lambda it, rel, n=name: log(f"  {n} outer {it}: {rel:.2e}"),
                              progress)
        lat, stats, u = timed_solves(W, prob, wl.tol, steps)
        total = sum(lat)
        st = stats[-1]
        out[name] = {"solves_per_s": steps / total,
                     "dof_updates_per_s": sum(x["dof_updates"] for x in stats) / total,
                     "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                     "p99_ms": 1e3 * float(np.percentile(lat, 99)), "solves_timed": steps,
                     "outer_iters": st["outer_iters"], "refine_steps": st["refine_steps"],
                     "wh_iters_max": st["wh_iters_max"],
                     "true_rel_residual_interface": st["true_rel_residual"],
                     "rel_residual_global_fp64": W.dd_residual(prob.h, u, prob.f),
                     "tau_in": tau, "relax": relax, "tc2": tc2}
        sols[name] = u
        log(f"variant {name}: {1e3 * total / steps:.0f} ms per solve, "
            f"{st['outer_iters']} outer iterations")
        prob.close()
    return out, sols


def c1_latency(W, steps=20):
    """The 16x16-element, P=2, 2x2-subdomain problem: latency of single
    solves (FP64, and FP32 sweeps with FP64 refinement) and of one sweep;
    returns the results and the solutions."""
    import workloads
    wl = workloads.c1()
    out, sols = {}, {}
    for name, prec, tau in (("fp64", W.DD_FP64, wl.tau_in), ("fp32_refined", W.DD_FP32, 1e-5)):
        prob = W.Problem(wl, precision=prec, tau_in=tau, max_wh=1000)
        lat, stats, u = timed_solves(W, prob, wl.tol, steps, warmup=3)
        st = stats[-1]
        out[name] = {"us_per_solve_p50": 1e6 * float(np.percentile(lat, 50)),
                     "us_per_solve_p99": 1e6 * float(np.percentile(lat, 99)),
                     "us_per_sweep": 1e6 * st["sweep_seconds"] / max(st["sweeps"], 1),
                     "sweeps_per_solve": st["sweeps"], "outer_iters": st["outer_iters"],
                     "solves_timed": steps, "tau_in": tau}
        sols[name] = u
        prob.close()
    return out, sols


BYTES_STREAM = {"fp64": 80, "fp32": 40}   # per DOF-update, STREAM layout (10 words)


def batch_bench(args):
    """A batch of independent problems (400 subdomains, P in 1..4, 8..64
    elements per subdomain side) solved together: every sweep round is one
    batched launch per launch configuration."""
    import torch
    import workloads
    from paper_2606_21695_amd import wavedd as W
    W.require_gpu()
    torch.cuda.set_device(0)
    wls = workloads.c4()
    specs = [W.workload_spec(wl) for wl in wls]
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    tau = wls[0].tau_in if prec == W.DD_FP32 else 1e-10
    if args.tau_in is not None:
        tau = args.tau_in
    t0 = time.perf_counter()
    b = W.dd_batch_setup(specs, W.dd_default_options(precision=prec, tau_in=tau,
                                                     relax=args.relax, max_wh=args.max_wh,
                                                     tc2=args.tc2))
    setup_s = time.perf_counter() - t0
    tol = wls[0].tol
    fs = [s_["f"] for s_ in specs]
    log(f"batch setup {setup_s:.1f} s, {len(specs)} problems")
    def solve_logged(tag):
        """One batched solve; each problem's completion is reported as it
        happens."""
        t1 = time.perf_counter()
        r = W.dd_batch_solve(b, fs, tol, 2000, allow_notconv=True, progress=lambda k: log(
            f"{tag}: {k}/{len(fs)} problems done at {time.perf_counter() - t1:.1f} s"))
        return r, time.perf_counter() - t1

    for _ in range(args.warmup):
        solve_logged("warm-up")
    lat, rounds, res = [], [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        (us, sts, rcs, rc), el = solve_logged("timed")
        lat.append(el)
        rounds.append(W.dd_batch_launches(b))
        res = (us, sts, rcs)
        log(f"batch solve: {lat[-1]:.3f} s, {rounds[-1]} batched launches")
    total = time.perf_counter() - t0
    us, sts, rcs = res
    dof = sum(st["dof_updates"] for st in sts) * args.steps
    sweep_s = max(st["sweep_seconds"] for st in sts)
    flop = sum(flops_per_update(wl.P) * st["dof_updates"] for wl, st in zip(wls, sts))
    achieved = flop / sweep_s / 1e12
    rel = [W.dd_residual(W.dd_batch_handle(b, i), us[i], specs[i]["f"]) for i in range(len(us))]
    # the paper's protocol: 5 WaveHoltz iterations on random complex interface data
    rng = np.random.default_rng(4)
    for i in range(len(specs)):
        h = W.dd_batch_handle(b, i)
        n = W.dd_sizes(h)["n_iface"]
        W.dd_set_state(h, rng.standard_normal(n) + 1j * rng.standard_normal(n))
    ms5, dof5, nl5 = W.dd_batch_time_sweep(b, reps=5, fixed_iters=5)
    W.dd_batch_destroy(b)
    peak = PEAK_TFLOPS[args.precision]
    out = {
        "metric": "WaveHoltz DOF-updates/s (batched DD solves)",
        "value": dof / total, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == W.DD_FP64 else "f32 sweep / f64 outer",
        "data": "synthetic (seeded log-normal wavespeed, Gaussian sources)",
        "config": {"workload": f"c4: {len(wls)} independent problems, "
                               f"{sum(wl.sx * wl.sy for wl in wls)} subdomains, P in 1..4, "
                               f"omega={wls[0].omega}, tol={tol}",
                   "precision": args.precision, "tau_in": tau, "relax": args.relax,
                   "max_wh": args.max_wh, "tc2": args.tc2},
        "problems": len(wls),
        "solves_per_s": len(wls) * args.steps / total,
        "batch_latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                             "p99": 1e3 * float(np.percentile(lat, 99))},
        "launches": rounds[-1],
        "not_converged": int(sum(r != 0 for r in rcs)),
        "rel_residual_global_max": float(max(rel)),
        "setup_s": setup_s,
        "paper_protocol_5_iterations": {"ms_per_round": ms5, "dof_updates": dof5,
                                        "dof_updates_per_s": dof5 / (ms5 * 1e-3),
                                        "launches_per_round": nl5},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "batched sweep launches (all layouts)",
                     "flop_per_dof_update": "4(P+2)+16"},
    }
    print(json.dumps(out))


def serve_sample(wl_list, requests, max_nodes, max_sub_nodes):
    """The first `requests` requests of the seeded stream whose global mesh
    has at most max_nodes nodes and whose subdomains at most max_sub_nodes."""
    out = []
    for wl in wl_list:
        n = (wl.nx * wl.P + 1) * (wl.ny * wl.P + 1)
        nl = ((wl.nx // wl.sx) * wl.P + 1) * ((wl.ny // wl.sy) * wl.P + 1)
        if n <= max_nodes and nl <= max_sub_nodes:
            out.append(wl)
        if len(out) == requests:
            break
    return out


def serve_bench(args):
    """Serving engine on a seeded sample of the request stream (each request
    its own mesh, degree, frequency, wavespeed and sources; FP32 sweeps with
    FP64 refinement, tol 1e-6): closed-loop saturated throughput, then
    Poisson arrivals at fractions rho of it (latency = arrival to result),
    then the closed loop again under a small HBM budget; beside it the plain
    FP64 form (one dd_solve at a time) on the first requests of the sample.

    The engine runs each active request's outer-iteration kernels on that
    request's stream and each round of sweeps on one of eight launch
    streams; HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 by
    default) and kernels of streams that share a queue run in order, so a
    request's short kernels would wait behind other requests' sweeps.  The
    serving run therefore asks for 32 hardware queues (set before the HIP
    runtime starts, unless the environment sets it)."""
    os.environ.setdefault("GPU_MAX_HW_QUEUES", "32")
    import torch
    import workloads
    from paper_2606_21695_amd import wavedd as W
    W.require_gpu()
    torch.cuda.set_device(0)
    wls = serve_sample(workloads.c5(n_requests=args.stream), args.requests, args.max_nodes,
                       args.max_sub_nodes)
    specs = [W.workload_spec(wl) for wl in wls]
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    o = W.dd_default_options(precision=prec, tau_in=wls[0].tau_in if prec == W.DD_FP32 else 1e-12,
                             relax=args.relax, max_wh=args.max_wh, tc2=args.tc2)

    def run(arrivals, budget, tag):
        e = W.dd_engine_create(budget, args.max_active, o)
        try:
            import threading
            where, submitted, errs, lock = {}, threading.Semaphore(0), [], threading.Lock()
            t0 = time.perf_counter()

            def submit_all():
                # arrivals on a thread of their own, so that results are
                # collected (and logged) while requests still arrive
                try:
                    for k, s_ in enumerate(specs):
                        if arrivals is not None:
                            dt = arrivals[k] - (time.perf_counter() - t0)
                            if dt > 0:
                                time.sleep(dt)
                        with lock:
                            where[W.dd_engine_submit(e, s_, s_["f"], wls[k].tol, 3000)] = k
                        submitted.release()
                except Exception as ex:   # reported by the collecting thread
                    errs.append(ex)
                    for _ in range(len(specs)):
                        submitted.release()

            th = threading.Thread(target=submit_all)
            th.start()
            res = [None] * len(specs)
            for n_done in range(len(specs)):
                submitted.acquire()
                if errs:
                    th.join()
                    raise errs[0]
                rid = W.dd_engine_wait_any(e)
                with lock:
                    k = where[rid]
                res[k] = W.dd_engine_wait(e, rid, specs[k]["c"].size, allow_notconv=True)
                log(f"{tag}: request {k} ({specs[k]['c'].size} nodes, P={specs[k]['P']}, "
                    f"{specs[k]['sx']}x{specs[k]['sy']} subdomains) done, "
                    f"{n_done + 1}/{len(specs)} at {time.perf_counter() - t0:.1f} s")
            th.join()
            wall = time.perf_counter() - t0
            info = W.dd_engine_get_info(e)
        finally:
            W.dd_engine_destroy(e)
        lat = [t[2] - t[0] for _, _, t, _ in res]
        out = {"solves_per_s": len(specs) / wall, "wall_s": wall,
                "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                               "p99": 1e3 * float(np.percentile(lat, 99))},
                "dof_updates_per_s": sum(st["dof_updates"] for _, st, _, _ in res) / wall,
                "launches": info["launches"], "peak_running": info["peak_running"],
                "not_converged": int(sum(rc != 0 for *_, rc in res)),
                "max_true_rel_residual": float(max(st["true_rel_residual"] for _, st, _, _ in res))}
        log(f"{tag}: " + json.dumps(out))
        return out

    budget = int(args.budget_gib * (1 << 30))
    if args.mu > 0:
        # saturated rate given (measured by an earlier closed-loop run)
        sat, mu = None, args.mu
    else:
        sat = run(None, budget, "closed loop")
        mu = sat["solves_per_s"]
    rhos = [float(r) for r in args.rhos.split(",") if r]
    at_rho = {}
    for i, rho in enumerate(rhos):
        rng = np.random.default_rng(5 + i)
        arr = np.cumsum(rng.exponential(1.0 / (rho * mu), len(specs)))
        at_rho[str(rho)] = dict(run(arr, budget, f"rho={rho}"), rho=rho)
    small = (run(None, int(args.small_budget_gib * (1 << 30)), "small budget")
             if args.small_budget_gib > 0 else None)
    # the plain FP64 form: one dd_solve at a time, FP64 sweeps to 1e-12, on
    # the first requests of the sample (no new solve after --plain-budget-s)
    plain_lat = []
    t_plain = time.perf_counter()
    for k in range(min(args.plain_requests, len(specs))):
        if time.perf_counter() - t_plain > args.plain_budget_s:
            break
        s_ = specs[k]
        h = W.dd_setup(s_["nx"], s_["ny"], s_["P"], s_["c"], s_["omega"], s_["sx"], s_["sy"],
                       s_["x0"], s_["x1"], s_["y0"], s_["y1"],
                       W.dd_default_options(tau_in=1e-12, max_wh=args.max_wh))
        try:
            W.dd_set_progress(h, lambda it, rel, k=k: log(f"plain FP64: request {k}: "
                                                          f"{it} matvecs, residual {rel:.2e}"), 25)
            t0 = time.perf_counter()
            W.dd_solve(h, s_["f"], None, wls[k].tol, 3000, allow_notconv=True)
            plain_lat.append(time.perf_counter() - t0)
            log(f"plain FP64: request {k} ({s_['c'].size} nodes) {plain_lat[-1]:.2f} s")
        finally:
            W.dd_destroy(h)
    n_plain = len(plain_lat)
    out = {
        "metric": "DD solves/s (serving, continuous batching)",
        "value": mu, "unit": "solves/s", "n_gpus": 1, "steps": len(specs),
        "warmup": 0, "ms_per_step": 1e3 / mu, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == W.DD_FP64 else "f32 sweep / f64 outer",
        "data": "synthetic (seeded request stream: own mesh, P, omega, wavespeed, sources)",
        "config": {"workload": f"c5: the first {len(specs)} requests of the seeded stream "
                               f"(seed 5, {args.stream} requests drawn) with at most "
                               f"{args.max_nodes} global nodes and {args.max_sub_nodes} nodes per "
                               f"subdomain",
                   "precision": args.precision, "max_active": args.max_active,
                   "budget_gib": args.budget_gib, "tc2": args.tc2, "relax": args.relax},
        "saturated": sat,
        "saturated_solves_per_s": mu,
        "poisson": at_rho,
        "small_budget": dict(small, budget_gib=args.small_budget_gib) if small else None,
        "plain_fp64_single_solves": {
            "requests": n_plain, "budget_s": args.plain_budget_s,
            "solves_per_s": n_plain / sum(plain_lat) if plain_lat else None,
            "latency_ms": {"p50": 1e3 * float(np.percentile(plain_lat, 50)),
                           "p99": 1e3 * float(np.percentile(plain_lat, 99))} if plain_lat else None},
        "request_sizes": {"nodes_min": int(min(s_["c"].size for s_ in specs)),
                          "nodes_max": int(max(s_["c"].size for s_ in specs)),
                          "nodes_total": int(sum(s_["c"].size for s_ in specs)),
                          "subdomains_total": int(sum(s_["sx"] * s_["sy"] for s_ in specs))},
    }
    print(json.dumps(out))


def operator_ms(W, h, reps=50):
    """Average time of one whole-domain FP64 operator evaluation y = S x
    (random x), HIP events on the stream the kernel runs on (a stream of its
    own: a null stream would send the launches to the handle's stream)."""
    import torch
    n = W.dd_sizes(h)["n_global"]
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(2 * n, dtype=torch.float64, device="cuda", generator=g)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for _ in range(3):
        W.dd_apply_operator_device(h, x, y, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        W.dd_apply_operator_device(h, x, y, s)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def flops_per_update3(P):
    """Algorithmic FLOP of one box DOF-update: the three (2P+1)-point
    stiffness windows with one merged centre tap 2(6P+1), p update 2,
    velocity update 6, filter 4."""
    return 2 * (6 * P + 1) + 12


def box_bench(args):
    out = box_result(args)
    if out is not None:
        print(json.dumps(out))


def box_result(args):
    """Box (3D) workloads: the DD cycle of the paper's 3D timing (every
    subdomain runs exactly 5 WaveHoltz iterations from random complex
    interface data, one launch) against one whole-box operator
    evaluation.  None after a --box-solve run (which prints its own line)."""
    import torch
    import workloads
    from paper_2606_21695_amd import wavedd as W
    W.require_gpu()
    torch.cuda.set_device(0)
    wl = workloads.CONFIGS3[args.config]()
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    X, Y, Z = W.dd3_mesh_coords(wl.nx, wl.ny, wl.nz, wl.P, *wl.box)
    o = W.dd_default_options(precision=prec, tau_in=0.0, max_wh=5)
    h = W.dd3_setup(wl.nx, wl.ny, wl.nz, wl.P, wl.c(X, Y, Z), wl.omega, wl.sx, wl.sy, wl.sz,
                    *wl.box, options=o)
    s = W.dd3_sizes(h)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(s["n_iface"]) + 1j * rng.standard_normal(s["n_iface"])
    # the timed launches start from this random interface state
    W.dd3_sweep(h, g, None, 0.0, want_u=False)
    if args.box_solve:
        box_solve_bench(args, W, wl, h, X, Y, Z, s)
        return None
    log(f"{args.config}: {s['n_sub']} subdomains of {s['n_local']} nodes, timing")
    ms, dof = W.dd3_time_sweep(h, args.steps, 5)
    n = s["n_global"]
    x = torch.randn(2 * n, dtype=torch.float64, device="cuda",
                 generator=torch.Generator(device="cuda").manual_seed(0))
    y = torch.empty_like(x)
    st = torch.cuda.Stream()
    for _ in range(3):
        W.dd3_apply_operator_device(h, x, y, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(50):
        W.dd3_apply_operator_device(h, x, y, st)
    e1.record(st)
    torch.cuda.synchronize()
    op_ms = e0.elapsed_time(e1) / 50
    nt = W.dd3_time_steps(h)
    W.dd3_destroy(h)
    # the library launches the register-capped build for FP64 workgroups of
    # at most 768 threads at P <= 3
    wg = (s["n_local"] + 63) // 64 * 64
    kname = ("sweep3_kernel_capped" if args.precision == "fp64" and wl.P <= 3 and wg <= 768
             else "sweep3_kernel")
    flop = flops_per_update3(wl.P) * dof
    peak = PEAK_TFLOPS[args.precision]
    ach = flop / (ms * 1e-3) / 1e12
    out = {"metric": "WaveHoltz DOF-updates/s (box DD cycle, 5 WaveHoltz iterations, random input)",
           "value": dof / (ms * 1e-3), "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision.replace("fp", "f"),
           "data": "synthetic (random complex interface data)",
           "config": {"workload": f"{args.config}: {wl.nx}x{wl.ny}x{wl.nz} elements P={wl.P}, "
                                  f"{wl.sx}x{wl.sy}x{wl.sz} subdomains of {s['n_local']} nodes, "
                                  f"c=1 on [-1,1]^3, omega={wl.omega:.2f}, N_t={int(nt.max())}",
                      "kernel": kname},
           "dof_updates_per_launch": dof,
           "operator_ms": op_ms, "dd_cycle_over_operator": ms / op_ms,
           "operator_gbs": 48.0 * n / (op_ms * 1e-3) / 1e9,
           "roofline": {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                        "frac": ach / peak, "kernel": kname,
                        "traffic": MEASURED_TRAFFIC3.get((kernel3_hash(), args.config,
                                                         args.precision))}}
    if not args.no_cpu:
        log("cpu baseline (oracle WaveHoltz on sampled subdomains)")
        out["cpu_baseline"] = cpu_baseline3(wl)
    return out


def box_solve_bench(args, W, wl, h, X, Y, Z, s):
    """Full box solves (outer FP64 GMRES over box sweeps, WaveHoltz to
    tau_in = 1e-12 with a cap of 1000; FP32 sweeps to 1e-5 with FP64
    refinement) with the workload's source; one JSON line with solves/s,
    outer iterations and the global FP64 residual."""
    W.dd3_destroy(h)
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    # FP32 WaveHoltz stagnates near 1e-6, so FP32 sweeps take 1e-5 (the FP64
    # refinement sweeps use their own tolerance)
    tau = 1e-12 if prec == W.DD_FP64 else 1e-5
    o = W.dd_default_options(precision=prec, tau_in=tau, max_wh=1000, relax=args.relax)
    h = W.dd3_setup(wl.nx, wl.ny, wl.nz, wl.P, wl.c(X, Y, Z), wl.omega, wl.sx, wl.sy, wl.sz,
                    *wl.box, options=o)
    f = wl.f(X, Y, Z)
    tol = args.box_tol
    times, st, rc, u = [], None, 0, None
    for i in range(args.steps):
        t0 = time.perf_counter()
        u, st, rc = W.dd3_solve(h, f, tol, 3000, allow_notconv=True)
        times.append(time.perf_counter() - t0)
        log(f"box solve {i}: {times[-1]:.2f} s, {st['outer_iters']} outer iterations, rc={rc}")
    rel = W.dd3_residual(h, u, f)
    W.dd3_destroy(h)
    t = float(np.mean(times))
    out = {"metric": "box DD solves/s (FP64 outer GMRES)", "value": 1.0 / t, "unit": "solves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": 0, "ms_per_step": 1e3 * t,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.precision.replace("fp", "f"), "data": "synthetic (workload source)",
           "config": {"workload": f"{args.config}: {wl.nx}x{wl.ny}x{wl.nz} elements P={wl.P}, "
                                  f"{wl.sx}x{wl.sy}x{wl.sz} subdomains, tol={tol}, tau_in={tau}",
                      "relax": args.relax},
           "outer_iters": st["outer_iters"], "converged": rc == 0,
           "true_rel_residual_interface": st["true_rel_residual"],
           "rel_residual_global_fp64": rel, "wh_iters_max": st["wh_iters_max"],
           "dof_updates_per_s": st["dof_updates"] / t}
    print(json.dumps(out))


def protocol_bench(args):
    print(json.dumps(protocol_result(args)))


def protocol_result(args):
    """The paper's DD-cycle timing (Sec. VII-A): sweeps of exactly 5
    WaveHoltz iterations per subdomain from random complex interface data,
    sources off, averaged over --steps launches after --warmup."""
    import torch
    import workloads
    from paper_2606_21695_amd import wavedd as W
    W.require_gpu()
    torch.cuda.set_device(0)
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    if args.config == "c4":
        wls = workloads.c4()
        b = W.dd_batch_setup([W.workload_spec(wl) for wl in wls],
                             W.dd_default_options(precision=prec))
        rng = np.random.default_rng(4)
        for i in range(len(wls)):
            h = W.dd_batch_handle(b, i)
            n = W.dd_sizes(h)["n_iface"]
            W.dd_set_state(h, rng.standard_normal(n) + 1j * rng.standard_normal(n))
        ms, dof, nl = W.dd_batch_time_sweep(b, reps=args.steps, fixed_iters=5)
        W.dd_batch_destroy(b)
        layout, kernel = "per problem (autotuned per shape)", f"{nl} batched launches per round"
        desc = f"c4: {len(wls)} problems, {sum(wl.sx * wl.sy for wl in wls)} subdomains"
        flop = None
        traffic = None
    else:
        wl = workloads.CONFIGS[args.config]()
        prob = W.Problem(wl, precision=prec, layout=LAYOUT_IDS[args.layout], tau_in=0.0, max_wh=5)
        h = prob.h
        rng = np.random.default_rng(1)
        n = W.dd_sizes(h)["n_iface"]
        W.dd_set_state(h, rng.standard_normal(n) + 1j * rng.standard_normal(n))
        ms, dof = W.dd_time_sweep(h, args.steps, 5)
        op_ms = operator_ms(W, h)
        lay, wg = W.dd_layout(h)
        traffic = MEASURED_TRAFFIC.get((kernel_hash(lay), "protocol", args.config, args.precision))
        prob.close()
        layout = LAYOUT_NAMES[lay]
        kernel = kernel_name(lay, wg)
        desc = (f"{args.config}: {wl.nx}x{wl.ny} elements P={wl.P}, {wl.sx}x{wl.sy} subdomains, "
                f"omega={wl.omega:.2f}")
        flop = flops_per_update(wl.P) * dof
    out = {"metric": "WaveHoltz DOF-updates/s (DD cycle, 5 WaveHoltz iterations, random input)",
           "value": dof / (ms * 1e-3), "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision.replace("fp", "f"),
           "data": "synthetic (random complex interface data)",
           "config": {"workload": desc, "layout": layout, "kernel": kernel},
           "dof_updates_per_launch": dof}
    if args.config != "c4":
        # the paper's normaliser (Sec. VII-A): DD-cycle time over the time of one
        # whole-domain operator evaluation y = S x in FP64
        out["operator_ms"] = op_ms
        out["dd_cycle_over_operator"] = ms / op_ms
        # algorithmic bytes of y = S x per node: x, y (complex) and M, H
        n_global = (wl.nx * wl.P + 1) * (wl.ny * wl.P + 1)
        out["operator_gbs"] = 48.0 * n_global / (op_ms * 1e-3) / 1e9
    if flop is not None:
        peak = PEAK_TFLOPS[args.precision]
        ach = flop / (ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                           "frac": ach / peak, "traffic": traffic, "kernel": kernel}
        if layout == "stream":
            gbs = BYTES_STREAM[args.precision] * dof / (ms * 1e-3) / 1e9
            out["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                               "frac": gbs / 8000.0, "traffic": traffic, "alu_tflops": ach,
                               "kernel": kernel, "byte_per_dof_update": BYTES_STREAM[args.precision]}
    return out


def other_workloads(args):
    """The DD-cycle protocol (5 WaveHoltz iterations per subdomain, random
    interface data) of the 512x512-element STREAM workload (FP64 and FP32)
    and the 64^3 box workload (FP64), a few seconds each, beside the default
    line: value, ms per DD cycle, roofline (a failure is recorded, not
    raised)."""
    res = {}
    for name, fn, cfg, prec in (("c3_protocol_fp64", protocol_result, "c3", "fp64"),
                                ("c3_protocol_fp32", protocol_result, "c3", "fp32"),
                                ("c6_protocol_fp64", box_result, "c6", "fp64")):
        a = argparse.Namespace(**vars(args))
        a.config, a.precision, a.steps, a.layout = cfg, prec, 3, "auto"
        a.no_cpu, a.box_solve, a.protocol = True, False, True
        try:
            r = fn(a)
            res[name] = {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "config",
                                           "roofline", "dd_cycle_over_operator") if k in r}
        except Exception as ex:   # the default line stays valid without them
            res[name] = {"error": repr(ex)}
        log(f"{name} done")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--layout", default="auto", choices=sorted(LAYOUT_IDS),
                    help="sweep layout (auto = the autotuner's choice)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--relax", type=float, default=0.0,
                    help="variable inner tolerance factor (0 = fixed inner tolerance)")
    ap.add_argument("--tau-in", type=float, default=None, help="override the inner tolerance")
    ap.add_argument("--tc2", type=float, default=0.0,
                    help="second-order transmission condition (0 = the paper's zeroth order)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c1", action="store_true",
                    help="skip the 16x16-element latency solves of the default run")
    ap.add_argument("--no-protocols", action="store_true",
                    help="skip the 512x512 and box DD-cycle lines of the default run")
    ap.add_argument("--global-lu", action="store_true",
                    help="also time the oracle's global sparse LU of the workload")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32 / relaxed-tolerance comparison solves")
    ap.add_argument("--variants", default=None,
                    help="comma-separated comparison solves (default: all for the "
                         "256x256 workloads, fp32_refined_relaxed for 512x512)")
    ap.add_argument("--progress", type=int, default=None,
                    help="print the outer residual every N iterations (default: 25 for "
                         "512x512, off otherwise)")
    ap.add_argument("--serve", action="store_true", help="serving engine on the c5 stream")
    ap.add_argument("--max-wh", type=int, default=1000,
                    help="WaveHoltz cap per subdomain solve (a safety limit: the stop rule "
                         "is the inner tolerance; the 256x256 waveguide needs up to 135 "
                         "periods, the 64-element subdomains of the larger workloads hundreds)")
    ap.add_argument("--protocol", action="store_true",
                    help="the paper's DD-cycle timing instead of solves: sweeps of exactly 5 "
                         "WaveHoltz iterations per subdomain on random interface data")
    ap.add_argument("--box-solve", action="store_true",
                    help="box workloads: full solves instead of the DD-cycle timing")
    ap.add_argument("--box-tol", type=float, default=1e-6,
                    help="outer tolerance of --box-solve")
    ap.add_argument("--requests", type=int, default=200,
                    help="serving mode: requests taken from the seeded stream")
    ap.add_argument("--stream", type=int, default=40000,
                    help="serving mode: requests drawn from the seeded stream")
    ap.add_argument("--plain-budget-s", type=float, default=150.0,
                    help="serving mode: no new plain FP64 solve after this many seconds")
    ap.add_argument("--mu", type=float, default=0.0,
                    help="serving mode: saturated solves/s from an earlier closed-loop run "
                         "(skips the closed loop)")
    ap.add_argument("--max-nodes", type=int, default=40000,
                    help="serving mode: skip requests with more global nodes")
    ap.add_argument("--max-sub-nodes", type=int, default=2500,
                    help="serving mode: skip requests with larger subdomains (the default "
                         "keeps requests whose subdomains fit the on-chip layouts)")
    ap.add_argument("--rhos", default="0.5,0.8,0.95",
                    help="serving mode: arrival rates as fractions of the saturated rate")
    ap.add_argument("--max-active", type=int, default=24)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--small-budget-gib", type=float, default=2.0,
                    help="serving mode: HBM budget of the admission run")
    ap.add_argument("--plain-requests", type=int, default=20,
                    help="serving mode: requests solved one at a time in plain FP64")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a kernel of known "
                         "traffic for scaling FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "wavedd runs on one GPU: the sweep shards by "
                                   "subdomain blocks across GPUs by design, but no multi-GPU "
                                   "path is built; use --gpus 1"}))
        sys.exit(2)

    if args.calibrate_copy:
        import torch
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.ones_like(a)
        torch.cuda.synchronize()
        a.copy_(b)
        torch.cuda.synchronize()
        del a, b
    if args.serve:
        return serve_bench(args)
    if args.config.startswith("c6"):
        return box_bench(args)
    if args.protocol:
        return protocol_bench(args)
    if args.config == "c4":
        return batch_bench(args)
    import torch
    import workloads
    from paper_2606_21695_amd import wavedd as W

    W.require_gpu()
    torch.cuda.set_device(0)
    wl = workloads.CONFIGS[args.config]()
    prec = W.DD_FP64 if args.precision == "fp64" else W.DD_FP32
    tau = wl.tau_in if prec == W.DD_FP64 else max(wl.tau_in, 1e-5)
    if args.tau_in is not None:
        tau = args.tau_in
    t0 = time.perf_counter()
    prob = W.Problem(wl, precision=prec, layout=LAYOUT_IDS[args.layout], tau_in=tau,
                     relax=args.relax, max_wh=args.max_wh, tc2=args.tc2)
    setup_s = time.perf_counter() - t0
    if args.progress is None:
        args.progress = 25 if args.config == "c3" else 0
    if args.progress:
        W.dd_set_progress(prob.h, lambda it, rel: log(f"  outer {it}: {rel:.2e}"), args.progress)
    h = prob.h
    log(f"setup {setup_s:.1f} s, layout {W.dd_layout(h)}")
    lat, stats, u = timed_solves(W, prob, wl.tol, args.steps, warmup=args.warmup)
    for k, (t, st) in enumerate(zip(lat, stats)):
        log(f"solve {k}: {t:.3f} s, {st['outer_iters']} outer iterations")
    total = sum(lat)

    dof = sum(s["dof_updates"] for s in stats)
    sweeps = sum(s["sweeps"] for s in stats)
    sweep_s = sum(s["sweep_seconds"] for s in stats)
    P = wl.P
    fl = flops_per_update(P)
    achieved = fl * dof / sweep_s / 1e12 if sweep_s > 0 else 0.0
    peak = PEAK_TFLOPS[args.precision]
    lay, wg = W.dd_layout(h)
    rel_res = W.dd_residual(h, u, prob.f)
    nt = W.dd_time_steps(h)
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak}
    if lay == 4:
        gbs = BYTES_STREAM[args.precision] * dof / sweep_s / 1e9 if sweep_s > 0 else 0.0
        roof = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                "frac": gbs / 8000.0, "byte_per_dof_update": BYTES_STREAM[args.precision],
                "alu_tflops": achieved}
    out = {
        "metric": "WaveHoltz DOF-updates/s (DD solve, FP64 outer)",
        "value": dof / total,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == W.DD_FP64 else "f32 sweep / f64 outer",
        "data": "synthetic (seeded Y-waveguide wavespeed, Gaussian source)",
        "config": {"workload": f"{args.config}: {wl.nx}x{wl.ny} elements P={P}, "
                               f"{wl.sx}x{wl.sy} subdomains, omega={wl.omega:.2f}, tol={wl.tol}",
                   "precision": args.precision,
                   "layout": LAYOUT_NAMES[lay],
                   "wg_threads": wg, "tau_in": tau, "relax": args.relax, "max_wh": args.max_wh,
                   "tc2": args.tc2},
        "solves_per_s": args.steps / total,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "outer_iters": stats[-1]["outer_iters"],
        "sweeps_per_solve": stats[-1]["sweeps"],
        "wh_iters_max": stats[-1]["wh_iters_max"],
        "wh_iters_mean": stats[-1]["wh_iters_total"] / (stats[-1]["sweeps"] * wl.sx * wl.sy),
        "nt_range": [int(nt.min()), int(nt.max())],
        "sweep_fraction_of_time": sweep_s / total,
        "rel_residual_global_fp64": rel_res,
        "true_rel_residual_interface": stats[-1]["true_rel_residual"],
        "rel_l2_vs_oracle": None,
        "setup_s": setup_s,
        "roofline": dict(roof, **{
            "traffic": MEASURED_TRAFFIC.get((kernel_hash(lay), "solve", args.config,
                                             args.precision)),
            "kernel": kernel_name(lay, wg),
            "flop_per_dof_update": fl,
            "avg_launch_ms": 1e3 * sweep_s / sweeps if sweeps else None}),
    }
    prob.close()
    sols = {}
    if not args.no_variants:
        names = (args.variants.split(",") if args.variants else
                 ["fp32_refined_relaxed"] if args.config == "c3" else list(VARIANTS))
        out["variants"], sols = variants(W, wl, names, args.max_wh, args.progress,
                                         steps=min(5, args.steps))
    c1_sols = {}
    if args.config == "c2" and not args.no_c1:
        out["c1_latency"], c1_sols = c1_latency(W)
        log("c1 latency done")
    if args.config == "c2" and not args.no_protocols:
        out["other_workloads"] = other_workloads(args)
    if not args.no_cpu:
        # the oracle: DD with exact subdomain solves at the same outer
        # tolerance on the host's cores; every GPU solution is compared with it
        log("cpu baseline: oracle DD on a process pool")
        base, u_ref = cpu_baseline_dd(wl, wl.tol)
        out["cpu_baseline"] = base
        out["rel_l2_vs_oracle"] = rel_l2(u, u_ref)
        for name, uv in sols.items():
            out["variants"][name]["rel_l2_vs_oracle"] = rel_l2(uv, u_ref)
        log("cpu baseline: WaveHoltz iterate rate")
        out["cpu_baseline"]["waveholtz_oracle"] = cpu_baseline(wl, seconds=6.0)
        if c1_sols:
            import workloads
            from oracle import dd
            wl1 = workloads.c1()
            mesh1, c_1, f_1 = oracle_setup(wl1)
            dec1 = dd.Decomposition(mesh1, dd.Partition(wl1.sx, wl1.sy), c_1, wl1.omega)
            t0 = time.perf_counter()
            us1, _ = dd.solve_dd(dec1, f_1, tol=wl1.tol)
            dd_s = time.perf_counter() - t0
            u1 = dec1.glue(us1)
            lu1, u1_lu = cpu_global_lu(wl1)
            for name, uv in c1_sols.items():
                out["c1_latency"][name]["rel_l2_vs_oracle"] = rel_l2(uv, u1)
                out["c1_latency"][name]["rel_l2_vs_global_lu"] = rel_l2(uv, u1_lu)
            out["c1_latency"]["oracle"] = {"dd_solve_s_one_thread": dd_s, "global_lu": lu1}
        if args.global_lu:
            log("cpu baseline: global sparse LU")
            lu, u_lu = cpu_global_lu(wl)
            lu["rel_l2_gpu_vs_global_lu"] = rel_l2(u, u_lu)
            lu["rel_l2_oracle_dd_vs_global_lu"] = rel_l2(u_ref, u_lu)
            out["cpu_baseline"]["global_lu"] = lu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
