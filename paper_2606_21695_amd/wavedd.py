"""ctypes binding of the wavedd C ABI (include/wavedd.h).

The functions keep the C names and only marshal arguments: every step of
the computation runs in the HIP library.  Loading fails loudly when the
library has not been built; there is no fallback path.

Host arrays are numpy float64 arrays; device arrays are torch CUDA tensors
(their ``data_ptr()`` is passed through), torch being used only for device
memory and streams.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavedd.so")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ENAN, DD_ENOTCONV, DD_ENODEV = 0, -1, -2, -3, -4, -5, -6
DD_FP64, DD_FP32 = 0, 1
DD_LAYOUT_AUTO, DD_LAYOUT_NODE, DD_LAYOUT_PATCH, DD_LAYOUT_PATCH_XCHG, DD_LAYOUT_STREAM = 0, 1, 2, 3, 4
DD_OUTER_GMRES, DD_OUTER_FIXED = 0, 1

EXPORTS = [
    "dd_default_options", "dd_setup", "dd_destroy", "dd_last_error", "dd_sizes",
    "dd_node_coords", "dd_time_steps", "dd_solve", "dd_solve_device", "dd_sweep",
    "dd_apply_stiffness", "dd_residual", "dd_residual_device_noalloc",
    "dd_apply_operator_device", "dd_get_state",
    "dd_set_state", "dd_time_sweep", "dd_layout", "dd_mesh_coords",
    "dd_batch_setup", "dd_batch_destroy", "dd_batch_handle", "dd_batch_solve",
    "dd_batch_time_sweep", "dd_batch_launches", "dd_batch_wait_progress",
    "dd_batch_solve_start", "dd_batch_solve_finish",
    "dd_engine_create", "dd_engine_destroy", "dd_engine_submit", "dd_engine_status",
    "dd_engine_wait", "dd_engine_get_info", "dd_engine_wait_any", "dd_set_progress",
    "dd3_setup", "dd3_destroy", "dd3_sizes", "dd3_time_steps", "dd3_mesh_coords", "dd3_sweep",
    "dd3_time_sweep", "dd3_apply_operator_device", "dd3_solve", "dd3_residual",
]
DD_REQ_QUEUED, DD_REQ_RUNNING, DD_REQ_DONE = 0, 1, 2


class dd_mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double)]


class dd_partition(C.Structure):
    _fields_ = [("sx", C.c_int), ("sy", C.c_int)]


class dd_box(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("z0", C.c_double), ("z1", C.c_double), ("nx", C.c_int), ("ny", C.c_int),
                ("nz", C.c_int)]


class dd_partition3(C.Structure):
    _fields_ = [("sx", C.c_int), ("sy", C.c_int), ("sz", C.c_int)]


class dd_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("layout", C.c_int), ("tau_in", C.c_double),
                ("max_wh", C.c_int), ("outer", C.c_int), ("restart", C.c_int),
                ("nt_override", C.c_int), ("cfl", C.c_double), ("refine", C.c_int),
                ("relax", C.c_double), ("warm", C.c_int), ("tc2", C.c_double)]


class dd_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("sweeps", C.c_int), ("rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("wh_iters_total", C.c_int64),
                ("wh_iters_max", C.c_int), ("nt_min", C.c_int), ("nt_max", C.c_int),
                ("dof_updates", C.c_double), ("sweep_seconds", C.c_double),
                ("seconds", C.c_double), ("refine_steps", C.c_int), ("fp64_sweeps", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dd_problem(C.Structure):
    _fields_ = [("mesh", dd_mesh), ("degree", C.c_int), ("wavespeed", C.POINTER(C.c_double)),
                ("omega", C.c_double), ("part", dd_partition)]


class dd_engine_info(C.Structure):
    _fields_ = [("queued", C.c_int64), ("running", C.c_int64), ("done", C.c_int64),
                ("launches", C.c_int64), ("peak_running", C.c_int64),
                ("budget_bytes", C.c_size_t), ("store_bytes", C.c_size_t),
                ("request_bytes", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# void (*)(void* user, int outer_iters, double rel_residual)
PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int, C.c_double)


class WaveddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wavedd error {code}: {msg}")
        self.code = code


_lib = None


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def load():
    """Load libwavedd.so (raises if it is missing).

    torch is imported first so that the library binds to the HIP runtime
    torch already uses (same SONAME): one runtime per process, so device
    pointers and streams from torch are valid in the library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2606_21695_amd.build`")
    import torch  # noqa: F401  (loads the process's HIP runtime)
    lib = C.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise RuntimeError(f"two HIP runtimes mapped in one process: {sorted(rts)}")
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    I64 = C.POINTER(C.c_int64)
    sig = {
        "dd_default_options": ([C.POINTER(dd_options)], C.c_int),
        "dd_setup": ([C.POINTER(P), C.POINTER(dd_mesh), C.c_int, D, C.c_double,
                      C.POINTER(dd_partition), C.POINTER(dd_options)], C.c_int),
        "dd_destroy": ([P], None),
        "dd_last_error": ([], C.c_char_p),
        "dd_sizes": ([P, I64, I64, I64, I64, I64], C.c_int),
        "dd_node_coords": ([P, D, D], C.c_int),
        "dd_time_steps": ([P, C.POINTER(C.c_int)], C.c_int),
        "dd_solve": ([P, D, D, D, D, C.c_double, C.c_int, D, D, C.POINTER(dd_stats)], C.c_int),
        "dd_solve_device": ([P, P, P, P, P, P, C.c_double, C.c_int, P, P, P,
                             C.POINTER(dd_stats)], C.c_int),
        "dd_sweep": ([P, D, D, D, D, C.c_double, D, D, D, D, C.POINTER(C.c_int)], C.c_int),
        "dd_apply_stiffness": ([P, D, D], C.c_int),
        "dd_residual": ([P, D, D, D, D, D, D, D], C.c_int),
        "dd_residual_device_noalloc": ([P, P, P, P, P, P, P, P, P], C.c_int),
        "dd_apply_operator_device": ([P, P, P, P], C.c_int),
        "dd_get_state": ([P, D], C.c_int),
        "dd_set_state": ([P, D], C.c_int),
        "dd_time_sweep": ([P, C.c_int, C.c_int, D, D], C.c_int),
        "dd_layout": ([P, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "dd_mesh_coords": ([C.POINTER(dd_mesh), C.c_int, D, D], C.c_int),
        "dd_batch_setup": ([C.POINTER(P), C.c_int, C.POINTER(dd_problem),
                            C.POINTER(dd_options)], C.c_int),
        "dd_batch_destroy": ([P], None),
        "dd_batch_handle": ([P, C.c_int, C.POINTER(P)], C.c_int),
        "dd_batch_solve": ([P, C.POINTER(D), C.POINTER(D), C.c_double, C.c_int, C.POINTER(D),
                            C.POINTER(D), C.POINTER(dd_stats), C.POINTER(C.c_int)], C.c_int),
        "dd_batch_time_sweep": ([P, C.c_int, C.c_int, D, D, C.POINTER(C.c_int)], C.c_int),
        "dd_batch_launches": ([P, I64], C.c_int),
        "dd_batch_wait_progress": ([P, C.c_int, C.POINTER(C.c_int)], C.c_int),
        "dd_batch_solve_start": ([P, C.POINTER(D), C.POINTER(D), C.c_double, C.c_int,
                                  C.POINTER(D), C.POINTER(D), C.POINTER(dd_stats),
                                  C.POINTER(C.c_int)], C.c_int),
        "dd_batch_solve_finish": ([P], C.c_int),
        "dd_engine_create": ([C.POINTER(P), C.c_size_t, C.c_int, C.POINTER(dd_options)],
                             C.c_int),
        "dd_engine_destroy": ([P], None),
        "dd_engine_submit": ([P, C.POINTER(dd_problem), D, D, C.c_double, C.c_int, I64],
                             C.c_int),
        "dd_engine_status": ([P, C.c_int64, C.POINTER(C.c_int)], C.c_int),
        "dd_engine_wait": ([P, C.c_int64, D, D, C.POINTER(dd_stats), D], C.c_int),
        "dd_engine_get_info": ([P, C.POINTER(dd_engine_info)], C.c_int),
        "dd_engine_wait_any": ([P, I64], C.c_int),
        "dd_set_progress": ([P, PROGRESS_FN, P, C.c_int], C.c_int),
        "dd3_setup": ([C.POINTER(P), C.POINTER(dd_box), C.c_int, D, C.c_double,
                       C.POINTER(dd_partition3), C.POINTER(dd_options)], C.c_int),
        "dd3_destroy": ([P], None),
        "dd3_sizes": ([P, I64, I64, I64, I64], C.c_int),
        "dd3_time_steps": ([P, C.POINTER(C.c_int)], C.c_int),
        "dd3_mesh_coords": ([C.POINTER(dd_box), C.c_int, D, D, D], C.c_int),
        "dd3_sweep": ([P, D, D, D, D, C.c_double, D, D, D, D, C.POINTER(C.c_int)], C.c_int),
        "dd3_time_sweep": ([P, C.c_int, C.c_int, D, D], C.c_int),
        "dd3_apply_operator_device": ([P, P, P, P], C.c_int),
        "dd3_solve": ([P, D, D, C.c_double, C.c_int, D, D, C.POINTER(dd_stats)], C.c_int),
        "dd3_residual": ([P, D, D, D, D, D], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def require_gpu():
    """Raise unless the library loads and a GPU is visible."""
    load()
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the wavedd path runs only on the GPU")


def _check(rc, allow=()):
    if rc != DD_OK and rc not in allow:
        raise WaveddError(rc, load().dd_last_error().decode())
    return rc


def _dp(a):
    """Pointer to a float64 numpy array, or NULL for None."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def dd_default_options(**kw):
    o = dd_options()
    _check(load().dd_default_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def dd_setup(nx, ny, degree, wavespeed, omega, sx, sy, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
             options=None):
    """Create a handle (returns an opaque c_void_p)."""
    lib = load()
    mesh = dd_mesh(nx, ny, x0, x1, y0, y1)
    part = dd_partition(sx, sy)
    c = _f64(wavespeed)
    h = C.c_void_p()
    _check(lib.dd_setup(C.byref(h), C.byref(mesh), degree, _dp(c), omega, C.byref(part),
                        C.byref(options) if options is not None else None))
    return h


def dd_destroy(h):
    load().dd_destroy(h)


def dd_last_error():
    return load().dd_last_error().decode()


def dd_sizes(h):
    v = [C.c_int64() for _ in range(5)]
    _check(load().dd_sizes(h, *[C.byref(x) for x in v]))
    return dict(zip(["n_global", "n_local", "n_sub", "n_iface", "n_trace"], [x.value for x in v]))


def dd_node_coords(h):
    n = dd_sizes(h)["n_global"]
    x, y = np.empty(n), np.empty(n)
    _check(load().dd_node_coords(h, _dp(x), _dp(y)))
    return x, y


def dd_time_steps(h):
    n = dd_sizes(h)["n_sub"]
    out = (C.c_int * n)()
    _check(load().dd_time_steps(h, out))
    return np.array(out[:], dtype=np.int64)


_progress_keep = {}


def dd_set_progress(h, fn=None, every=10):
    """Call fn(outer_iters, rel_residual) every `every` outer iterations of
    the handle's solves (fn=None switches it off)."""
    key = h.value
    if fn is None:
        _check(load().dd_set_progress(h, PROGRESS_FN(), None, 1))
        _progress_keep.pop(key, None)
        return
    cb = PROGRESS_FN(lambda _u, it, rel: fn(it, rel))
    _progress_keep[key] = cb   # keep the thunk alive while the library holds it
    _check(load().dd_set_progress(h, cb, None, every))


def dd_layout(h):
    lay, wg = C.c_int(), C.c_int()
    _check(load().dd_layout(h, C.byref(lay), C.byref(wg)))
    return lay.value, wg.value


def dd_solve(h, f=None, g=None, tol=1e-8, max_iter=1000, allow_notconv=False):
    """Host-array solve; f (N) and g (boundary trace) complex or real.
    Returns (u complex N-array, stats dict, return code)."""
    s = dd_sizes(h)
    f_re = f_im = g_re = g_im = None
    if f is not None:
        f = np.asarray(f)
        f_re, f_im = _f64(f.real), _f64(f.imag) if np.iscomplexobj(f) else None
    if g is not None:
        g = np.asarray(g)
        g_re, g_im = _f64(g.real), _f64(np.imag(g))
    u_re, u_im = np.empty(s["n_global"]), np.empty(s["n_global"])
    st = dd_stats()
    rc = load().dd_solve(h, _dp(f_re), _dp(f_im), _dp(g_re), _dp(g_im), tol, max_iter,
                         _dp(u_re), _dp(u_im), C.byref(st))
    _check(rc, (DD_ENOTCONV,) if allow_notconv else ())
    return u_re + 1j * u_im, st.as_dict(), rc


def dd_solve_device(h, f_re, f_im=None, g_re=None, g_im=None, tol=1e-8, max_iter=1000,
                    u_re=None, u_im=None, u_sub=None, stream=None, allow_notconv=False):
    """Device solve on torch CUDA float64 tensors (outputs preallocated)."""
    def ptr(t):
        return None if t is None else C.c_void_p(t.data_ptr())
    st = dd_stats()
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    rc = load().dd_solve_device(h, sp, ptr(f_re), ptr(f_im), ptr(g_re), ptr(g_im), tol, max_iter,
                                ptr(u_re), ptr(u_im), ptr(u_sub), C.byref(st))
    _check(rc, (DD_ENOTCONV,) if allow_notconv else ())
    return st.as_dict(), rc


def dd_sweep(h, g_in, f=None, src=1.0, want_u=True):
    """One DD cycle; g_in complex in the g layout.  Returns (g_out, u_sub,
    wh_iters)."""
    s = dd_sizes(h)
    g_in = np.asarray(g_in, dtype=complex)
    g_re, g_im = _f64(g_in.real), _f64(g_in.imag)
    f_re = f_im = None
    if f is not None:
        f = np.asarray(f)
        f_re = _f64(f.real)
        f_im = _f64(f.imag) if np.iscomplexobj(f) else None
    go_re, go_im = np.empty(s["n_iface"]), np.empty(s["n_iface"])
    nn = s["n_sub"] * s["n_local"]
    u_re = np.empty(nn) if want_u else None
    u_im = np.empty(nn) if want_u else None
    its = (C.c_int * s["n_sub"])()
    _check(load().dd_sweep(h, _dp(g_re), _dp(g_im), _dp(f_re), _dp(f_im), src, _dp(go_re),
                           _dp(go_im), _dp(u_re), _dp(u_im), its))
    u = (u_re + 1j * u_im) if want_u else None
    return go_re + 1j * go_im, u, np.array(its[:])


def dd_apply_stiffness(h, p):
    p = _f64(p)
    q = np.empty_like(p)
    _check(load().dd_apply_stiffness(h, _dp(p), _dp(q)))
    return q


def dd_residual(h, u, f=None, g=None):
    u = np.asarray(u, dtype=complex)
    f_re = f_im = g_re = g_im = None
    if f is not None:
        f = np.asarray(f)
        f_re = _f64(f.real)
        f_im = _f64(f.imag) if np.iscomplexobj(f) else None
    if g is not None:
        g = np.asarray(g)
        g_re, g_im = _f64(g.real), _f64(np.imag(g))
    rel = C.c_double()
    _check(load().dd_residual(h, _dp(_f64(u.real)), _dp(_f64(u.imag)), _dp(f_re), _dp(f_im),
                              _dp(g_re), _dp(g_im), C.byref(rel)))
    return rel.value


def dd_residual_device_noalloc(h, u_re, u_im=None, f_re=None, f_im=None, g_re=None, g_im=None,
                               out=None, stream=None):
    """||b - S u|| / ||b|| on torch float64 device tensors without device
    allocation by the library; written to out[0] (a float64 device tensor,
    allocated here when not given) in stream order."""
    import torch
    def ptr(t):
        return None if t is None else C.c_void_p(t.data_ptr())
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=u_re.device)
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().dd_residual_device_noalloc(h, sp, ptr(u_re), ptr(u_im), ptr(f_re), ptr(f_im),
                                             ptr(g_re), ptr(g_im), ptr(out)))
    return out


def dd_apply_operator_device(h, x, y, stream=None):
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().dd_apply_operator_device(h, sp, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))


def dd_get_state(h):
    n = dd_sizes(h)["n_iface"]
    G = np.empty(2 * n)
    _check(load().dd_get_state(h, _dp(G)))
    return G[0::2] + 1j * G[1::2]


def dd_set_state(h, G):
    G = np.asarray(G, dtype=complex)
    buf = np.empty(2 * G.size)
    buf[0::2], buf[1::2] = G.real, G.imag
    _check(load().dd_set_state(h, _dp(buf)))


def dd_time_sweep(h, reps=10, fixed_iters=0):
    ms, du = C.c_double(), C.c_double()
    _check(load().dd_time_sweep(h, reps, fixed_iters, C.byref(ms), C.byref(du)))
    return ms.value, du.value


def dd_mesh_coords(nx, ny, degree, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """Global GLL node coordinates of a mesh (host computation, no handle)."""
    mesh = dd_mesh(nx, ny, x0, x1, y0, y1)
    n = (nx * degree + 1) * (ny * degree + 1)
    x, y = np.empty(n), np.empty(n)
    _check(load().dd_mesh_coords(C.byref(mesh), degree, _dp(x), _dp(y)))
    return x, y


def _problem(spec):
    """(dd_problem, keep-alive wavespeed array) from a dict with keys nx, ny,
    P, x0, x1, y0, y1, sx, sy, omega, c (nodal wavespeed array)."""
    c = _f64(spec["c"])
    q = dd_problem(dd_mesh(spec["nx"], spec["ny"], spec["x0"], spec["x1"], spec["y0"], spec["y1"]),
                   spec["P"], _dp(c), spec["omega"], dd_partition(spec["sx"], spec["sy"]))
    return q, c


def workload_spec(wl):
    """Problem dict of a workload with its wavespeed and source sampled at
    the mesh's GLL nodes."""
    X, Y = dd_mesh_coords(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
    return dict(nx=wl.nx, ny=wl.ny, P=wl.P, x0=wl.x0, x1=wl.x1, y0=wl.y0, y1=wl.y1, sx=wl.sx,
                sy=wl.sy, omega=wl.omega, c=np.asarray(wl.c(X, Y), dtype=float),
                f=np.asarray(wl.f(X, Y), dtype=float), tol=wl.tol, X=X, Y=Y)


def dd_batch_setup(specs, options=None):
    """Batch of problem dicts (see _problem).  Returns an opaque pointer."""
    qs = [_problem(s) for s in specs]
    arr = (dd_problem * len(qs))(*[q for q, _ in qs])
    b = C.c_void_p()
    _check(load().dd_batch_setup(C.byref(b), len(qs), arr,
                                 C.byref(options) if options is not None else None))
    return b


def dd_batch_destroy(b):
    load().dd_batch_destroy(b)


def dd_batch_handle(b, i):
    h = C.c_void_p()
    _check(load().dd_batch_handle(b, i, C.byref(h)))
    return h


def dd_batch_solve(b, fs, tol=1e-8, max_iter=1000, allow_notconv=False, progress=None):
    """Solve every problem of the batch; fs: list of real nodal sources (or
    None).  progress(k): called each time the k-th problem finishes.
    Returns (list of complex u, list of stats dicts, per-problem codes,
    overall code)."""
    n = len(fs)
    sizes = [dd_sizes(dd_batch_handle(b, i))["n_global"] for i in range(n)]
    keep = [None if f is None else _f64(f) for f in fs]
    PD = C.POINTER(C.c_double)
    f_re = (PD * n)(*[_dp(f) if f is not None else PD() for f in keep])
    ure = [np.empty(m) for m in sizes]
    uim = [np.empty(m) for m in sizes]
    u_re = (PD * n)(*[_dp(u) for u in ure])
    u_im = (PD * n)(*[_dp(u) for u in uim])
    st = (dd_stats * n)()
    rcs = (C.c_int * n)()
    lib = load()
    _check(lib.dd_batch_solve_start(b, f_re, None, tol, max_iter, u_re, u_im, st, rcs))
    done = 0
    if progress is not None:
        while done < n:
            done = dd_batch_wait_progress(b, done)
            progress(done)
    rc = lib.dd_batch_solve_finish(b)
    _check(rc, (DD_ENOTCONV,) if allow_notconv else ())
    return ([ure[i] + 1j * uim[i] for i in range(n)], [st[i].as_dict() for i in range(n)],
            list(rcs), rc)


def dd_batch_time_sweep(b, reps=5, fixed_iters=5):
    ms, du, nl = C.c_double(), C.c_double(), C.c_int()
    _check(load().dd_batch_time_sweep(b, reps, fixed_iters, C.byref(ms), C.byref(du),
                                      C.byref(nl)))
    return ms.value, du.value, nl.value


def dd_batch_wait_progress(b, seen):
    """Block until more than `seen` problems of a running dd_batch_solve have
    finished; returns the count."""
    v = C.c_int()
    _check(load().dd_batch_wait_progress(b, seen, C.byref(v)))
    return v.value


def dd_batch_launches(b):
    v = C.c_int64()
    _check(load().dd_batch_launches(b, C.byref(v)))
    return v.value


def dd_engine_create(budget_bytes, max_active, options=None):
    e = C.c_void_p()
    _check(load().dd_engine_create(C.byref(e), int(budget_bytes), max_active,
                                   C.byref(options) if options is not None else None))
    return e


def dd_engine_destroy(e):
    load().dd_engine_destroy(e)


def dd_engine_submit(e, spec, f=None, tol=1e-6, max_iter=1000):
    q, keep = _problem(spec)
    fr = _f64(f)
    rid = C.c_int64()
    _check(load().dd_engine_submit(e, C.byref(q), _dp(fr), None, tol, max_iter, C.byref(rid)))
    return rid.value


def dd_engine_status(e, rid):
    s = C.c_int()
    _check(load().dd_engine_status(e, rid, C.byref(s)))
    return s.value


def dd_engine_wait(e, rid, n_global, allow_notconv=False):
    """Block for request rid; returns (u complex, stats dict, (t_submit,
    t_start, t_done), code)."""
    ure, uim = np.empty(n_global), np.empty(n_global)
    st = dd_stats()
    t = np.empty(3)
    rc = load().dd_engine_wait(e, rid, _dp(ure), _dp(uim), C.byref(st), _dp(t))
    _check(rc, (DD_ENOTCONV,) if allow_notconv else ())
    return ure + 1j * uim, st.as_dict(), tuple(t), rc


def dd_engine_wait_any(e):
    """Id of some finished, not yet collected request (blocks)."""
    rid = C.c_int64()
    _check(load().dd_engine_wait_any(e, C.byref(rid)))
    return rid.value


def dd_engine_get_info(e):
    info = dd_engine_info()
    _check(load().dd_engine_get_info(e, C.byref(info)))
    return info.as_dict()


class Problem:
    """Convenience owner of a handle built from a workload description
    (mesh, degree, partition, omega, wavespeed and source callables)."""

    def __init__(self, wl, precision=DD_FP64, layout=DD_LAYOUT_AUTO, tau_in=None, **opt):
        self.wl = wl
        o = dd_default_options(precision=precision, layout=layout,
                               tau_in=wl.tau_in if tau_in is None else tau_in, **opt)
        # sample the wavespeed at the library's own node coordinates
        self.X, self.Y = dd_mesh_coords(wl.nx, wl.ny, wl.P, wl.x0, wl.x1, wl.y0, wl.y1)
        self.c = np.asarray(wl.c(self.X, self.Y), dtype=float)
        self.f = np.asarray(wl.f(self.X, self.Y), dtype=float)
        self.h = dd_setup(wl.nx, wl.ny, wl.P, self.c, wl.omega, wl.sx, wl.sy, wl.x0, wl.x1,
                          wl.y0, wl.y1, o)

    def solve(self, tol=None, max_iter=2000, allow_notconv=False):
        return dd_solve(self.h, self.f, None, self.wl.tol if tol is None else tol, max_iter,
                        allow_notconv)

    def close(self):
        if self.h is not None:
            dd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Box (3D) decomposition, include/wavedd3.h
# ---------------------------------------------------------------------------
def dd3_setup(nx, ny, nz, degree, wavespeed, omega, sx, sy, sz, x0=-1.0, x1=1.0, y0=-1.0,
              y1=1.0, z0=-1.0, z1=1.0, options=None):
    """Create a box handle (returns an opaque c_void_p)."""
    lib = load()
    box = dd_box(x0, x1, y0, y1, z0, z1, nx, ny, nz)
    part = dd_partition3(sx, sy, sz)
    c = _f64(wavespeed)
    h = C.c_void_p()
    _check(lib.dd3_setup(C.byref(h), C.byref(box), degree, _dp(c), omega, C.byref(part),
                         C.byref(options) if options is not None else None))
    return h


def dd3_destroy(h):
    load().dd3_destroy(h)


def dd3_sizes(h):
    v = [C.c_int64() for _ in range(4)]
    _check(load().dd3_sizes(h, *[C.byref(x) for x in v]))
    return dict(zip(["n_global", "n_local", "n_sub", "n_iface"], [x.value for x in v]))


def dd3_time_steps(h):
    n = dd3_sizes(h)["n_sub"]
    out = (C.c_int * n)()
    _check(load().dd3_time_steps(h, out))
    return np.array(out[:], dtype=np.int64)


def dd3_mesh_coords(nx, ny, nz, degree, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, z0=-1.0, z1=1.0):
    """Global GLL node coordinates of a box (no handle)."""
    box = dd_box(x0, x1, y0, y1, z0, z1, nx, ny, nz)
    n = (nx * degree + 1) * (ny * degree + 1) * (nz * degree + 1)
    x, y, z = np.empty(n), np.empty(n), np.empty(n)
    _check(load().dd3_mesh_coords(C.byref(box), degree, _dp(x), _dp(y), _dp(z)))
    return x, y, z


def dd3_sweep(h, g_in=None, f=None, src=1.0, want_u=True):
    """One DD cycle on the box; g_in complex in the g layout (None = 0).
    Returns (g_out, u_sub, wh_iters)."""
    s = dd3_sizes(h)
    g_re = g_im = None
    if g_in is not None:
        g_in = np.asarray(g_in, dtype=complex)
        g_re, g_im = _f64(g_in.real), _f64(g_in.imag)
    f_re = f_im = None
    if f is not None:
        f = np.asarray(f)
        f_re = _f64(f.real)
        f_im = _f64(f.imag) if np.iscomplexobj(f) else None
    go_re, go_im = np.empty(s["n_iface"]), np.empty(s["n_iface"])
    nn = s["n_sub"] * s["n_local"]
    u_re = np.empty(nn) if want_u else None
    u_im = np.empty(nn) if want_u else None
    its = (C.c_int * s["n_sub"])()
    _check(load().dd3_sweep(h, _dp(g_re), _dp(g_im), _dp(f_re), _dp(f_im), src, _dp(go_re),
                            _dp(go_im), _dp(u_re), _dp(u_im), its))
    u = (u_re + 1j * u_im) if want_u else None
    return go_re + 1j * go_im, u, np.array(its[:])


def dd3_time_sweep(h, reps=10, fixed_iters=0):
    ms, du = C.c_double(), C.c_double()
    _check(load().dd3_time_sweep(h, reps, fixed_iters, C.byref(ms), C.byref(du)))
    return ms.value, du.value


def dd3_apply_operator_device(h, x, y, stream=None):
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().dd3_apply_operator_device(h, sp, C.c_void_p(x.data_ptr()),
                                            C.c_void_p(y.data_ptr())))


def dd3_solve(h, f=None, tol=1e-8, max_iter=1000, allow_notconv=False):
    """Box solve from host arrays; f at the global nodes (real or complex).
    Returns (u complex N-array, stats dict, return code)."""
    n = dd3_sizes(h)["n_global"]
    f_re = f_im = None
    if f is not None:
        f = np.asarray(f)
        f_re = _f64(f.real)
        f_im = _f64(f.imag) if np.iscomplexobj(f) else None
    u_re, u_im = np.empty(n), np.empty(n)
    st = dd_stats()
    rc = load().dd3_solve(h, _dp(f_re), _dp(f_im), tol, max_iter, _dp(u_re), _dp(u_im),
                          C.byref(st))
    _check(rc, (DD_ENOTCONV,) if allow_notconv else ())
    return u_re + 1j * u_im, st.as_dict(), rc


def dd3_residual(h, u, f=None):
    u = np.asarray(u, dtype=complex)
    f_re = f_im = None
    if f is not None:
        f = np.asarray(f)
        f_re = _f64(f.real)
        f_im = _f64(f.imag) if np.iscomplexobj(f) else None
    rel = C.c_double()
    _check(load().dd3_residual(h, _dp(_f64(u.real)), _dp(_f64(u.imag)), _dp(f_re), _dp(f_im),
                               C.byref(rel)))
    return rel.value
