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
DD_LAYOUT_AUTO, DD_LAYOUT_NODE, DD_LAYOUT_PATCH, DD_LAYOUT_PATCH_XCHG = 0, 1, 2, 3
DD_OUTER_GMRES, DD_OUTER_FIXED = 0, 1

EXPORTS = [
    "dd_default_options", "dd_setup", "dd_destroy", "dd_last_error", "dd_sizes",
    "dd_node_coords", "dd_time_steps", "dd_solve", "dd_solve_device", "dd_sweep",
    "dd_apply_stiffness", "dd_residual", "dd_apply_operator_device", "dd_get_state",
    "dd_set_state", "dd_time_sweep", "dd_layout",
]


class dd_mesh(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x0", C.c_double), ("x1", C.c_double),
                ("y0", C.c_double), ("y1", C.c_double)]


class dd_partition(C.Structure):
    _fields_ = [("sx", C.c_int), ("sy", C.c_int)]


class dd_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("layout", C.c_int), ("tau_in", C.c_double),
                ("max_wh", C.c_int), ("outer", C.c_int), ("restart", C.c_int),
                ("nt_override", C.c_int), ("cfl", C.c_double), ("refine", C.c_int),
                ("relax", C.c_double)]


class dd_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("sweeps", C.c_int), ("rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("wh_iters_total", C.c_int64),
                ("wh_iters_max", C.c_int), ("nt_min", C.c_int), ("nt_max", C.c_int),
                ("dof_updates", C.c_double), ("sweep_seconds", C.c_double),
                ("seconds", C.c_double), ("refine_steps", C.c_int), ("fp64_sweeps", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


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
        "dd_apply_operator_device": ([P, P, P, P], C.c_int),
        "dd_get_state": ([P, D], C.c_int),
        "dd_set_state": ([P, D], C.c_int),
        "dd_time_sweep": ([P, C.c_int, C.c_int, D, D], C.c_int),
        "dd_layout": ([P, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
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


class Problem:
    """Convenience owner of a handle built from a workload description
    (mesh, degree, partition, omega, wavespeed and source callables)."""

    def __init__(self, wl, precision=DD_FP64, layout=DD_LAYOUT_AUTO, tau_in=None, **opt):
        self.wl = wl
        o = dd_default_options(precision=precision, layout=layout,
                               tau_in=wl.tau_in if tau_in is None else tau_in, **opt)
        # sample the wavespeed at the library's own node coordinates
        probe = dd_setup(wl.nx, wl.ny, wl.P, np.ones((wl.nx * wl.P + 1) * (wl.ny * wl.P + 1)),
                         wl.omega, wl.sx, wl.sy, wl.x0, wl.x1, wl.y0, wl.y1, o)
        try:
            self.X, self.Y = dd_node_coords(probe)
        finally:
            dd_destroy(probe)
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
