"""The oracle DD sweep on a pool of host processes (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Within one sweep every subdomain solve reads only the previous interface data
(Sec. III: the subdomain problems of one DD cycle are independent; Sec. VI
runs them concurrently), so the solves of one sweep may run on several
processes.  Each worker process builds the same ``dd.Decomposition`` and
owns a fixed set of subdomains, whose sparse LU factors it keeps between
sweeps.  Every slot of the output interface vector is written by exactly one
subdomain (the one facing it), so the parent assembles the sweep by adding
the workers' disjoint contributions: the result is bit for bit the serial
``Decomposition.sweep``.  Nothing else changes: ``ParallelDecomposition``
forwards every other attribute to a local ``Decomposition`` and can be
passed to ``dd.solve_dd`` in its place.

Workers are started with the ``spawn`` method (a fresh interpreter that
imports only this package, numpy and scipy) and with one BLAS / OpenMP
thread each.
"""
import multiprocessing as mp
import os

import numpy as np

from . import dd, sem

_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS",
                "BLIS_NUM_THREADS", "NUMEXPR_NUM_THREADS")


def host_workers():
    """Worker count: the CPUs this process may run on (affinity mask), at
    most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _worker(conn, geom, own):
    mesh, part, c, omega, q = geom
    dec = dd.Decomposition(mesh, part, c, omega, q)
    f = None
    while True:
        msg = conn.recv()
        op = msg[0]
        if op == "stop":
            break
        if op == "f":
            f = msg[1]
            conn.send(True)
        elif op == "factor":
            for l in own:
                dec.lu(l)
            conn.send(True)
        elif op == "sweep":
            _, g_in, src, want_u = msg
            g_out = np.zeros(dec.n_if, dtype=complex)
            us = {}
            for l in own:
                b = dec.rhs(l, f, g_in, src)
                u = dec.lu(l).solve(b)
                dec.exchange(l, u, g_in, g_out)
                if want_u:
                    us[l] = u
            conn.send((g_out, us))


class ParallelDecomposition:
    """``dd.Decomposition`` whose exact-solve sweep runs on worker processes."""

    def __init__(self, mesh, part, c, omega, q=0.0, workers=None):
        self.dec = dd.Decomposition(mesh, part, c, omega, q)
        n = host_workers() if workers is None else int(workers)
        n = max(1, min(n, self.dec.L))
        self.workers = n
        ctx = mp.get_context("spawn")
        geom = (mesh, part, np.asarray(c, dtype=float), float(omega), float(q))
        saved = {k: os.environ.get(k) for k in _THREAD_VARS}
        self._conns, self._procs = [], []
        try:
            for k in _THREAD_VARS:
                os.environ[k] = "1"
            for w in range(n):
                own = list(range(w, self.dec.L, n))
                a, b = ctx.Pipe()
                p = ctx.Process(target=_worker, args=(b, geom, own), daemon=True)
                p.start()
                self._conns.append(a)
                self._procs.append(p)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        self._f = None

    def __getattr__(self, name):
        return getattr(self.__dict__["dec"], name)

    def _bcast(self, msg):
        for cn in self._conns:
            cn.send(msg)
        out = []
        for cn, p in zip(self._conns, self._procs):
            while not cn.poll(1.0):
                if not p.is_alive():
                    raise RuntimeError(f"oracle worker {p.pid} ended (exit code {p.exitcode})")
            out.append(cn.recv())
        return out

    def factor(self):
        """Factor every subdomain system on its worker (otherwise done by the
        first sweep)."""
        self._bcast(("factor",))

    def _set_f(self, f):
        f = None if f is None else np.asarray(f, dtype=complex)
        same = (self._f is None and f is None) or (
            self._f is not None and f is not None and self._f.shape == f.shape
            and np.array_equal(self._f, f))
        if not same:
            self._f = None if f is None else f.copy()
            self._bcast(("f", self._f if self._f is not None else
                         np.zeros(self.dec.mesh.N, dtype=complex)))

    def sweep(self, g_in, f, src, solver=None, want_u=True):
        """Same result as ``Decomposition.sweep`` with exact LU solves."""
        if solver is not None:
            raise ValueError("the process-pool sweep uses the exact subdomain LU only")
        self._set_f(f)
        g_in = np.asarray(g_in, dtype=complex)
        parts = self._bcast(("sweep", g_in, float(src), bool(want_u)))
        g_out = np.zeros(self.dec.n_if, dtype=complex)
        us = [None] * self.dec.L
        for go, ud in parts:
            g_out += go
            for l, u in ud.items():
                us[l] = u
        return g_out, (us if want_u else None)

    def close(self):
        for cn in self._conns:
            try:
                cn.send(("stop",))
            except (BrokenPipeError, OSError):
                pass
        for p in self._procs:
            p.join(timeout=10)
            if p.is_alive():
                p.terminate()
        self._conns, self._procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

