"""GPU: the no-allocation residual entry point (row partials in a library
array instead of an allocated buffer) against dd_residual on the same
inputs, on two calls in a row, the second with a smaller problem.

The two sum the same per-node values in different orders (rows of the grid
against fixed chunks of the node list), so they agree to rounding: 1e-12
relative."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(W, nx, ny, P, sx, sy, omega, seed):
    X, Y = W.dd_mesh_coords(nx, ny, P)
    c = 1.0 + 0.3 * np.sin(4 * X + 0.5) * np.cos(3 * Y - 0.1)
    h = W.dd_setup(nx, ny, P, c, omega, sx, sy, options=W.dd_default_options(tau_in=1e-10))
    rng = np.random.default_rng(seed)
    N = X.size
    n_tr = 2 * (ny * P + 1) + 2 * (nx * P + 1)
    u = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    g = rng.standard_normal(n_tr) + 1j * rng.standard_normal(n_tr)
    return h, u, f, g


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_noalloc_residual_matches_dd_residual(gpu_lib):
    import torch
    W = gpu_lib
    lib = W.load()
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    # larger problem first, then a smaller one: the second call reuses the
    # array the first one filled further
    for (nx, ny, P, sx, sy, om, seed) in ((48, 40, 3, 4, 2, 20.0, 1), (6, 4, 2, 2, 2, 9.0, 2)):
        h, u, f, g = _problem(W, nx, ny, P, sx, sy, om, seed)
        try:
            ref = W.dd_residual(h, u, f, g)
            args = [_dev(torch, x) for x in (u.real, u.imag, f.real, f.imag, g.real, g.imag)]
            torch.cuda.synchronize()
            rc = lib.dd_residual_device_noalloc(
                h, None, *[C.c_void_p(a.data_ptr()) for a in args], C.c_void_p(out.data_ptr()))
            assert rc == 0, W.dd_last_error()
            torch.cuda.synchronize()
            got = float(out.cpu()[0])
            # source only (g and the imaginary parts absent)
            ref_f = W.dd_residual(h, u, f.real)
            got_f = float(W.dd_residual_device_noalloc(h, args[0], args[1], args[2])[0].cpu())
        finally:
            W.dd_destroy(h)
        print(f"{nx}x{ny} P={P}: noalloc {got:.15e} dd_residual {ref:.15e}", flush=True)
        assert abs(got - ref) <= 1e-12 * ref
        assert abs(got_f - ref_f) <= 1e-12 * ref_f


def test_noalloc_residual_rejects_too_many_rows(gpu_lib):
    """A mesh with more grid rows than the scratch array holds is refused
    before any launch, with a message naming the limit."""
    import torch
    W = gpu_lib
    # a 2 x 4096 strip of unit elements at P = 4: Ny = 16385 > 16384
    nx, ny, P = 2, 4096, 4
    box = (0.0, 2.0, 0.0, 4096.0)
    X, Y = W.dd_mesh_coords(nx, ny, P, *box)
    h = W.dd_setup(nx, ny, P, np.ones(X.size), 2.0, 1, 64, *box)
    try:
        u = torch.zeros(X.size, dtype=torch.float64, device="cuda")
        with pytest.raises(W.WaveddError) as ei:
            W.dd_residual_device_noalloc(h, u)
        assert ei.value.code == W.DD_EINVAL and "16384" in str(ei.value)
    finally:
        W.dd_destroy(h)
