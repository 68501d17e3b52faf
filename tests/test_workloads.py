"""CPU checks of the seeded workload generators: the shapes the benchmarks
and parity tests rely on (no GPU)."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("name", sorted(workloads.CONFIGS3))
def test_box_workloads_fit_one_node_per_thread(name):
    """Every box workload's subdomain fits one workgroup (<= 1024 nodes),
    its partition divides the mesh, and omega gives 10 GLL points per
    wavelength at c = 1."""
    wl = workloads.CONFIGS3[name]()
    assert wl.nx % wl.sx == 0 and wl.ny % wl.sy == 0 and wl.nz % wl.sz == 0
    nloc = ((wl.nx // wl.sx) * wl.P + 1) * ((wl.ny // wl.sy) * wl.P + 1) * \
        ((wl.nz // wl.sz) * wl.P + 1)
    assert nloc <= 1024
    h = (wl.box[1] - wl.box[0]) / wl.nx
    wavelength = 2 * np.pi / wl.omega
    assert wavelength / (h / wl.P) == pytest.approx(10.0)


def test_box_workload_sizes():
    assert (workloads.c6().nx, workloads.c6().P, workloads.c6().sx) == (64, 3, 32)
    assert (workloads.c6_p1().nx, workloads.c6_p1().P, workloads.c6_p1().sx) == (128, 1, 16)


def test_box_workload_fields_are_seeded_and_smooth():
    wl = workloads.c6_small()
    x = np.linspace(-1, 1, 5)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    assert np.all(wl.c(X, Y, Z) == 1.0)
    f = wl.f(X, Y, Z)
    assert f.max() <= 1.0 and f.min() > 0.0
    assert np.array_equal(f, workloads.c6_small().f(X, Y, Z))


# ---- 2D workloads: the recipe the benchmarks and parity tests rely on ----

@pytest.mark.parametrize("name,shape", [("c1", (16, 2, 2)), ("c2", (256, 3, 16)),
                                        ("c2_small", (64, 3, 4)), ("c2_t1", (256, 3, 32)),
                                        ("c3", (512, 3, 8))])
def test_square_workload_shapes(name, shape):
    wl = workloads.CONFIGS[name]()
    assert (wl.nx, wl.P, wl.sx) == shape and wl.ny == wl.nx and wl.sy == wl.sx
    assert wl.nx % wl.sx == 0
    assert wl.tol == 1e-8 and wl.tau_in == 1e-12


@pytest.mark.parametrize("name,ppw", [("c2", 10.0), ("c2_small", 10.0), ("c3", 20.0)])
def test_waveguide_workloads_resolve_the_core(name, ppw):
    """omega gives 10 GLL points per wavelength at the core speed 1/3 (c3:
    the c2 problem, same omega, on a mesh twice as fine), and the sampled
    wavespeed spans the core and background values."""
    wl = workloads.CONFIGS[name]()
    h = (wl.x1 - wl.x0) / wl.nx
    wavelength = 2 * np.pi * (1.0 / 3.0) / wl.omega
    assert wavelength / (h / wl.P) == pytest.approx(ppw)
    g = np.linspace(0.0, 1.0, 401)
    X, Y = np.meshgrid(g, g)
    c = wl.c(X, Y)
    assert c.min() == pytest.approx(1.0 / 3.0, abs=1e-3)
    assert c.max() == pytest.approx(1.0, abs=1e-6)
    assert np.all((c >= 1.0 / 3.0 - 1e-12) & (c <= 1.0 + 1e-12))


def test_c4_batch_recipe():
    """400 subdomains over independent problems, P in 1..4, 8..64 elements
    per subdomain side, 10 points per wavelength at the field's slowest
    speed, seeded."""
    a, b = workloads.c4(), workloads.c4()
    assert sum(w.sx * w.sy for w in a) == 400
    for w, w2 in zip(a, b):
        assert (w.nx, w.ny, w.P, w.sx, w.sy, w.x0, w.y0) == \
            (w2.nx, w2.ny, w2.P, w2.sx, w2.sy, w2.x0, w2.y0)
        assert 1 <= w.P <= 4 and w.nx % w.sx == 0 and w.ny % w.sy == 0
        assert 8 <= w.nx // w.sx <= 64 and w.nx // w.sx == w.ny // w.sy
        h = (w.x1 - w.x0) / w.nx
        assert (w.y1 - w.y0) / w.ny == pytest.approx(h)
        assert 2 * np.pi * w.c.cmin / w.omega / (h / w.P) == pytest.approx(10.0)
        assert w.tol == 1e-6 and w.tau_in == 1e-5


def test_c5_request_recipe():
    """Every request: omega in [10, 80], P in {2, 3, 4}, s in {16, 24, ..., 64}
    elements per subdomain side, g x g subdomains with ceil(64/s) <= g <=
    floor(512/s), at least 8 points per wavelength at the slowest speed,
    1-4 sources; the stream is seeded."""
    a, b = workloads.c5(n_requests=300), workloads.c5(n_requests=300)
    for w, w2 in zip(a, b):
        assert (w.nx, w.P, w.sx, w.omega) == (w2.nx, w2.P, w2.sx, w2.omega)
        assert 10.0 <= w.omega <= 80.0 and w.P in (2, 3, 4)
        s = w.nx // w.sx
        assert w.nx == s * w.sx and w.ny == w.nx and w.sy == w.sx
        assert s in range(16, 65, 8)
        assert -(-64 // s) <= w.sx <= 512 // s
        assert w.tol == 1e-6
    # points per wavelength at the slowest sampled speed.  (n, P) are drawn
    # for the slowest speed of the field and of the slower core; where two
    # waveguides share their stem the speeds multiply, so a request with two
    # cores can fall below 8 there, by at most the other core's factor (>= 1/3)
    g = np.linspace(0.0, 1.0, 129)
    X, Y = np.meshgrid(g, g)
    ppw = np.array([2 * np.pi * w.c(X, Y).min() / w.omega * w.nx * w.P for w in a[:120]])
    assert ppw.min() >= 8.0 / 3.0
    assert (ppw >= 8.0 * (1 - 1e-9)).mean() >= 0.9


def test_lognormal_field_contrast():
    """log c is scaled so that max c / min c is the contrast (3) over the
    unit period."""
    c = workloads.lognormal_field(11)
    g = np.linspace(0.0, 1.0, 257)
    X, Y = np.meshgrid(g, g)
    v = c(X, Y)
    assert v.max() / v.min() <= 3.0 * (1 + 1e-12)
    assert v.min() >= c.cmin * (1 - 1e-12)
    assert max(v.max(), 1.0 / v.min()) == pytest.approx(np.sqrt(3.0), rel=1e-12)
