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
