"""Pins for the oracle's spectral-element assembly (paper Sec. IV, eqs.
(3)-(5)): textbook reductions, brute force from explicit polynomials,
conservation sums and plane-wave convergence."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import brute, sem


def test_stiffness_constants_and_symmetry():
    m = sem.Rect(3, 2, 3, 0.0, 1.0, 0.0, 0.5)
    A, _, _, _ = sem.operators(m)
    assert np.abs(A @ np.ones(m.N)).max() < 1e-11
    assert abs(A - A.T).max() < 1e-12


def test_p1_is_five_point_laplacian():
    """With GLL (trapezoidal) quadrature and square elements, Q1 stiffness is
    the textbook 5-point Laplacian kron(I,T) + kron(T,I), T=tridiag(-1,2,-1)
    with halved diagonal entries at the two ends (Neumann rows)."""
    n = 5
    m = sem.Rect(n, n, 1)
    A, _, _, _ = sem.operators(m)
    T = sp.diags([-np.ones(n), 2 * np.ones(n + 1), -np.ones(n)], [-1, 0, 1]).tolil()
    T[0, 0] = T[n, n] = 1.0
    I = sp.diags(np.r_[0.5, np.ones(n - 1), 0.5])
    ref = sp.kron(I, T) + sp.kron(T, I)
    assert abs(A - ref).max() < 1e-12


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (2, 1)])
def test_brute_force_assembly(P, shape):
    rng = np.random.default_rng(P * 10 + shape[0])
    m = sem.Rect(shape[0], shape[1], P, -0.2, 0.9, 0.1, 0.6)
    c = 0.5 + rng.random(m.N)
    f = rng.standard_normal(m.N)
    Ab, Mb, Hb, bb = brute.assemble(m, c, f)
    S, A, M, H = sem.system(m, c, 2.0)
    scale = np.abs(Ab).max()
    assert np.abs(Ab - A.toarray()).max() < 1e-13 * scale
    # quadrature at the nodes makes mass and boundary matrices diagonal
    assert np.abs(Mb - np.diag(M)).max() < 1e-15
    assert np.abs(Hb - np.diag(H)).max() < 1e-15
    assert np.abs(bb - sem.load(m, f)).max() < 1e-14


def test_mass_boundary_and_load_sums():
    m = sem.Rect(6, 4, 3, 0.0, 1.5, -0.5, 0.5)
    c = np.full(m.N, 2.0)
    _, _, M, H = sem.system(m, c, 1.0)
    assert abs(M.sum() - 1.5 * 1.0 / 4.0) < 1e-13
    assert abs(H.sum() - 2 * (1.5 + 1.0) / 2.0) < 1e-13
    X, Y = sem.node_coords(m)
    # integrate a polynomial of degree <= 2P-1 in each variable exactly
    f = X ** 5 * Y ** 3 + 1.0
    exact = (1.5 ** 6 / 6) * ((0.5 ** 4 - 0.5 ** 4) / 4) + 1.5
    assert abs(sem.load(m, f).sum() - exact) < 1e-12


def test_gaussian_load_integral():
    m = sem.Rect(16, 16, 2)
    X, Y = sem.node_coords(m)
    s = 0.05
    f = np.exp(-((X - 0.3) ** 2 + (Y - 0.6) ** 2) / (2 * s * s))
    assert abs(sem.load(m, f).sum().real - 2 * np.pi * s * s) < 1e-4 * 2 * np.pi * s * s


def test_complex_symmetric_and_real_block_symmetric():
    m = sem.Rect(3, 3, 2)
    c = 1.0 + np.random.default_rng(1).random(m.N)
    S, A, M, H = sem.system(m, c, 7.0)
    assert abs(S - S.T).max() < 1e-12               # S^T = S (not Hermitian)
    assert abs(S - S.conj().T).max() > 1.0
    om = 7.0
    Am = A.toarray()
    B = np.block([[Am - om ** 2 * np.diag(M), om * np.diag(H)],
                  [om * np.diag(H), om ** 2 * np.diag(M) - Am]])
    assert np.abs(B - B.T).max() < 1e-12           # eq. (5) is symmetric
    rng = np.random.default_rng(2)
    b = rng.standard_normal(m.N) + 1j * rng.standard_normal(m.N)
    u = np.linalg.solve(S.toarray(), b)
    z = np.linalg.solve(B, np.r_[b.real, -b.imag])
    assert np.abs(z[:m.N] + 1j * z[m.N:] - u).max() < 1e-10 * np.abs(u).max()


def test_sparse_lu_matches_dense():
    m = sem.Rect(4, 3, 3)
    c = 1.0 + 0.5 * np.random.default_rng(3).random(m.N)
    f = np.random.default_rng(4).standard_normal(m.N)
    u = sem.solve(m, c, 9.0, f)
    S, _, _, _ = sem.system(m, c, 9.0)
    ud = np.linalg.solve(S.toarray(), sem.load(m, f))
    assert np.abs(u - ud).max() < 1e-12 * np.abs(ud).max()


@pytest.mark.parametrize("P", [1, 2, 3])
def test_plane_wave_convergence(P):
    """u = exp(i k d.x) with g = i k (d.n - 1) u solves eq. (1) exactly;
    the discrete error must fall at order >= P + 1/2."""
    errs = []
    for n in (4, 8, 16):
        m = sem.Rect(n, n, P)
        ue, g = sem.plane_wave(m, 10.0, 1.0, (np.cos(0.3), np.sin(0.3)))
        uh = sem.solve(m, np.ones(m.N), 10.0, np.zeros(m.N), g)
        errs.append(np.linalg.norm(uh - ue) / np.linalg.norm(ue))
    rate = np.log2(errs[1] / errs[2])
    assert rate >= P + 0.5, errs
