"""Pins of the 3-D part of the oracle: Q_p element scalings, the 27-point
coarse stencil, the 3-D decomposition and the 3-D two-grid cycle (CPU)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import fem, qsfem3d, smoother, transfer, twogrid


# ------------------------------------------------------------ Q_p in 3-D ----
@pytest.mark.parametrize("p", [1, 2, 3])
def test_3d_element_matrices_integrate_exactly(p):
    """On a cell of size h: int |grad u|^2 for u = x + 2y + 3z is 14 h^3,
    int 1 = h^3, and a face integral of 1 is h^2 (scalings h^{d-2}, h^d, h^{d-1})."""
    h = 0.37
    S, M = fem.element_matrices(p, h, 3)
    x, _ = fem.gll(p)
    X = np.array([[a, b, c] for c in x for b in x for a in x]) * h  # x fastest
    u = X @ np.array([1.0, 2.0, 3.0])
    one = np.ones(len(u))
    assert abs(u @ S @ u - 14 * h ** 3) < 1e-12
    assert abs(one @ M @ one - h ** 3) < 1e-14
    assert np.allclose(S @ one, 0.0, atol=1e-12)
    F = fem.face_matrix(p, h, 3)
    assert abs(F.sum() - h ** 2) < 1e-14


def test_3d_neumann_matrix_is_symmetric_and_annihilates_constants_without_mass():
    N, p = 3, 2
    k = np.zeros((N, N, N))
    A = fem.helmholtz_matrix(p, k, robin=(False,) * 6)
    assert abs(A - A.T).max() < 1e-14
    assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12


# ------------------------------------------------------- 27-point stencil ----
@pytest.mark.parametrize("eta", [0.4, 1.0, 1.5])
def test_27pt_symbol_vanishes_on_the_sphere_along_the_fit_directions(eta):
    P = qsfem3d.stencil_P(eta)
    for d in qsfem3d.DIRS:
        assert abs(qsfem3d.symbol(P, eta * d)) < 1e-12


def test_27pt_scaled_symbol_is_consistent_with_helmholtz():
    """N sigma(xi) - (|xi|^2 - eta^2) = o(eta^2) for |xi| ~ eta as eta -> 0."""
    rng = np.random.default_rng(0)
    dirs = rng.standard_normal((20, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    rel = []
    for eta in (0.4, 0.2, 0.1):
        P = qsfem3d.stencil_P(eta)
        N = -eta * eta / (P[0] + 6 * P[1] + 12 * P[2] + 8 * P[3])
        err = max(abs(N * qsfem3d.symbol(P, 0.7 * eta * d) - (0.49 - 1) * eta ** 2) for d in dirs)
        rel.append(err / eta ** 2)
    assert rel[1] < rel[0] / 3 and rel[2] < rel[1] / 3, rel


def _radius(f, eta):
    from scipy.optimize import brentq
    return brentq(f, 0.5 * eta, 1.5 * eta, xtol=1e-15)


def test_27pt_dispersion_is_far_below_that_of_trilinear_fe():
    """Radius of the numerical wavenumber sphere over random directions:
    relative error of the fitted stencil << that of Q1 finite elements
    (Q1 symbol: sum of 1-D stiffness x mass x mass products)."""
    eta = 1.0
    P = qsfem3d.stencil_P(eta)
    rng = np.random.default_rng(1)
    dirs = np.abs(rng.standard_normal((40, 3)))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]

    def q1(xi):
        c = np.cos(xi)
        s = 2 - 2 * c            # 1-D stiffness symbol (h = 1)
        m = (2 + c) / 3          # 1-D mass symbol
        return s[0] * m[1] * m[2] + m[0] * s[1] * m[2] + m[0] * m[1] * s[2] - eta ** 2 * m.prod()

    e27 = max(abs(_radius(lambda r: qsfem3d.symbol(P, r * d), eta) / eta - 1) for d in dirs)
    eq1 = max(abs(_radius(lambda r: q1(r * d), eta) / eta - 1) for d in dirs)
    assert e27 < eq1 / 10, (e27, eq1)


def test_27pt_quasi_fe_interior_stencil_and_absorbing_row_sums():
    """Interior row h_c N P (the 3-D cell stiffness scales as h_c); absorbing
    row sums of the face mass."""
    Nc, eta = 4, 0.9
    kc = np.full((Nc, Nc, Nc), eta * Nc)
    A = qsfem3d.coarse_matrix_3d(kc)
    n1 = Nc + 1
    P = qsfem3d.stencil_P(eta)
    Nn = -eta * eta / (P[0] + 6 * P[1] + 12 * P[2] + 8 * P[3])
    c = (2 * n1 + 2) * n1 + 2
    row = A.getrow(c).toarray().ravel()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                cls = abs(dx) + abs(dy) + abs(dz)
                assert abs(row[c + (dz * n1 + dy) * n1 + dx] - Nn * P[cls] / Nc) < 1e-13
    assert row.nonzero()[0].size == 27
    assert abs(A - A.T).max() < 1e-14
    # absorbing term -i k int_face u v: row sums of the face Q1 mass are
    # h_c^2 on a face, h_c^2 / 2 + h_c^2 / 2 on an edge, 3 h_c^2 / 4 at a corner
    hc2 = 1.0 / Nc ** 2
    k = kc[0, 0, 0]
    for node, s in [((0 * n1 + 2) * n1 + 2, 1.0), ((0 * n1 + 0) * n1 + 2, 1.0),
                    (0, 0.75)]:
        assert abs(A.getrow(node).toarray().sum().imag + k * hc2 * s) < 1e-12


# --------------------------------------------------- decomposition in 3-D ----
def test_3d_averaging_weights_partition_unity():
    N, p = 7, 2
    subs = smoother.decompose(N, p, 3, 3)
    assert len(subs) == 27
    L = smoother.multiplicity(subs, (N * p + 1) ** 3)
    tot = np.zeros_like(L)
    for s in subs:
        tot[s.u_nodes] += 1.0 / L[s.u_nodes]
    assert np.allclose(tot, 1.0)
    assert set(np.unique(L)) == {1.0, 2.0, 4.0, 8.0}


def test_3d_subdomain_matrix_rows_inside_omega_equal_global_rows():
    """Away from the boundary of Omega^(i) the local shifted matrix has the
    rows of the global shifted matrix (the absorbing terms sit only on its
    boundary faces)."""
    N, p, l_dd, alpha = 5, 2, 2, 0.5
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 3, 0.3, 1.5, 3.0, seed=3), 1.0)
    sm = smoother.CSDDSmoother(p, k, None, alpha, l_dd)
    As = fem.helmholtz_matrix(p, k, alpha=alpha).tocsr()
    n1 = N * p + 1
    checked = 0
    for s in sm.subs:
        pos = {int(g): i for i, g in enumerate(s.om_nodes)}
        for li, g in enumerate(s.om_nodes):
            g = int(g)
            ix, iy, iz = g % n1, (g // n1) % n1, g // (n1 * n1)
            inner = all(box[0] * p < c < box[1] * p
                        for c, box in zip((ix, iy, iz), s.Om))
            if not inner:
                continue
            grow = As.getrow(g)
            lrow = s.A_loc.getrow(li).toarray().ravel()
            for j, v in zip(grow.indices, grow.data):
                assert abs(lrow[pos[int(j)]] - v) < 1e-12
            checked += 1
    assert checked > 100


def test_3d_single_subdomain_smoother_is_exact_shifted_solve():
    N, p = 3, 2
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 3, 0.3, 1.5, 3.0, seed=4), 1.0)
    sm = smoother.CSDDSmoother(p, k, None, 0.4, l_dd=N)
    u = syn.random_complex(sm.n_nodes, seed=5)
    f = syn.random_complex(sm.n_nodes, seed=6)
    As = fem.helmholtz_matrix(p, k, alpha=0.4).toarray()
    A = fem.helmholtz_matrix(p, k).toarray()
    assert np.allclose(sm.apply(u, f), u + np.linalg.solve(As, f - A @ u), atol=1e-11)


@pytest.mark.parametrize("p", [2, 4])
def test_3d_prolongation_reproduces_degree_p_over_2(p):
    N = 2
    r = p // 2
    I = transfer.prolongation(N, p, 3)
    xc = np.linspace(0, 1, N * r + 1)
    xf = fem.node_coords_1d(N, p)
    f = lambda x, y, z: x ** r * y + z ** r - 2 * x * y * z
    Zc, Yc, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    Zf, Yf, Xf = np.meshgrid(xf, xf, xf, indexing="ij")
    assert np.allclose(I @ f(Xc, Yc, Zc).ravel(), f(Xf, Yf, Zf).ravel(), atol=1e-13)


# ------------------------------------------------------- 3-D two-grid -------
def test_3d_dense_solve_matches_twogrid_gmres():
    N, p = 4, 2
    k = np.full((N, N, N), 5.0)
    tg = twogrid.TwoGrid(p, k, alpha_s=0.5, l_dd=2)
    f = syn.random_complex(tg.A.shape[0], seed=3)
    x, it, _ = tg.gmres(f, 1e-12)
    ex = spla.spsolve(tg.A.tocsc(), f)
    assert np.linalg.norm(x - ex) / np.linalg.norm(ex) < 1e-10


def test_3d_twogrid_fixed_point():
    N, p = 4, 2
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 3, 0.3, 1.5, 3.0, seed=9), 1.0)
    tg = twogrid.TwoGrid(p, k, alpha_s=0.5, l_dd=2)
    f = syn.random_complex(tg.A.shape[0], seed=10)
    x = spla.spsolve(tg.A.tocsc(), f)
    assert np.linalg.norm(tg.twogrid_step(x, f) - x) / np.linalg.norm(x) < 1e-11


# ------------------------------------------------ fine dispersion in 3-D ----
@pytest.mark.parametrize("p,N", [(1, 3), (2, 2)])
def test_3d_bloch_symbol_by_periodic_brute_force(p, N):
    """eig of the assembled periodic 3-D FE matrix = union over
    theta in (2 pi / N) Z^3 of eig(A^(theta))."""
    kh = 0.7
    K1, M1 = fem.ref_matrices(p)
    kr = lambda a, b, c: np.kron(a, np.kron(b, c))
    Ae = kr(K1, M1, M1) + kr(M1, K1, M1) + kr(M1, M1, K1) - kh * kh * kr(M1, M1, M1)
    n1 = N * p
    A = np.zeros((n1 ** 3, n1 ** 3))
    for cz in range(N):
        for cy in range(N):
            for cx in range(N):
                nodes = [(((cz * p + az) % n1) * n1 + (cy * p + ay) % n1) * n1 + (cx * p + ax) % n1
                         for az in range(p + 1) for ay in range(p + 1) for ax in range(p + 1)]
                A[np.ix_(nodes, nodes)] += Ae
    ev = np.sort(np.linalg.eigvalsh(A))
    sym = []
    for j in np.ndindex(N, N, N):
        sym.extend(np.linalg.eigvalsh(qsfem3d.bloch_symbol_3d(p, kh, 2 * math.pi * np.array(j) / N)))
    assert np.allclose(ev, np.sort(sym), atol=1e-11)


def test_3d_fine_radius_p1_is_the_trilinear_closed_form():
    kh = 0.8
    d = qsfem3d.DIRS[1]
    r = qsfem3d.fine_radius_3d(1, kh, d)
    c = np.cos(r * d)
    s_ = (2 - 2 * c) * 1.0
    m = (2 + c) / 3
    sigma = s_[0] * m[1] * m[2] + m[0] * s_[1] * m[2] + m[0] * m[1] * s_[2] - kh ** 2 * m.prod()
    assert abs(sigma) < 1e-13


def test_3d_fine_radius_converges_to_k_with_order():
    kh = 2 * math.pi * 4 / 10
    d = qsfem3d.DIRS[2]
    errs = [abs(qsfem3d.fine_radius_3d(p, kh * p / 4, d) / (kh * p / 4) - 1) for p in (2, 4)]
    assert errs[1] < errs[0] * 1e-1


def test_3d_plain_fit_tracks_the_fine_dispersion_better_than_the_exact_k_stencil():
    eta, p = 0.9, 2
    kh = eta * p / 2
    qf = qsfem3d.plain_fit_3d(eta, p)
    qe = qsfem3d.q_weights(eta)
    rng = np.random.default_rng(4)
    dirs = np.abs(rng.standard_normal((12, 3)))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]

    def P_of(q):
        N = q[0]  # q0 = N P0 / 8 = N
        return 8.0, 4 * q[1] / N, 2 * q[2] / N, q[3] / N

    def mismatch(q):
        P = P_of(q)
        out = 0.0
        for d in dirs:
            zc = _radius(lambda r: qsfem3d.symbol(P, r * d), eta)
            zf = qsfem3d.fine_radius_3d(p, kh, d) * 2 / p
            out = max(out, abs(zc - zf) / eta)
        return out
    assert mismatch(qf) < mismatch(qe) / 5, (mismatch(qf), mismatch(qe))
