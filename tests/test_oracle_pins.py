"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics
(printed stencils and values, closed forms, textbook special cases,
invariants, brute force on tiny meshes).  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import fem, lfa, qsfem, smoother, transfer, twogrid

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_blocks(name):
    out, cur = {}, None
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line[0].isalpha():
            cur = line
            out[cur] = []
        else:
            out[cur].append([float(Fraction(x)) for x in line.split()])
    return {k: np.array(v) for k, v in out.items()}


# ---------------------------------------------------------------- basis -----
def test_gll_nodes_and_weights_closed_forms():
    x, w = fem.gll(2)
    assert np.allclose(x, [0, 0.5, 1], atol=1e-15)
    assert np.allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    x, w = fem.gll(4)
    a = math.sqrt(3 / 7)
    assert np.allclose(x, [0, (1 - a) / 2, 0.5, (1 + a) / 2, 1], atol=1e-15)
    assert np.allclose(w, [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], atol=1e-15)


def test_reference_matrices_textbook():
    K1, M1 = fem.ref_matrices(1)
    assert np.allclose(K1, [[1, -1], [-1, 1]], atol=1e-15)
    assert np.allclose(M1, [[1 / 3, 1 / 6], [1 / 6, 1 / 3]], atol=1e-15)
    K2, M2 = fem.ref_matrices(2)  # quadratic element on [0,1], nodes 0, 1/2, 1
    assert np.allclose(K2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3, atol=1e-14)
    assert np.allclose(M2, np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30, atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_reference_matrices_invariants(p):
    K1, M1 = fem.ref_matrices(p)
    assert np.allclose(K1 @ np.ones(p + 1), 0, atol=1e-12)   # constants in the kernel
    assert abs(M1.sum() - 1.0) < 1e-13                       # integral of 1
    x, _ = fem.gll(p)
    assert abs(x @ M1 @ np.ones(p + 1) - 0.5) < 1e-13        # integral of x
    assert abs(x @ K1 @ x - 1.0) < 1e-12                     # integral of (x')^2


def test_q1_stencils_printed_in_the_paper():
    gold = read_blocks("q1_stencils.txt")
    N = 5
    h = 1.0 / N
    zero = np.zeros((N, N), complex)
    S = fem.assemble_box(1, N, 2, fem.global_box(N, 2), zero, None, (False,) * 4)
    SpM = fem.assemble_box(1, N, 2, fem.global_box(N, 2), zero - 1.0, None, (False,) * 4)
    n1 = N + 1
    c = 3 * n1 + 2   # an interior vertex
    def stencil(A):
        row = A.getrow(c).toarray().ravel()
        return np.array([[row[c + dy * n1 + dx] for dx in (-1, 0, 1)] for dy in (-1, 0, 1)])
    assert np.allclose(stencil(S).real, gold["stiffness"], atol=1e-14)
    assert np.allclose(stencil(SpM - S).real / h ** 2, gold["mass_over_h2"], atol=1e-14)


def _plane_wave_error(N, p, k, d):
    """Galerkin solution of the plane wave u = exp(i k d.x), which satisfies
    -Lap u - k^2 u = 0 and du/dn - i k u = g := i k (d.n - 1) u on the sides;
    returns the GLL-quadrature L2 error."""
    A = fem.helmholtz_matrix(p, np.full((N, N), float(k)))
    xg, wg = fem.gll(p)
    coord = fem.node_coords_1d(N, p)
    n1 = N * p + 1
    h = 1.0 / N
    F = np.zeros(n1 * n1, complex)
    # boundary load int_side g phi_j ds with (p+3)-point Gauss per edge
    xq, wq = np.polynomial.legendre.leggauss(p + 3)
    xq, wq = (xq + 1) / 2, wq / 2
    L, _ = fem.lagrange(xg, xq)
    for side, (nx_, ny_) in enumerate([(-1, 0), (1, 0), (0, -1), (0, 1)]):
        for c in range(N):
            t = (c + xq) * h
            if side < 2:
                X = np.full_like(t, 0.0 if side == 0 else 1.0); Y = t
            else:
                X = t; Y = np.full_like(t, 0.0 if side == 2 else 1.0)
            u = np.exp(1j * k * (d[0] * X + d[1] * Y))
            g = 1j * k * (d[0] * nx_ + d[1] * ny_ - 1.0) * u
            vals = (L * (wq * g * h)[:, None]).sum(axis=0)
            for a in range(p + 1):
                i = c * p + a
                if side == 0: node = i * n1
                elif side == 1: node = i * n1 + n1 - 1
                elif side == 2: node = i
                else: node = (n1 - 1) * n1 + i
                F[node] += vals[a]
    uh = spla.spsolve(A.tocsc(), F)
    X, Y = np.meshgrid(coord, coord)
    ue = np.exp(1j * k * (d[0] * X + d[1] * Y)).ravel()
    wsum = np.zeros(n1)
    for c in range(N):
        wsum[c * p: c * p + p + 1] += wg * h
    W = np.outer(wsum, wsum).ravel()
    return math.sqrt(np.sum(W * np.abs(uh - ue) ** 2))


@pytest.mark.parametrize("p", [2, 4])
def test_plane_wave_converges_at_order_p_plus_1(p):
    k, d = 6.0, (math.cos(0.3), math.sin(0.3))
    Ns = [4, 8, 16] if p == 2 else [2, 4, 8]
    errs = [_plane_wave_error(N, p, k, d) for N in Ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > p + 1 - 0.3, (errs, rates)


def test_dense_solve_matches_twogrid_gmres():
    N, p = 6, 2
    k = np.full((N, N), 9.0)
    tg = twogrid.TwoGrid(p, k, alpha_s=0.5, l_dd=3)
    f = syn.random_complex(tg.A.shape[0], seed=3)
    x, it, _ = tg.gmres(f, 1e-12)
    ex = np.linalg.solve(tg.A.toarray(), f)
    assert np.linalg.norm(x - ex) / np.linalg.norm(ex) < 1e-10


# ---------------------------------------------------------------- QSFEM -----
@pytest.mark.parametrize("eta", [0.3, 0.8, 1.2566, 2.0])
def test_qsfem_symbol_vanishes_at_the_matched_angles(eta):
    P = qsfem.stencil_P(eta)
    for t in (math.pi / 16, 3 * math.pi / 16, 5 * math.pi / 16, 7 * math.pi / 16,
              -math.pi / 16, math.pi / 2 + math.pi / 16):
        s = qsfem.symbol(P, 1.0, eta * math.cos(t), eta * math.sin(t))
        assert abs(s) < 1e-11, (eta, t, s)


@pytest.mark.parametrize("eta", [0.05, 0.2, 0.5])
def test_qsfem_scaled_symbol_is_consistent_with_helmholtz(eta):
    """h^-2 N(eta) sigma_P(xi) approximates |xi|^2 - k^2 for h|xi| small."""
    h, k = 1.0, eta
    P = qsfem.stencil_P(eta)
    N = qsfem.scaling_N(eta)
    assert abs(N * qsfem.symbol(P, h, 0, 0) + eta ** 2) < 1e-12
    for xi in [(0.3 * eta, 0.4 * eta), (eta, 0.0), (0.7 * eta, 0.7 * eta)]:
        approx = N * qsfem.symbol(P, h, *xi) / h ** 2
        exact = xi[0] ** 2 + xi[1] ** 2 - k ** 2
        assert abs(approx - exact) < 0.05 * k ** 2 * max(eta, 0.1) ** 2 + 1e-6 * k ** 2


def test_qsfem_quasi_fe_interior_stencil_is_N_times_P():
    Nc = 6
    eta = 1.1
    kc = np.full((Nc, Nc), eta * Nc)
    A = qsfem.coarse_matrix(kc)
    n1 = Nc + 1
    c = 3 * n1 + 3
    row = A.getrow(c).toarray().ravel()
    st = np.array([[row[c + dy * n1 + dx] for dx in (-1, 0, 1)] for dy in (-1, 0, 1)])
    P0, P1, P2 = qsfem.stencil_P(eta)
    Nn = qsfem.scaling_N(eta)
    expect = Nn * np.array([[P2, P1, P2], [P1, P0, P1], [P2, P1, P2]])
    assert np.allclose(st, expect, atol=1e-13)
    # boundary edge vertex: absorbing term -i k * (1-D Q1 mass row sum = h_c)
    b = 3  # on the y- side
    rowb = A.getrow(b).toarray().ravel()
    assert abs(rowb.imag.sum() + kc[0, 0] / Nc) < 1e-12
    assert np.allclose(A.toarray(), A.toarray().T)


# ------------------------------------------------------------- transfers ----
@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_prolongation_interpolates_and_reproduces_polynomials(p):
    N = 3
    r = p // 2
    IP = transfer.prolongation(N, p)
    xf = fem.node_coords_1d(N, p)
    xc = np.linspace(0, 1, N * r + 1)
    Xc, Yc = np.meshgrid(xc, xc)
    Xf, Yf = np.meshgrid(xf, xf)
    q = lambda X, Y: (X ** r - 0.3 * X + 0.2) * (Y ** r + 0.5 * Y ** (r - 1) - 1.0) + 1j * X * Y
    out = IP @ q(Xc, Yc).ravel()
    assert np.allclose(out, q(Xf, Yf).ravel(), atol=1e-12)
    # interpolation property: the fine function takes the coarse values at the
    # coarse vertices (evaluated through the fine cell's Lagrange basis)
    uc = syn.random_complex(IP.shape[1], seed=1)
    u = (IP @ uc).reshape(N * p + 1, N * p + 1)
    xg, _ = fem.gll(p)
    Lv, _ = fem.lagrange(xg, np.arange(r + 1) / r)   # (r+1) x (p+1)
    nc1 = N * r + 1
    ucg = uc.reshape(nc1, nc1)
    for cy in range(N):
        for cx in range(N):
            ue = u[cy * p: cy * p + p + 1, cx * p: cx * p + p + 1]
            vals = Lv @ ue @ Lv.T
            assert np.allclose(vals, ucg[cy * r: cy * r + r + 1, cx * r: cx * r + r + 1], atol=1e-12)


def test_p2_galerkin_coarse_operator_is_the_q1_matrix():
    """For p = 2 the coarse space Q1 on the same mesh is a subspace and I_P
    is the exact embedding, so I_P^T A_Q2 I_P = A_Q1 (Galerkin identity)."""
    N = 5
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.5, 3.0, seed=2), 1.3)
    A2 = fem.helmholtz_matrix(2, k)
    A1 = fem.helmholtz_matrix(1, k)
    IP = transfer.prolongation(N, 2)
    G = (IP.T @ A2 @ IP).toarray()
    assert np.allclose(G, A1.toarray(), atol=1e-12)


# -------------------------------------------------------------- smoother ----
def test_block_partition_reading():
    assert smoother.block_sizes(200, 16) == [(0, 16), (16, 32), (32, 48), (48, 64), (64, 80)] + \
        [(80 + 15 * i, 95 + 15 * i) for i in range(8)]
    assert smoother.block_sizes(64, 8) == [(8 * i, 8 * i + 8) for i in range(8)]


def test_single_subdomain_smoother_is_exact_shifted_solve():
    N, p = 5, 2
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.5, 3.0, seed=4), 1.5)
    sm = smoother.CSDDSmoother(p, k, None, 0.4, l_dd=N)
    u = syn.random_complex(sm.n_nodes, seed=5)
    f = syn.random_complex(sm.n_nodes, seed=6)
    As = fem.helmholtz_matrix(p, k, alpha=0.4).toarray()
    A = fem.helmholtz_matrix(p, k).toarray()
    ref = u + np.linalg.solve(As, f - A @ u)
    assert np.allclose(sm.apply(u, f), ref, atol=1e-11)
    sm0 = smoother.CSDDSmoother(p, k, None, 0.0, l_dd=N)
    assert np.allclose(sm0.apply(np.zeros_like(f), f), np.linalg.solve(A, f), atol=1e-10)


def test_subdomain_matrices_by_masked_global_assembly():
    """A_s^(i) equals the global-numbering assembly over the cells of
    Omega^(i) only, with absorbing terms on its internal sides, restricted to
    the Omega^(i) nodes (an independent route through the global numbering)."""
    N, p, l_dd, alpha = 7, 2, 3, 0.5
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.5, 3.0, seed=8), 1.2)
    sm = smoother.CSDDSmoother(p, k, None, alpha, l_dd)
    h = 1.0 / N
    Sref, Mref = fem.element_matrices(p, h, 2)
    Fm = fem.face_matrix(p, h, 2)
    n1 = N * p + 1
    for s in sm.subs:
        G = np.zeros((n1 * n1, n1 * n1), complex)
        (x0, x1), (y0, y1) = s.Om
        for cy in range(y0, y1):
            for cx in range(x0, x1):
                nodes = np.array([(cy * p + ay) * n1 + cx * p + ax
                                  for ay in range(p + 1) for ax in range(p + 1)])
                G[np.ix_(nodes, nodes)] += Sref - k[cy, cx] ** 2 * (1 + 1j * alpha) * Mref
                edges = [(cx == x0, [a * (p + 1) for a in range(p + 1)]),
                         (cx == x1 - 1, [a * (p + 1) + p for a in range(p + 1)]),
                         (cy == y0, list(range(p + 1))),
                         (cy == y1 - 1, [p * (p + 1) + a for a in range(p + 1)])]
                for on, loc in edges:
                    if on:  # every side of Omega^(i) is absorbing here (all-Robin problem)
                        idx = nodes[loc]
                        G[np.ix_(idx, idx)] += -1j * k[cy, cx] * Fm
        sub = G[np.ix_(s.om_nodes, s.om_nodes)]
        assert np.allclose(sub, s.A_loc.toarray(), atol=1e-12)


def test_averaging_weights_partition_unity():
    N, p = 11, 2
    subs = smoother.decompose(N, p, 2, 4)
    L = smoother.multiplicity(subs, (N * p + 1) ** 2)
    tot = np.zeros_like(L)
    for s in subs:
        tot[s.u_nodes] += 1.0 / L[s.u_nodes]
    assert np.allclose(tot, 1.0)
    assert set(np.unique(L)) == {1.0, 2.0, 4.0}


# --------------------------------------------------------- two-grid / GMRES --
def test_twogrid_fixed_point():
    N, p = 6, 4
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.5, 3.0, seed=9), 2.0)
    tg = twogrid.TwoGrid(p, k, alpha_s=0.5, l_dd=3)
    f = syn.random_complex(tg.A.shape[0], seed=10)
    x = spla.spsolve(tg.A.tocsc(), f)
    assert np.linalg.norm(tg.twogrid_step(x, f) - x) / np.linalg.norm(x) < 1e-11


def test_gmres_matches_krylov_least_squares():
    rng = np.random.default_rng(0)
    n, m = 30, 6
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 6 * np.eye(n)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, _ = twogrid.gmres_right(lambda v: A @ v, lambda v: v, f, rtol=1e-300, maxit=m)
    Kr = np.stack([np.linalg.matrix_power(A, j) @ f for j in range(m)], axis=1)
    y, *_ = np.linalg.lstsq(A @ Kr, f, rcond=None)
    assert np.linalg.norm(x - Kr @ y) / np.linalg.norm(x) < 1e-9


def test_gmres_converged_iterate_meets_rtol_on_the_true_residual():
    """With short restarts and a preconditioner that varies from call to call
    (rounded to single precision, as the complex64 two-grid step is), the
    returned iterate meets rtol on f - A x itself."""
    rng = np.random.default_rng(3)
    n = 60
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    Minv = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)))
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    prec = lambda v: (Minv.astype(np.complex64) @ v.astype(np.complex64)).astype(np.complex128)
    for restart in (2, 3, None):
        for rtol in (1e-6, 1e-10):
            x, it, _ = twogrid.gmres_right(lambda v: A @ v, prec, f, rtol=rtol, maxit=400,
                                           restart=restart)
            assert it < 400
            assert np.linalg.norm(f - A @ x) <= rtol * np.linalg.norm(f)


def test_givens_zeroes_second_component():
    for a, b in [(1 + 2j, 3 - 1j), (0.0, 2j), (1.5, 0.0)]:
        c, s, r = twogrid.givens(a, b)
        assert abs(-np.conj(s) * a + np.conj(c) * b) < 1e-14
        assert abs(c * a + s * b - r) < 1e-14


# ---------------------------------------------------------------- toy LFA ----
def test_toy_c_values_printed_in_the_paper():
    rows = [l.split() for l in open(os.path.join(GOLD, "lfa_toy_c.txt")) if l[0] != "#"]
    for ppw, c in rows:
        kh = 2 * math.pi / float(ppw)
        assert round(float(lfa.toy_c(kh)), 2) == float(c)


@pytest.mark.parametrize("c,R", [(0.73, 0.5), (0.9, 3.0), (0.4, 10.0), (1.0, 2.0)])
def test_lemma_closed_form_by_brute_force(c, R):
    zc, et = 0.4, 0.01
    zf = zc + R * et
    th = zc + et * np.tan(np.linspace(-math.pi / 2 + 1e-7, math.pi / 2 - 1e-7, 400001))
    brute = np.max(np.abs(lfa.lemma_f(th, c, zf, zc, et)))
    assert abs(brute - lfa.lemma_max(c, R)) < 1e-6 * lfa.lemma_max(c, R)


def test_toy_rho_near_R_for_second_order_fd():
    """Sec. 5.4: rho is close to R = 2 pi |delta| / D (second-order FD, D = 0.01,
    alpha_s = 0.2)."""
    D, alpha, k = 0.01, 0.2, 1.0
    for ppw in (10, 14):
        h = 2 * math.pi / (ppw * k)
        # zeta_f, zeta_c: roots of the real symbols on the two grids
        zf = 2 * math.asin(k * h / 2)
        zc = math.asin(k * h) if k * h <= 1 else None
        R = 2 * math.pi * abs((zc - zf) / (k * h)) / D
        rho = lfa.toy_rho(k, h, D, alpha, n_theta=20001)
        assert 0.5 * R < rho < 1.5 * R + 0.5, (ppw, rho, R)
