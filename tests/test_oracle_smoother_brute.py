"""Brute-force pins of the oracle's multi-subdomain smoother and of the coarse
mass terms.  CPU only.

The CSDD smoother (Alg. 2, eq. RAS_like_update) is rebuilt here with explicit
dense matrices that share nothing with `oracle.smoother` beyond the pinned
element matrices of `oracle.fem`: the node sets of U^(i) and Omega^(i) come
from coordinates, every restriction R is a dense 0/1 matrix, A, A_s and every
A_s^(i) are assembled cell by cell in the global numbering, L_j is the column
sum of the R_U's, and the DDStep takes the paper's form
    A_s^(i) w_i = -(R_i A_s - A_s^(i) R_i) v + R_i r
(not the oracle's rewritten form) with a dense inverse.  The whole smoother is
then compared as a matrix: column j of the oracle's map f -> S(0, f) against
the brute-force matrix, and the affine map u -> S(u, f) on random data.

The coarse pins check the -i eps mass and the absorbing boundary mass of the
quasi-FE coarse matrix (Sec. 3.3: the remaining mass matrix is kept as an FE
mass) against the p = 1 Galerkin assembly, whose stencils are pinned to the
printed Q1 stencils.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import fem, qsfem, qsfem3d, smoother


# ------------------------------------------------ dense brute-force smoother --
def _cells(box):
    """Cell multi-indices (x first) of a cell box, any order."""
    rng = [range(b0, b1) for (b0, b1) in box]
    return [c[::-1] for c in np.ndindex(*[len(r) for r in rng[::-1]])], [r.start for r in rng]


def _node_id(idx, n1):
    g = 0
    for a in reversed(range(len(idx))):
        g = g * n1 + idx[a]
    return g


def _dense_galerkin(p, N, dim, box, kappa, k, absorbing):
    """Dense n x n (global numbering) matrix of the bilinear form restricted to
    the cells of `box`: stiffness - kappa mass per cell, and -i k(cell) times
    the face mass on every side of the box for which absorbing(axis, side) is
    true.  kappa, k indexed [z][y][x]."""
    n1 = N * p + 1
    h = 1.0 / N
    S, M = fem.element_matrices(p, h, dim)
    F = fem.face_matrix(p, h, dim)
    G = np.zeros((n1 ** dim, n1 ** dim), complex)
    local = [loc[::-1] for loc in np.ndindex(*([p + 1] * dim))]   # x first
    rel, start = _cells(box)
    for c in rel:
        cell = tuple(start[a] + c[a] for a in range(dim))
        nodes = np.array([_node_id([cell[a] * p + lo[a] for a in range(dim)], n1) for lo in local])
        G[np.ix_(nodes, nodes)] += S - kappa[cell[::-1]] * M
        for a in range(dim):
            for side in (0, 1):
                edge = box[a][0] if side == 0 else box[a][1] - 1
                if cell[a] == edge and absorbing(a, side):
                    sel = [i for i, lo in enumerate(local) if lo[a] == (0 if side == 0 else p)]
                    idx = nodes[sel]
                    G[np.ix_(idx, idx)] += -1j * k[cell[::-1]] * F
    return G


def _nodes_of_box(box, N, p):
    n1 = N * p + 1
    dim = len(box)
    out = []
    for idx in np.ndindex(*([n1] * dim)):
        x = idx[::-1]
        if all(box[a][0] * p <= x[a] <= box[a][1] * p for a in range(dim)):
            out.append(_node_id(x, n1))
    return np.array(sorted(out))


def _dirichlet_nodes(N, p, dim, dirichlet):
    n1 = N * p + 1
    out = set()
    for idx in np.ndindex(*([n1] * dim)):
        x = idx[::-1]
        for a in range(dim):
            if (dirichlet[2 * a] and x[a] == 0) or (dirichlet[2 * a + 1] and x[a] == n1 - 1):
                out.add(_node_id(x, n1))
    return np.array(sorted(out), dtype=np.int64)


def _unit_rows(G, nodes):
    """Replace the rows and columns of `nodes` by those of the identity."""
    G = G.copy()
    G[nodes, :] = 0.0
    G[:, nodes] = 0.0
    G[nodes, nodes] = 1.0
    return G


def brute_force_smoother(p, k, eps, alpha_s, l_dd, n_dd, robin, dirichlet=None):
    """Returns (A, S_of) where S_of(u, f) is Alg. 2 on dense matrices."""
    dim = k.ndim
    N = k.shape[0]
    n = (N * p + 1) ** dim
    kappa = k * k + 1j * eps
    kappa_s = k * k * (1 + 1j * alpha_s) + 1j * eps
    whole = tuple((0, N) for _ in range(dim))
    outer = lambda a, side: robin[2 * a + side]
    A = _dense_galerkin(p, N, dim, whole, kappa, k, outer)
    As = _dense_galerkin(p, N, dim, whole, kappa_s, k, outer)
    dn = _dirichlet_nodes(N, p, dim, dirichlet) if dirichlet else np.zeros(0, np.int64)
    if len(dn):
        A, As = _unit_rows(A, dn), _unit_rows(As, dn)
    # blocks: ceil(N / l_dd) per direction, sizes differing by at most one, larger first
    m = -(-N // l_dd)
    sizes = [N // m + (1 if b < N % m else 0) for b in range(m)]
    edges = np.concatenate([[0], np.cumsum(sizes)])
    subs = []
    for bidx in np.ndindex(*([m] * dim)):
        U = tuple((int(edges[b]), int(edges[b + 1])) for b in bidx[::-1])
        Om = tuple((max(u0 - 1, 0), min(u1 + 1, N)) for (u0, u1) in U)
        # inner sides of Omega^(i) absorbing; sides on the boundary inherit its condition
        absorbing = (lambda Om: lambda a, side: robin[2 * a + side]
                     if Om[a][side] == (0 if side == 0 else N) else True)(Om)
        om = _nodes_of_box(Om, N, p)
        un = _nodes_of_box(U, N, p)
        G = _dense_galerkin(p, N, dim, Om, kappa_s, k, absorbing)[np.ix_(om, om)]
        if len(dn):
            G = _unit_rows(G, np.nonzero(np.isin(om, dn))[0])
        R_om = np.zeros((len(om), n))
        R_om[np.arange(len(om)), om] = 1.0
        R_u = np.zeros((len(un), n))
        R_u[np.arange(len(un)), un] = 1.0
        subs.append((R_om, R_u, G, np.linalg.inv(G)))
    L = sum(R_u.T @ np.ones(R_u.shape[0]) for (_, R_u, _, _) in subs)
    assert L.min() >= 1.0

    def S_of(u, f):
        r = f - A @ u
        v = np.zeros(n, complex)
        for _ in range(n_dd):
            acc = np.zeros(n, complex)
            for R_om, R_u, G, Ginv in subs:
                w = Ginv @ (-(R_om @ As - G @ R_om) @ v + R_om @ r)
                acc += R_u.T @ (R_u @ R_om.T @ w)
            v = acc / L
        return u + v

    return A, S_of


CASES = [
    # (dim, N, p, l_dd, n_dd, robin sides, dirichlet sides)
    (2, 5, 2, 2, 1, (True,) * 4, None),                               # 3 x 3 blocks 2, 2, 1
    (2, 5, 2, 2, 2, (True,) * 4, None),
    (2, 6, 2, 3, 2, (True, False, False, True), (False, False, True, False)),  # Dirichlet y-, Neumann x+
    (2, 4, 4, 2, 2, (True,) * 4, None),                               # p = 4
    (3, 3, 2, 2, 2, (True,) * 6, None),                               # 3-D, 2 x 2 x 2 blocks 2, 1
]


@pytest.mark.parametrize("dim,N,p,l_dd,n_dd,robin,dirichlet", CASES)
def test_multi_subdomain_smoother_equals_dense_brute_force(dim, N, p, l_dd, n_dd, robin, dirichlet):
    alpha_s = 0.4
    c = syn.grf_speed(N, dim, 0.3, 1.5, 3.0, seed=11)
    k = syn.wavenumber_from_speed(c, 1.4)
    eps = 0.3 * k * k * syn.grf_speed(N, dim, 0.3, 0.0, 1.0, seed=12)   # a damped medium
    A, S_of = brute_force_smoother(p, k, eps, alpha_s, l_dd, n_dd, robin, dirichlet)
    sm = smoother.CSDDSmoother(p, k, eps, alpha_s, l_dd, robin=robin, n_dd=n_dd,
                               dirichlet=dirichlet)
    assert len(sm.subs) >= 4
    n = A.shape[0]
    # the linear part f -> S(0, f) as a matrix, column by column
    M_or = np.empty((n, n), complex)
    M_bf = np.empty((n, n), complex)
    zero = np.zeros(n, complex)
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1.0
        M_or[:, j] = sm.apply(zero, e)
        M_bf[:, j] = S_of(zero, e)
    scale = np.abs(M_bf).max()
    assert np.abs(M_or - M_bf).max() <= 1e-12 * scale
    # the affine map with a nonzero u (exercises r = f - A u)
    u = syn.random_complex(n, seed=13)
    f = syn.random_complex(n, seed=14)
    if dirichlet:
        f[_dirichlet_nodes(N, p, dim, dirichlet)] = 0.0
    ref = S_of(u, f)
    assert np.linalg.norm(sm.apply(u, f) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_brute_force_smoother_two_steps_differ_from_one():
    """Guard on the pin itself: with n_dd = 2 the correction through A_s v is
    active, so the second step changes the result (an A in place of A_s, or a
    dropped 1/L, cannot hide behind a vanishing v)."""
    N, p = 5, 2
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.5, 3.0, seed=11), 1.4)
    eps = np.zeros_like(k)
    _, S1 = brute_force_smoother(p, k, eps, 0.4, 2, 1, (True,) * 4)
    _, S2 = brute_force_smoother(p, k, eps, 0.4, 2, 2, (True,) * 4)
    f = syn.random_complex((N * p + 1) ** 2, seed=3)
    z = np.zeros_like(f)
    assert np.linalg.norm(S2(z, f) - S1(z, f)) > 1e-3 * np.linalg.norm(S1(z, f))


# ------------------------------------------------------- coarse mass terms --
def _q1_terms(Nc, dim, kc, epsc, absorbing_sides):
    """-i eps mass and -i k boundary mass of the Q1 Galerkin assembly
    (p = 1, cells of size 1/Nc), isolated by subtracting the stiffness."""
    box = fem.global_box(Nc, dim)
    zero = np.zeros_like(kc, dtype=complex)
    stiff = fem.assemble_box(1, Nc, dim, box, zero, kc, (False,) * (2 * dim))
    mass = fem.assemble_box(1, Nc, dim, box, 1j * epsc, kc, (False,) * (2 * dim)) - stiff
    bnd = fem.assemble_box(1, Nc, dim, box, zero, kc, absorbing_sides) - stiff
    return mass.toarray(), bnd.toarray()


@pytest.mark.parametrize("dim", [2, 3])
def test_coarse_eps_and_absorbing_terms_are_q1_masses(dim):
    Nc = 5 if dim == 2 else 3
    kc = syn.wavenumber_from_speed(syn.grf_speed(Nc, dim, 0.4, 1.5, 3.0, seed=21), 1.1)
    epsc = syn.grf_speed(Nc, dim, 0.4, 0.1, 2.0, seed=22) * kc * kc
    sides = (True, False, True, True, False, True)[: 2 * dim]
    mass, bnd = _q1_terms(Nc, dim, kc, epsc, sides)
    q = np.zeros(kc.shape + ((3,) if dim == 2 else (4,)))
    build = qsfem.coarse_matrix if dim == 2 else qsfem3d.coarse_matrix_3d
    A_eps = build(kc, epsc, (False,) * (2 * dim), q=q).toarray()
    A_bnd = build(kc, None, sides, q=q).toarray()
    scale = np.abs(mass).max()
    assert scale > 0 and np.abs(A_eps - mass).max() <= 1e-14 * max(1.0, scale)
    assert np.abs(A_bnd - bnd).max() <= 1e-13 * np.abs(bnd).max()
    # all three parts together: weights + mass + boundary add up
    A_all = build(kc, epsc, sides).toarray()
    A_q = build(kc, None, (False,) * (2 * dim)).toarray()
    assert np.abs(A_all - (A_q + mass + bnd)).max() <= 1e-12 * np.abs(A_all).max()
