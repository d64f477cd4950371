"""Pins of the oracle's homogeneous Dirichlet sides (eq. Helmholtz_eq, the part
Gamma_0 of the boundary) on both levels and in the transfers (CPU).

The reading pinned here: the nodes of a closed Dirichlet side are eliminated
(unit rows and columns, zero right-hand side there), on the fine grid, on the
coarse vertex grid, inside every subdomain matrix, and from I_P.  The pins are
manufactured solutions (the discrete solutions converge to a smooth exact
solution at the rate of the discretisation), exact interpolation, exactness of
a single-subdomain smoother and invariants of the two-grid iteration.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import fem, qsfem, qsfem3d, smoother, transfer, twogrid


def _mass(p, N, dim):
    """Global consistent mass matrix: A(k = 0) - A(k = 1) without boundary terms."""
    z = np.zeros((N,) * dim)
    return (fem.helmholtz_matrix(p, z, robin=(False,) * (2 * dim))
            - fem.helmholtz_matrix(p, z + 1.0, robin=(False,) * (2 * dim)))


def _grid(coord, dim):
    g = np.meshgrid(*([coord] * dim), indexing="ij")[::-1]  # g[0] = x, x fastest
    return [a.ravel() for a in g]


def _manufactured_error(N, p, dim, k, sides, waves):
    """Max nodal error of the Galerkin solution of -Lap u - k^2 u = f with
    u = prod_a sin(w_a x_a), the Dirichlet sides flagged in `sides` and
    Neumann elsewhere; f is interpolated at the nodes and weighted with the
    consistent mass matrix."""
    A = fem.helmholtz_matrix(p, np.full((N,) * dim, float(k)), robin=(False,) * (2 * dim),
                             dirichlet=sides)
    X = _grid(fem.node_coords_1d(N, p), dim)
    u = np.prod([np.sin(w * x) for w, x in zip(waves, X)], axis=0)
    f = (sum(w * w for w in waves) - k * k) * u
    F = _mass(p, N, dim) @ f
    mask = fem.side_mask(N * p + 1, dim, sides)
    F[mask] = 0.0
    uh = spla.spsolve(A.tocsc(), F.astype(complex))
    assert np.all(uh[mask] == 0.0)
    return np.max(np.abs(uh - u))


@pytest.mark.parametrize("p", [2, 4])
def test_fine_dirichlet_all_sides_converges(p):
    """u = sin(pi x) sin(pi y) vanishes on all four sides."""
    Ns = [2, 4, 8]
    e = [_manufactured_error(N, p, 2, 3.0, (True,) * 4, (math.pi, math.pi)) for N in Ns]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert rates[-1] > p + 0.7, (e, rates)


def test_fine_dirichlet_neumann_mix_converges():
    """u = sin(pi x / 2) sin(pi y / 2): zero on x = 0 and y = 0, zero normal
    derivative on x = 1 and y = 1 (Dirichlet x-, y-; Neumann x+, y+).  Putting
    the Dirichlet sides on x+, y+ instead leaves an O(1) error."""
    w = (math.pi / 2, math.pi / 2)
    e = [_manufactured_error(N, 2, 2, 2.0, (True, False, True, False), w) for N in (4, 8)]
    assert math.log2(e[0] / e[1]) > 2.7, e
    assert _manufactured_error(8, 2, 2, 2.0, (False, True, False, True), w) > 0.1


def test_fine_dirichlet_3d_converges():
    e = [_manufactured_error(N, 2, 3, 2.0, (True,) * 6, (math.pi,) * 3) for N in (2, 4)]
    assert math.log2(e[0] / e[1]) > 2.7, e
    assert e[1] < 2e-3


def _coarse_error(Nc, dim, k, sides, waves):
    """Max vertex error of the quasi-FE QSFEM solution with Q1 mass weighting
    of the interpolated load."""
    kc = np.full((Nc,) * dim, float(k))
    if dim == 2:
        A = qsfem.coarse_matrix(kc, robin=(False,) * 4, dirichlet=sides)
    else:
        A = qsfem3d.coarse_matrix_3d(kc, robin=(False,) * 6, dirichlet=sides)
    X = _grid(np.linspace(0.0, 1.0, Nc + 1), dim)
    u = np.prod([np.sin(w * x) for w, x in zip(waves, X)], axis=0)
    f = (sum(w * w for w in waves) - k * k) * u
    F = _mass(1, Nc, dim) @ f
    mask = fem.side_mask(Nc + 1, dim, sides)
    F[mask] = 0.0
    uh = spla.spsolve(A.tocsc(), F.astype(complex))
    assert np.all(uh[mask] == 0.0)
    return np.max(np.abs(uh - u))


@pytest.mark.parametrize("dim,Ns", [(2, (8, 16, 32)), (3, (4, 8))])
def test_coarse_quasi_fe_dirichlet_converges_second_order(dim, Ns):
    sides = (True, False) * dim  # Dirichlet on the low sides, Neumann on the high ones
    w = (math.pi / 2,) * dim
    e = [_coarse_error(Nc, dim, 4.0, sides, w) for Nc in Ns]
    assert math.log2(e[-2] / e[-1]) > 1.6, e


@pytest.mark.parametrize("p", [2, 4])
def test_prolongation_with_dirichlet_sides_interpolates_vanishing_functions(p):
    """x y (degree 1 per direction) vanishes on x = 0 and y = 0: I_P of its
    coarse samples is exact; any coarse vector prolongs to zero on the
    Dirichlet nodes, and the restriction is the transpose."""
    N = 3
    sides = (True, False, True, False)
    P = transfer.prolongation(N, p, 2, sides)
    Xc = _grid(np.linspace(0.0, 1.0, N * (p // 2) + 1), 2)
    Xf = _grid(fem.node_coords_1d(N, p), 2)
    assert np.abs(P @ (Xc[0] * Xc[1]) - Xf[0] * Xf[1]).max() < 1e-14
    v = syn.random_complex(P.shape[1], seed=5)
    assert np.all(P @ v == 0.0, where=fem.side_mask(N * p + 1, 2, sides))
    R = transfer.restriction(N, p, 2, sides)
    assert abs(R - P.T).max() == 0.0
    # the coarse Dirichlet vertices receive nothing
    r = syn.random_complex(P.shape[0], seed=6)
    assert np.all((R @ r)[fem.side_mask(N * (p // 2) + 1, 2, sides)] == 0.0)


def test_single_subdomain_smoother_with_dirichlet_is_exact_solve():
    """One subdomain covering the mesh and alpha_s = 0: the smoother step is
    the exact solve of the eliminated system (the local elimination equals the
    global one)."""
    N, p = 4, 4
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.3, 1.0, 2.0, seed=2), 2.0)
    sides = (False, True, True, False)
    robin = tuple(not s for s in sides)
    sm = smoother.CSDDSmoother(p, k, None, 0.0, N, robin=robin, dirichlet=sides)
    A = fem.helmholtz_matrix(p, k, None, robin, 0.0, sides)
    f = syn.random_complex(A.shape[0], seed=1)
    u = sm.apply(np.zeros_like(f), f)
    ex = spla.spsolve(A.tocsc(), f)
    assert np.abs(u - ex).max() / np.abs(ex).max() < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_twogrid_with_dirichlet_keeps_eliminated_nodes_at_zero_and_converges(dim):
    """A right-hand side that vanishes on the Dirichlet nodes gives two-grid
    iterates that vanish there; the exact solution is a fixed point; GMRES
    reaches the sparse direct solution."""
    N, p = (6, 2) if dim == 2 else (4, 2)
    k = np.full((N,) * dim, 7.0)
    sides = (True, False, False, True) + ((True, False) if dim == 3 else ())
    robin = tuple(not s for s in sides)
    tg = twogrid.TwoGrid(p, k, alpha_s=0.5, l_dd=3 if dim == 2 else 2, robin=robin,
                         dirichlet=sides)
    mask = fem.side_mask(N * p + 1, dim, sides)
    f = syn.random_complex(tg.A.shape[0], seed=9)
    f[mask] = 0.0
    u = tg.twogrid_step(np.zeros_like(f), f)
    assert np.all(u[mask] == 0.0)
    ex = spla.spsolve(tg.A.tocsc(), f)
    assert np.abs(tg.twogrid_step(ex, f) - ex).max() / np.abs(ex).max() < 1e-11
    x, it, _ = tg.gmres(f, 1e-10)
    assert np.all(x[mask] == 0.0)
    assert np.abs(x - ex).max() / np.abs(ex).max() < 1e-8
    assert it < 25
