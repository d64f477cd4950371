"""Prolongation I_P and restriction I_P^* between the coarse vertex grid and the
fine Q_p space.

Follows Sec. 4.2 of the paper: the coarse mesh is square with spacing 2h/p;
I_P u_c is, on every fine cell, the polynomial of degree p/2 (per direction)
that interpolates u_c at the coarse vertices lying in that cell; the
restriction of Alg. 1 is the adjoint I_P^* (the transpose, the form being
bilinear).

The paper builds I_P through NGSolve's hierarchical basis (vertex, then edge,
then cell coefficients).  That construction defines the same function; in the
GLL nodal basis used here the fine coefficients are simply the values of that
interpolant at the fine GLL nodes.  On a fine cell the interpolant is the
tensor product of 1-D interpolants, and a fine node on a cell edge receives the
same value from both cells (the 1-D interpolant on the shared edge only uses
the coarse vertices on that edge), so the global matrix is the Kronecker
product of the 1-D global matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import gll, lagrange, side_mask


def prolong_1d(N: int, p: int) -> sp.csr_matrix:
    """(pN+1) x (pN/2+1) matrix: fine GLL node values of the piecewise
    degree-p/2 interpolant of the coarse vertex values."""
    if p % 2:
        raise ValueError("p must be even")
    r = p // 2
    xf, _ = gll(p)
    xc = np.linspace(0.0, 1.0, r + 1)
    L, _ = lagrange(xc, xf)  # (p+1) x (r+1)
    nf, nc = N * p + 1, N * r + 1
    P = np.zeros((nf, nc))
    for c in range(N):
        P[c * p: c * p + p + 1, c * r: c * r + r + 1] = L
    P[np.abs(P) < 1e-15] = 0.0
    return sp.csr_matrix(P)


def prolongation(N: int, p: int, dim: int = 2, dirichlet=None) -> sp.csr_matrix:
    """Global I_P (fine nodes x coarse vertices), x fastest on both grids.

    With Dirichlet sides (2*dim booleans) the eliminated nodes leave both
    spaces.  Reading: the rows of fine nodes and the columns of coarse
    vertices on those sides are dropped (set to zero), so I_P maps the free
    coarse vertices to the free fine nodes."""
    P1 = prolong_1d(N, p)
    out = P1
    for _ in range(dim - 1):
        out = sp.kron(P1, out, format="csr")
    if dirichlet is not None and any(dirichlet):
        free_f = sp.diags((~side_mask(N * p + 1, dim, dirichlet)).astype(float))
        free_c = sp.diags((~side_mask(N * (p // 2) + 1, dim, dirichlet)).astype(float))
        out = free_f @ out @ free_c
    return out.tocsr()


def restriction(N: int, p: int, dim: int = 2, dirichlet=None) -> sp.csr_matrix:
    """I_P^* = I_P^T."""
    return prolongation(N, p, dim, dirichlet).T.tocsr()
