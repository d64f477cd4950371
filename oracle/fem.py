"""Continuous Galerkin Q_p discretisation on the regular square/cube mesh.

Follows Sec. 2 (eq. Helmholtz_eq and eq. bilin_form) and Sec. 3.1 of the
paper:  a(u,v; Omega, Gamma_abs) = int grad u . grad v - int (k^2 + i eps) u v
- int_{Gamma_abs} i k u v  (bilinear, not sesquilinear), discretised with
order-p continuous elements on cells of size h of the unit square/cube.

Reading (the paper uses NGSolve's hierarchical basis): a Lagrange basis on the
Gauss-Lobatto-Legendre points of every cell.  The space, the matrix up to a
change of basis and the Galerkin solution are the same; exact Gauss quadrature
is used since k and eps are constant per cell.

Node numbering: global lexicographic on the (pN+1)^d GLL grid, x fastest.
Cell numbering: x fastest.  Local node index in a cell: x fastest.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gll(p: int):
    """GLL nodes and weights on [0, 1]: the end points and the roots of P_p'."""
    if p == 1:
        t = np.array([-1.0, 1.0])
    else:
        d = np.polynomial.legendre.Legendre.basis(p).deriv()
        t = np.concatenate([[-1.0], np.sort(d.roots().real), [1.0]])
    pp = np.polynomial.legendre.Legendre.basis(p)(t)
    w = 2.0 / (p * (p + 1) * pp * pp)
    return (t + 1.0) / 2.0, w / 2.0


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values and derivatives of the Lagrange polynomials through `nodes`
    at points x: arrays of shape (len(x), len(nodes))."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    val = np.ones((len(x), n))
    der = np.zeros((len(x), n))
    for j in range(n):
        others = [m for m in range(n) if m != j]
        denom = np.prod([nodes[j] - nodes[m] for m in others])
        for m in others:
            val[:, j] *= (x - nodes[m])
        # product rule for the derivative
        for m in others:
            term = np.ones(len(x))
            for q in others:
                if q != m:
                    term *= (x - nodes[q])
            der[:, j] += term
        val[:, j] /= denom
        der[:, j] /= denom
    return val, der


def ref_matrices(p: int):
    """1-D reference stiffness K1[a,b] = int_0^1 phi_a' phi_b' and mass
    M1[a,b] = int_0^1 phi_a phi_b on the GLL Lagrange basis (exact Gauss)."""
    xq, wq = np.polynomial.legendre.leggauss(p + 2)
    xq = (xq + 1.0) / 2.0
    wq = wq / 2.0
    nodes, _ = gll(p)
    v, d = lagrange(nodes, xq)
    K1 = (d * wq[:, None]).T @ d
    M1 = (v * wq[:, None]).T @ v
    return K1, M1


def _kron_all(mats):
    out = np.ones((1, 1))
    for m in mats:  # slowest axis first
        out = np.kron(out, m)
    return out


def element_matrices(p: int, h: float, dim: int):
    """Cell stiffness and mass matrices on a cell of size h, local index x
    fastest: stiffness h^{d-2} sum_dirs (K1 in that direction, M1 elsewhere),
    mass h^d M1 x ... x M1."""
    K1, M1 = ref_matrices(p)
    S = np.zeros(((p + 1) ** dim,) * 2)
    for dd in range(dim):
        mats = [K1 if e == dd else M1 for e in range(dim)]
        S += _kron_all(mats)
    S *= h ** (dim - 2)
    M = _kron_all([M1] * dim) * h ** dim
    return S, M


def face_matrix(p: int, h: float, dim: int):
    """Mass matrix of a cell face (d-1 dimensional), h^{d-1} M1 x ... x M1."""
    _, M1 = ref_matrices(p)
    return _kron_all([M1] * (dim - 1)) * h ** (dim - 1)


def n_nodes_1d(n_cells: int, p: int) -> int:
    return n_cells * p + 1


def assemble_box(p: int, N: int, dim: int, box, kappa: np.ndarray,
                 robin_k: np.ndarray | None, robin_sides) -> sp.csr_matrix:
    """Galerkin matrix of  int grad.grad - int kappa u v - sum_sides int i k u v
    on the cell box `box` = ((c0, c1) per axis, axis 0 = x) of the global mesh
    with N cells per direction.

    kappa: complex per-cell coefficient on the global mesh, shape (N,)*dim
           indexed [z][y][x] (volume term coefficient, e.g. k^2 + i eps).
    robin_k: per-cell k (global mesh) used for the absorbing term on the box
           sides flagged in robin_sides, a tuple of 2*dim booleans
           (x-, x+, y-, y+, z-, z+).
    Local node numbering of the box, x fastest.
    """
    h = 1.0 / N
    S, M = element_matrices(p, h, dim)
    Fm = face_matrix(p, h, dim)
    ncb = [box[a][1] - box[a][0] for a in range(dim)]
    nb = [c * p + 1 for c in ncb]
    # local node offsets in one cell, x fastest
    loc = np.indices((p + 1,) * dim).reshape(dim, -1)[::-1]  # loc[axis] per local node
    # loc from np.indices is [slowest..fastest]; reversed -> loc[0] = x index
    strides = [int(np.prod(nb[:a])) for a in range(dim)]
    rows, cols, vals = [], [], []
    cell_ids = np.indices(ncb[::-1]).reshape(dim, -1)[::-1]  # cell_ids[axis], x fastest
    for ci in range(cell_ids.shape[1]):
        c = [int(cell_ids[a, ci]) for a in range(dim)]
        gidx = tuple(box[a][0] + c[a] for a in range(dim))[::-1]  # [z][y][x]
        nodes = sum((c[a] * p + loc[a]) * strides[a] for a in range(dim))
        Ae = S - kappa[gidx] * M
        for a in range(dim):
            for side in (0, 1):
                on_side = (c[a] == 0) if side == 0 else (c[a] == ncb[a] - 1)
                if on_side and robin_sides[2 * a + side]:
                    sel = loc[a] == (0 if side == 0 else p)
                    idx = np.nonzero(sel)[0]
                    Ae[np.ix_(idx, idx)] += -1j * robin_k[gidx] * Fm
        rows.append(np.repeat(nodes, len(nodes)))
        cols.append(np.tile(nodes, len(nodes)))
        vals.append(Ae.ravel())
    n = int(np.prod(nb))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def global_box(N: int, dim: int):
    return tuple((0, N) for _ in range(dim))


def helmholtz_matrix(p: int, k: np.ndarray, eps: np.ndarray | None = None,
                     robin=None, alpha: float = 0.0, dirichlet=None) -> sp.csr_matrix:
    """Global matrix A (alpha = 0) or the complex-shifted A_s (alpha = alpha_s,
    Sec. 4.1: volume coefficient k^2 + i alpha k^2 + i eps; the boundary term
    keeps -i k).  `dirichlet`: 2*dim booleans, sides whose nodes are
    eliminated (unit rows and columns)."""
    dim = k.ndim
    N = k.shape[0]
    if eps is None:
        eps = np.zeros_like(k)
    if robin is None:
        robin = (True,) * (2 * dim)
    kappa = k * k * (1.0 + 1j * alpha) + 1j * eps
    A = assemble_box(p, N, dim, global_box(N, dim), kappa, k, robin)
    if dirichlet is not None and any(dirichlet):
        A = eliminate(A, side_mask(N * p + 1, dim, dirichlet))
    return A


def node_coords_1d(N: int, p: int) -> np.ndarray:
    x, _ = gll(p)
    h = 1.0 / N
    out = np.empty(N * p + 1)
    for c in range(N):
        out[c * p: c * p + p + 1] = (c + x) * h
    return out


# Homogeneous Dirichlet sides (eq. Helmholtz_eq, the part Gamma_0 of the
# boundary).  Reading: the nodes of a closed Dirichlet side are not unknowns;
# vectors keep full length and the matrix takes unit rows and columns there,
# so with a zero right-hand side on those nodes the solution is the one of the
# system with the nodes removed.
def side_mask(n1: int, dim: int, sides) -> np.ndarray:
    """Boolean mask over the n1^dim grid (x fastest): nodes lying on a side
    flagged in `sides` (2*dim booleans, x-, x+, y-, y+, z-, z+)."""
    grid = np.indices((n1,) * dim)[::-1]  # grid[axis], axis 0 = x
    m = np.zeros((n1,) * dim, dtype=bool)
    for a in range(dim):
        if sides[2 * a]:
            m |= grid[a] == 0
        if sides[2 * a + 1]:
            m |= grid[a] == n1 - 1
    return m.ravel()


def eliminate(A: sp.spmatrix, mask: np.ndarray) -> sp.csr_matrix:
    """D A D + (I - D) with D the diagonal of the free (unmasked) nodes:
    masked rows and columns are replaced by those of the identity."""
    free = sp.diags((~mask).astype(float))
    return (free @ A @ free + sp.diags(mask.astype(float))).tocsr()
