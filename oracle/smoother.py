"""Complex-shifted domain-decomposition smoother (CSDDSmoother, Alg. 2).

Follows Sec. 4.1 and Sec. 4.4 of the paper:
  * U^(i): non-overlapping blocks of l_dd cells per direction (some one cell
    smaller so they tile the mesh).  Reading: M = ceil(N / l_dd) blocks per
    direction with balanced sizes, the larger ones first.
  * Omega^(i): U^(i) plus one layer of neighbouring cells (edge or vertex
    neighbours), clipped to the domain; the overlap is two cells.
  * A_s^(i): the bilinear form on Omega^(i) with the shifted coefficient
    k^2 + i alpha_s k^2 + i eps, absorbing conditions on the internal
    boundary of Omega^(i) and the inherited conditions on the part of the
    boundary shared with Omega.  Reading: the absorbing term keeps -i k,
    with k of the adjacent cell; nodes on a Dirichlet side of Omega are
    eliminated from A_s^(i) as from A (unit rows and columns).
  * Averaged update, eq. RAS_like_update: every dof takes the mean of the
    local solutions of the closed U^(i) that contain it (L_j of them).
  * DDStep solves A_s^(i) w_i = -(R_i A_s - A_s^(i) R_i) v + R_i r, i.e.
    w_i = R_i v + (A_s^(i))^{-1} R_i (r - A_s v).

Subdomain solves are sparse LU factorisations (scipy splu) in FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import assemble_box, eliminate, helmholtz_matrix, side_mask


def block_sizes(N: int, l_dd: int):
    """Balanced partition of N cells in ceil(N / l_dd) blocks, larger first."""
    M = max(1, math.ceil(N / l_dd))
    base, rem = divmod(N, M)
    sizes = [base + 1] * rem + [base] * (M - rem)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    return [(int(starts[i]), int(starts[i + 1])) for i in range(M)]


@dataclass
class Subdomain:
    U: tuple            # cell box per axis (x first), half-open
    Om: tuple           # cell box of Omega^(i)
    om_nodes: np.ndarray   # global node ids of Omega^(i) (local order, x fastest)
    u_nodes: np.ndarray    # global node ids of closed U^(i)
    u_in_om: np.ndarray    # positions of the U nodes inside the Omega node list
    lu: object = field(default=None, repr=False)
    A_loc: sp.csr_matrix = field(default=None, repr=False)


def box_nodes(box, N: int, p: int) -> np.ndarray:
    """Global node ids of the closed cell box, local order x fastest."""
    dim = len(box)
    n1 = N * p + 1
    axes = [np.arange(box[a][0] * p, box[a][1] * p + 1) for a in range(dim)]
    ids = np.zeros(1, dtype=np.int64)
    for a in reversed(range(dim)):  # slowest first
        ids = (ids[:, None] * n1 + axes[a][None, :]).ravel()
    return ids


def decompose(N: int, p: int, dim: int, l_dd: int):
    parts = block_sizes(N, l_dd)
    subs = []
    for idx in np.ndindex(*([len(parts)] * dim)):
        ix = idx[::-1]  # x fastest over subdomains
        U = tuple(parts[ix[a]] for a in range(dim))
        Om = tuple((max(U[a][0] - 1, 0), min(U[a][1] + 1, N)) for a in range(dim))
        om_nodes = box_nodes(Om, N, p)
        u_nodes = box_nodes(U, N, p)
        pos = {int(g): i for i, g in enumerate(om_nodes)}
        u_in_om = np.array([pos[int(g)] for g in u_nodes], dtype=np.int64)
        subs.append(Subdomain(U, Om, om_nodes, u_nodes, u_in_om))
    return subs


def multiplicity(subs, n_nodes: int) -> np.ndarray:
    """L_j = number of closed U^(i) containing node j."""
    L = np.zeros(n_nodes)
    for s in subs:
        L[s.u_nodes] += 1.0
    return L


class CSDDSmoother:
    """Alg. 2 with exact (sparse LU) subdomain solves."""

    def __init__(self, p, k, eps, alpha_s, l_dd, robin=None, n_dd=1, A=None, A_s=None,
                 dirichlet=None):
        self.dim = k.ndim
        self.N = k.shape[0]
        self.p = p
        dim, N = self.dim, self.N
        if eps is None:
            eps = np.zeros_like(k)
        if robin is None:
            robin = (True,) * (2 * dim)
        self.n_dd = n_dd
        kappa_s = k * k * (1.0 + 1j * alpha_s) + 1j * eps
        self.subs = decompose(N, p, dim, l_dd)
        dmask = None
        if dirichlet is not None and any(dirichlet):
            dmask = side_mask(N * p + 1, dim, dirichlet)
        for s in self.subs:
            sides = []
            for a in range(dim):
                for side in (0, 1):
                    on_boundary = (s.Om[a][0] == 0) if side == 0 else (s.Om[a][1] == N)
                    sides.append(robin[2 * a + side] if on_boundary else True)
            s.A_loc = assemble_box(p, N, dim, s.Om, kappa_s, k, tuple(sides))
            if dmask is not None:
                s.A_loc = eliminate(s.A_loc, dmask[s.om_nodes])
            s.A_loc = s.A_loc.tocsc()
            s.lu = spla.splu(s.A_loc)
        self.n_nodes = (N * p + 1) ** dim
        self.L = multiplicity(self.subs, self.n_nodes)
        if A is None:
            A = helmholtz_matrix(p, k, eps, robin, 0.0, dirichlet)
        if A_s is None:
            A_s = helmholtz_matrix(p, k, eps, robin, alpha_s, dirichlet)
        self.A = A
        self.A_s = A_s

    def dd_step(self, v: np.ndarray, r: np.ndarray) -> np.ndarray:
        """One DDStep(v, r; A_s) with the averaged update."""
        rr = r - self.A_s @ v
        acc = np.zeros(self.n_nodes, dtype=np.complex128)
        for s in self.subs:
            w = v[s.om_nodes] + s.lu.solve(rr[s.om_nodes])
            acc[s.u_nodes] += w[s.u_in_om]
        return acc / self.L

    def apply(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        """u <- CSDDSmoother(u, f); returns the new u."""
        r = f - self.A @ u
        v = np.zeros_like(r)
        for _ in range(self.n_dd):
            v = self.dd_step(v, r)
        return u + v

    def subdomain_inverse_rows(self, i: int) -> np.ndarray:
        """Dense B_i = diag(1/L_j) R_U (A_s^(i))^{-1}  (n_U x n_Omega)."""
        s = self.subs[i]
        n = s.A_loc.shape[0]
        inv = s.lu.solve(np.eye(n, dtype=np.complex128))
        return inv[s.u_in_om, :] / self.L[s.u_nodes][:, None]
