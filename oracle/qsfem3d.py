"""Compact 27-point coarse stencil for 3-D (project definition).

The paper works in 2-D and refers the 3-D dispersion-minimising scheme to a
separate reference that is not part of it.  This build uses the natural 3-D
analogue of the 2-D QSFEM construction (Sec. 3.2): the symmetric 27-point
family with classes center P0, face neighbours P1, edge neighbours P2,
corner neighbours P3, symbol
    sigma(xi) = P0 + 2 P1 (c1 + c2 + c3) + 4 P2 (c1 c2 + c1 c3 + c2 c3) + 8 P3 c1 c2 c3,
c_i = cos(h xi_i), with P0 = 8 and (P1, P2, P3) chosen so that sigma vanishes
at |xi| = k along three fixed directions of the symmetry sector
(normalised (1, 0.2, 0.1), (1, 0.6, 0.3), (1, 0.9, 0.7)), scaled by
N = -eta^2 / sigma(0) (as eq. scaling_factor_QSFEM).  The quasi-FE element
distribution follows Sec. 3.3: a vertex pair of one coarse cell gets N P0 / 8
(same vertex), N P1 / 4 (edge), N P2 / 2 (face diagonal), N P3 (body
diagonal).  Parity of this stencil is unpinned beyond its defining zeros, the
consistency limit and the assembly invariants.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRS = np.array([[1.0, 0.2, 0.1], [1.0, 0.6, 0.3], [1.0, 0.9, 0.7]])
DIRS = DIRS / np.linalg.norm(DIRS, axis=1)[:, None]


def stencil_P(eta: float, radii=None):
    """(P0, P1, P2, P3) with zeros at radius radii[m] (default eta) along DIRS."""
    radii = [eta] * 3 if radii is None else radii
    M = np.zeros((3, 3))
    rhs = np.full(3, -8.0)
    for m in range(3):
        c = np.cos(radii[m] * DIRS[m])
        M[m] = [2 * c.sum(), 4 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2]), 8 * c.prod()]
    P1, P2, P3 = np.linalg.solve(M, rhs)
    return 8.0, P1, P2, P3


def symbol(P, xi):
    c = np.cos(np.asarray(xi, dtype=float))
    P0, P1, P2, P3 = P
    return (P0 + 2 * P1 * c.sum() + 4 * P2 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2])
            + 8 * P3 * c.prod())


def q_weights(eta: float, radii=None):
    P = stencil_P(eta, radii)
    N = -eta * eta / (P[0] + 6 * P[1] + 12 * P[2] + 8 * P[3])
    return N * P[0] / 8.0, N * P[1] / 4.0, N * P[2] / 2.0, N * P[3]


def coarse_matrix_3d(kc: np.ndarray, epsc=None, robin=None, q=None) -> sp.csr_matrix:
    """Quasi-FE 27-point matrix on the coarse vertex grid (kc indexed [z][y][x])."""
    Nc = kc.shape[0]
    hc = 1.0 / Nc
    if epsc is None:
        epsc = np.zeros_like(kc)
    if robin is None:
        robin = (True,) * 6
    m1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    Mq = np.kron(m1, np.kron(m1, m1)) * hc ** 3
    Fq = np.kron(m1, m1) * hc ** 2
    n1 = Nc + 1
    rows, cols, vals = [], [], []
    for cz in range(Nc):
        for cy in range(Nc):
            for cx in range(Nc):
                qq = q_weights(hc * kc[cz, cy, cx]) if q is None else q[cz, cy, cx]
                verts = [(az, ay, ax) for az in (0, 1) for ay in (0, 1) for ax in (0, 1)]
                nodes = np.array([((cz + az) * n1 + cy + ay) * n1 + cx + ax for az, ay, ax in verts])
                E = np.zeros((8, 8), dtype=complex)
                for a, va in enumerate(verts):
                    for b, vb in enumerate(verts):
                        E[a, b] = qq[sum(int(va[i] != vb[i]) for i in range(3))]
                E += -1j * epsc[cz, cy, cx] * Mq
                sides = [(cx == 0, 2, 0), (cx == Nc - 1, 2, 1), (cy == 0, 1, 0),
                         (cy == Nc - 1, 1, 1), (cz == 0, 0, 0), (cz == Nc - 1, 0, 1)]
                for s, (on, axis, val) in enumerate(sides):
                    if on and robin[s]:
                        idx = [i for i, v in enumerate(verts) if v[axis] == val]
                        E[np.ix_(idx, idx)] += -1j * kc[cz, cy, cx] * Fq
                rows.append(np.repeat(nodes, 8))
                cols.append(np.tile(nodes, 8))
                vals.append(E.ravel())
    n = n1 ** 3
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A
