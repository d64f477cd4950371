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

Plain fit in 3-D (project definition, as the 2-D plain fit): the zeros are put
at the fine Q_p discrete wave vectors along the same three directions, found
from the p^3 x p^3 Bloch symbol of the fine element (Sec. 6.1 in three
dimensions) by a sign change of its eigenvalue nearest to zero and Brent's
method, as in the 2-D oracle.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.optimize import brentq

from .fem import eliminate, ref_matrices, side_mask

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


def coarse_matrix_3d(kc: np.ndarray, epsc=None, robin=None, q=None,
                     dirichlet=None) -> sp.csr_matrix:
    """Quasi-FE 27-point matrix on the coarse vertex grid (kc indexed [z][y][x]);
    vertices on the Dirichlet sides (6 booleans) are eliminated.

    The weights q are normalised so that the stencil symbol at 0 is -eta^2,
    the scale of a 2-D element matrix.  In 3-D the stiffness of a cell scales
    as h_c (h^{d-2}), so a cell contributes h_c q next to the h_c^3 mass of
    the -i eps term and the h_c^2 face mass of the absorbing term."""
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
                        E[a, b] = hc * qq[sum(int(va[i] != vb[i]) for i in range(3))]
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
    if dirichlet is not None and any(dirichlet):
        A = eliminate(A, side_mask(n1, 3, dirichlet))
    return A


def bloch_symbol_3d(p: int, kh: float, theta) -> np.ndarray:
    """A^(theta) on the unit cell of the 3-D Q_p space (h = 1): element matrix
    K M M + M K M + M M K - (kh)^2 M M M (kron order z, y, x), element node
    (az, ay, ax) -> cell dof (a mod p) with lattice shift (a // p)."""
    K1, M1 = ref_matrices(p)
    kr = lambda a, b, c: np.kron(a, np.kron(b, c))
    Ae = kr(K1, M1, M1) + kr(M1, K1, M1) + kr(M1, M1, K1) - kh * kh * kr(M1, M1, M1)
    n = p ** 3
    loc = [(az, ay, ax) for az in range(p + 1) for ay in range(p + 1) for ax in range(p + 1)]
    dof = np.array([((az % p) * p + ay % p) * p + ax % p for az, ay, ax in loc])
    shift = np.array([[ax // p, ay // p, az // p] for az, ay, ax in loc], dtype=float)
    ph = np.exp(1j * shift @ np.asarray(theta, dtype=float))
    S = np.zeros((n, n), dtype=complex)
    np.add.at(S, (dof[:, None], dof[None, :]), Ae * np.conj(ph)[:, None] * ph[None, :])
    return S


def _nearest_zero_eig_3d(p, kh, r, d):
    ev = np.linalg.eigvalsh(bloch_symbol_3d(p, kh, r * np.asarray(d)))
    return ev[np.argmin(np.abs(ev))]


def fine_radius_3d(p: int, kh: float, d, rel_window: float = 0.08, samples: int = 9) -> float:
    """Radius r (units of 1/h) of the fine discrete dispersion surface along d."""
    if not kh < math.pi:
        raise ValueError("only kh < pi is supported")
    rs = np.linspace(kh * (1 - rel_window), kh * (1 + rel_window), samples)
    vals = [_nearest_zero_eig_3d(p, kh, r, d) for r in rs]
    for i in range(samples - 1):
        if vals[i] == 0.0:
            return float(rs[i])
        if vals[i] * vals[i + 1] < 0:
            return brentq(lambda r: _nearest_zero_eig_3d(p, kh, r, d), rs[i], rs[i + 1],
                          xtol=1e-15, rtol=1e-15, maxiter=200)
    raise RuntimeError("no sign change of the symbol near r = kh")


def plain_fit_3d(eta_c: float, p: int, shift: float = 0.0):
    """(q0, q_face, q_edge, q_corner) matched to the fine dispersion of one
    coarse cell (eta_c = h_c k, h_c = 2h/p; shift = eps / k^2 as in 2-D)."""
    eta = float(((1.0 + 1j * shift) ** 0.5).real * eta_c)
    kh = eta * p / 2.0
    radii = [fine_radius_3d(p, kh, DIRS[m]) * 2.0 / p for m in range(3)]
    return q_weights(eta, radii)
