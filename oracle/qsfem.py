"""QSFEM compact stencil and its quasi-finite-element coarse matrix.

Follows Sec. 3.2 (eq. P_QSFEM, eq. scaling_factor_QSFEM) and Sec. 3.3
(element-wise q_gamma and eq. element_wise_qsfem, boundary version) of the
paper.

Readings:
  * eta = h k(c) where h is the spacing of the mesh that carries the stencil,
    i.e. the coarse spacing 2h/p inside the two-grid method (Sec. 4.2).
  * The paper's formulas are evaluated exactly as printed, in FP64; for small
    eta the numerators and the denominator are O(eta^4), which loses digits
    (relative error about 1e-16 / eta^4).  The oracle keeps the printed
    formula; the pins in the tests use eta >= 0.3.
  * The coarse level carries no complex shift (the shift only enters A_s of
    the smoother, Sec. 4.1); the eps term is the Q1 mass (Sec. 3.3: nothing is
    done with the remaining mass matrix) and the absorbing term is the
    boundary Q1 mass with k of the adjacent coarse cell.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .fem import eliminate, side_mask


def cs(eta):
    eta = np.asarray(eta, dtype=np.float64)
    a1, a2 = math.pi / 16.0, 3.0 * math.pi / 16.0
    c1 = np.cos(eta * math.cos(a1))
    s1 = np.cos(eta * math.sin(a1))
    c2 = np.cos(eta * math.cos(a2))
    s2 = np.cos(eta * math.sin(a2))
    return c1, s1, c2, s2


def stencil_P(eta):
    """(P0, P1, P2) of eq. P_QSFEM."""
    c1, s1, c2, s2 = cs(eta)
    den = c2 * s2 * (c1 + s1) - c1 * s1 * (c2 + s2)
    P0 = np.full_like(np.asarray(eta, dtype=np.float64), 4.0)
    P1 = 2.0 * (c1 * s1 - c2 * s2) / den
    P2 = (c2 + s2 - c1 - s1) / den
    return P0, P1, P2


def symbol(P, h, xi1, xi2):
    """sigma_P(xi) of the 3x3 symmetric stencil, eq. symbol_sigma_P."""
    P0, P1, P2 = P
    a, b = np.cos(h * xi1), np.cos(h * xi2)
    return P0 + 2.0 * P1 * (a + b) + 4.0 * P2 * a * b


def scaling_N(eta):
    """N(eta) = -eta^2 / sigma_P(0), eq. scaling_factor_QSFEM."""
    P0, P1, P2 = stencil_P(eta)
    return -np.asarray(eta) ** 2 / (P0 + 4.0 * P1 + 4.0 * P2)


def q_weights(eta):
    """Per-cell (q_(0,0), q_edge, q_diag) = (N P0 / 4, N P1 / 2, N P2)."""
    P0, P1, P2 = stencil_P(eta)
    N = -np.asarray(eta) ** 2 / (P0 + 4.0 * P1 + 4.0 * P2)
    return N * P0 / 4.0, N * P1 / 2.0, N * P2


def cell_q_matrix(q0, qe, qd, dim: int = 2):
    """4x4 (2-D) element contribution: vertex pair (a, b) of one cell gets
    q_{b-a}: q0 on the diagonal, qe across an edge, qd across the face."""
    nv = 2 ** dim
    E = np.zeros((nv, nv))
    for a in range(nv):
        for b in range(nv):
            diff = bin(a ^ b).count("1")
            E[a, b] = (q0, qe, qd)[diff]
    return E


def coarse_matrix(kc: np.ndarray, epsc: np.ndarray | None = None, robin=None,
                  q: np.ndarray | None = None, dirichlet=None) -> sp.csr_matrix:
    """Quasi-FE QSFEM matrix on the coarse vertex grid (2-D).

    kc: per coarse cell k, shape (Nc, Nc) indexed [y][x]; coarse spacing
        hc = 1/Nc.  q (optional) overrides the per-cell weights, shape
        (Nc, Nc, 3) = (q0, qe, qd); by default the QSFEM weights at
        eta = hc k(c).
    (A_q)_{ab} = sum_{c in C(a,b)} q_{b-a}(hc k(c)) - int i eps phi_a phi_b
                 - int_{Gamma_abs} i k phi_a phi_b ds.
    Vertices on the Dirichlet sides (4 booleans, x-, x+, y-, y+) are
    eliminated (unit rows and columns), as on the fine level.
    """
    Nc = kc.shape[0]
    hc = 1.0 / Nc
    if epsc is None:
        epsc = np.zeros_like(kc)
    if robin is None:
        robin = (True,) * 4
    if q is None:
        q0, qe, qd = q_weights(hc * kc)
    else:
        q0, qe, qd = q[..., 0], q[..., 1], q[..., 2]
    m1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])
    Mq1 = np.kron(m1, m1) * hc * hc
    Fq1 = m1 * hc
    n1 = Nc + 1
    rows, cols, vals = [], [], []
    for cy in range(Nc):
        for cx in range(Nc):
            nodes = np.array([cy * n1 + cx, cy * n1 + cx + 1,
                              (cy + 1) * n1 + cx, (cy + 1) * n1 + cx + 1])
            E = cell_q_matrix(q0[cy, cx], qe[cy, cx], qd[cy, cx]).astype(np.complex128)
            E += -1j * epsc[cy, cx] * Mq1
            sides = [(cx == 0, [0, 2]), (cx == Nc - 1, [1, 3]),
                     (cy == 0, [0, 1]), (cy == Nc - 1, [2, 3])]
            for s, (on, idx) in enumerate(sides):
                if on and robin[s]:
                    E[np.ix_(idx, idx)] += -1j * kc[cy, cx] * Fq1
            rows.append(np.repeat(nodes, 4))
            cols.append(np.tile(nodes, 4))
            vals.append(E.ravel())
    n = n1 * n1
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    if dirichlet is not None and any(dirichlet):
        A = eliminate(A, side_mask(n1, 2, dirichlet))
    return A


def coarse_cell_values(field_fine: np.ndarray, p: int) -> np.ndarray:
    """Coarse cells (spacing 2h/p) nest in the fine cells for even p; every
    coarse cell takes the value of the fine cell containing it."""
    r = p // 2
    out = field_fine
    for ax in range(field_fine.ndim):
        out = np.repeat(out, r, axis=ax)
    return out
