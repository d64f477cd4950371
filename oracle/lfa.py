"""Local Fourier analysis of the two-grid method.

Part 1 -- toy 1-D problem (Sec. 5): -u'' - (k^2 + i eps) u = f on R with
eps = k^2 D / pi (eq. epsilon_ksquare_D), second-order central differences
on both grids, linear interpolation, full weighting, exact smoother
A_s^{-1} with A_s = A - i alpha_s k^2 I.  Symbols on the 2-dimensional spaces
E_{f,theta} = span(e^{i theta x/h}, e^{i (theta+pi) x/h}).

Readings:
  * The factor c of Sec. 5.4 is printed as (1/2)(1 + cos kh)^2 but the printed
    values (0.56 / 0.73 / 0.87 at 6 / 8 / 12 points per wavelength) and the
    symbol K_11 = 1 - (1/4)(1 + cos theta)^2 A_c^{-1} A above it both give
    c = (1/4)(1 + cos kh)^2; that is used.
  * M = S^{nu2} K S^{nu1} (the exponent in the printed 2x2 product is
    misplaced); the coarse symbol in K is evaluated at the same theta.

Part 2 -- Bloch-wave LFA of the finite-element method (Sec. 6.1) lives in
`bloch_symbols` / `twogrid_symbol` below.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# toy problem


def toy_c(kh):
    """c = (1/4) (1 + cos kh)^2 (prolongation/restriction factor at theta = kh)."""
    return 0.25 * (1.0 + np.cos(kh)) ** 2


def lemma_max(c, R):
    """Closed form of max_theta |1 - c (theta - zf - i e)/(theta - zc - i e)|
    (Lemma of Sec. 5.5) with R = |zf - zc| / e."""
    return math.sqrt((1.0 - c) ** 2 + (c * R / 2.0) ** 2) + c * R / 2.0


def lemma_f(theta, c, zf, zc, et):
    return 1.0 - c * (theta - zf - 1j * et) / (theta - zc - 1j * et)


def toy_symbols(theta, k, h, D, alpha_s, M=1):
    """Return (A_f 2x2, A_s 2x2, A_c scalar, I_P 2x1, I_R 1x2) at theta.

    D_{2,M}: central difference of width 2M+1 (M = 1: second order, M = 2:
    fourth order) on the fine grid (spacing h) and on the coarse grid (2h)."""
    eps = k * k * D / math.pi
    kap = k * k + 1j * eps

    def d2(t, hh):
        if M == 1:
            return (2.0 - 2.0 * np.cos(t)) / hh ** 2
        if M == 2:  # -(-1/12, 4/3, -5/2, 4/3, -1/12)
            return (5.0 / 2.0 - (8.0 / 3.0) * np.cos(t) + (1.0 / 6.0) * np.cos(2 * t)) / hh ** 2
        raise ValueError(M)

    a1 = d2(theta, h) - kap
    a2 = d2(theta + math.pi, h) - kap
    Af = np.diag([a1, a2])
    As = Af - 1j * alpha_s * k * k * np.eye(2)
    Ac = d2(2.0 * theta, 2.0 * h) - kap
    cth = np.cos(theta)
    IP = np.array([[0.5 + 0.5 * cth], [0.5 - 0.5 * cth]], dtype=complex)
    IR = IP.T.copy()
    return Af, As, Ac, IP, IR


def toy_two_grid_symbol(theta, k, h, D, alpha_s, nu1=1, nu2=1, omega_c=1.0, M=1):
    Af, As, Ac, IP, IR = toy_symbols(theta, k, h, D, alpha_s, M)
    S = np.eye(2) - np.linalg.solve(As, Af)
    K = np.eye(2) - omega_c * IP @ (IR @ Af) / Ac
    return np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)


def toy_rho(k, h, D, alpha_s, n_theta=4001, **kw):
    th = np.linspace(-math.pi / 2, math.pi / 2, n_theta, endpoint=False)
    return max(np.max(np.abs(np.linalg.eigvals(toy_two_grid_symbol(t, k, h, D, alpha_s, **kw))))
               for t in th)


# ---------------------------------------------------------------------------
# Bloch-wave LFA of the finite-element two-grid method (Sec. 6.1)
#
# Operators on the N x N periodic mesh (constant k, eps = D k^2 / pi): fine A,
# shifted A_s (exact smoother S = I - A_s^{-1} A), coarse QSFEM quasi-FE A_c on
# the periodic coarse mesh of spacing 2h/p, interpolation I_P and restriction
# I_P^T.  Their symbols use eq. symbol_sum, sigma(P)(theta) = sum_beta
# e^{i theta . beta} P_{0,beta}, with the unit cell of p^2 fine and (p/2)^2
# coarse dofs; S^ = I - A_s^-1 A^, K^ = I - omega_c I_P^ A_c^-1 I_P^H A^,
# M^ = S^{n_s} K^ S^{n_s}.  Reading: the printed K^ omits omega_c, which
# Fig. 4 varies; it is included.

def periodic_fine_matrix(p, N, kappa):
    """Periodic Q_p matrix (h = 1/N) of int grad.grad - kappa int u v."""
    from .fem import element_matrices
    h = 1.0 / N
    S, M = element_matrices(p, h, 2)
    Ae = S - kappa * M
    n1 = N * p
    A = np.zeros((n1 * n1, n1 * n1), dtype=complex)
    for cy in range(N):
        for cx in range(N):
            nodes = [((cy * p + ay) % n1) * n1 + (cx * p + ax) % n1
                     for ay in range(p + 1) for ax in range(p + 1)]
            A[np.ix_(nodes, nodes)] += Ae
    return A


def periodic_coarse_matrix(p, N, k, eps):
    """Periodic quasi-FE QSFEM matrix on the coarse mesh (spacing 2h/p)."""
    from .qsfem import cell_q_matrix, q_weights
    r = p // 2
    Nc = N * r
    hc = 1.0 / Nc
    q0, qe, qd = q_weights(hc * k)
    m1 = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    E = cell_q_matrix(q0, qe, qd).astype(complex) - 1j * eps * np.kron(m1, m1) * hc * hc
    A = np.zeros((Nc * Nc, Nc * Nc), dtype=complex)
    for cy in range(Nc):
        for cx in range(Nc):
            nodes = [((cy + ay) % Nc) * Nc + (cx + ax) % Nc for ay in (0, 1) for ax in (0, 1)]
            A[np.ix_(nodes, nodes)] += E
    return A


def periodic_prolongation(p, N):
    from .fem import gll, lagrange
    r = p // 2
    xf, _ = gll(p)
    L, _ = lagrange(np.linspace(0, 1, r + 1), xf)
    n1, nc = N * p, N * r
    P1 = np.zeros((n1, nc))
    for c in range(N):
        for a in range(p):  # node c p + a (a = p belongs to the next cell)
            for b in range(r + 1):
                P1[c * p + a, (c * r + b) % nc] = L[a, b]
    return np.kron(P1, P1)


def _lattice(n1, per_cell):
    idx = np.arange(n1 * n1)
    ix, iy = idx % n1, idx // n1
    return ix // per_cell, iy // per_cell, (iy % per_cell) * per_cell + ix % per_cell


def symbol_of(P, N, rows_per, cols_per, theta):
    """sigma(P)(theta) from a periodic matrix: rows = dofs of the unit cell at
    the origin, phases of the minimal-image lattice offsets of the columns."""
    nr, nc = N * rows_per, N * cols_per
    ax_r, ay_r, j_r = _lattice(nr, rows_per)
    ax_c, ay_c, j_c = _lattice(nc, cols_per)
    out = np.zeros((rows_per * rows_per, cols_per * cols_per), dtype=complex)
    origin = np.nonzero((ax_r == 0) & (ay_r == 0))[0]
    bx = ((ax_c + N // 2) % N) - N // 2
    by = ((ay_c + N // 2) % N) - N // 2
    ph = np.exp(1j * (theta[0] * bx + theta[1] * by))
    for row in origin:
        np.add.at(out[j_r[row]], j_c, P[row] * ph)
    return out


class BlochTwoGrid:
    """Symbols and the periodic brute-force operators of the two-grid cycle."""

    def __init__(self, p, N, kh, D=0.01, alpha_s=0.2, n_s=1, omega_c=1.0):
        self.p, self.N, self.n_s, self.omega_c = p, N, n_s, omega_c
        k = kh * N  # h = 1 / N
        eps = k * k * D / math.pi
        self.A = periodic_fine_matrix(p, N, k * k + 1j * eps)
        self.As = periodic_fine_matrix(p, N, k * k * (1 + 1j * alpha_s) + 1j * eps)
        self.Ac = periodic_coarse_matrix(p, N, k, eps)
        self.IP = periodic_prolongation(p, N)

    def brute_force(self):
        n = self.A.shape[0]
        S = np.eye(n) - np.linalg.solve(self.As, self.A)
        K = np.eye(n) - self.omega_c * self.IP @ np.linalg.solve(self.Ac, self.IP.T @ self.A)
        Sn = np.linalg.matrix_power(S, self.n_s)
        return Sn @ K @ Sn

    def symbol(self, theta):
        p, N, r = self.p, self.N, self.p // 2
        Ah = symbol_of(self.A, N, p, p, theta)
        Ash = symbol_of(self.As, N, p, p, theta)
        Ach = symbol_of(self.Ac, N, r, r, theta)
        IPh = symbol_of(self.IP, N, p, r, theta)
        n = p * p
        S = np.eye(n) - np.linalg.solve(Ash, Ah)
        K = np.eye(n) - self.omega_c * IPh @ np.linalg.solve(Ach, IPh.conj().T @ Ah)
        Sn = np.linalg.matrix_power(S, self.n_s)
        return Sn @ K @ Sn

    def rho(self, n_theta=32):
        ts = np.linspace(-math.pi, math.pi, n_theta, endpoint=False)
        return max(np.max(np.abs(np.linalg.eigvals(self.symbol((a, b))))) for a in ts for b in ts)
