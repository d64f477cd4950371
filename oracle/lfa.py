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
