"""Pins of the oracle's fine dispersion, plain fit and surrogate network (CPU)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dispersion as d
from oracle import fem, mlp, qsfem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def q1_symbol(kh, th):
    """Symbol of the Q1 stencils printed in Sec. 3.3 (stiffness - (kh)^2 mass)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "q1_stencils.txt"))
            if l.strip() and not l.startswith("#")]
    S = np.array([[float(Fraction(v)) for v in r] for r in rows[1:4]])
    M = np.array([[float(Fraction(v)) for v in r] for r in rows[5:8]])
    tot = 0.0
    for iy, dy in enumerate((-1, 0, 1)):
        for ix, dx in enumerate((-1, 0, 1)):
            ph = np.exp(1j * (th[0] * dx + th[1] * dy))
            tot += (S[iy, ix] - kh * kh * M[iy, ix]) * ph
    return tot


@pytest.mark.parametrize("th", [(0.3, -0.7), (1.1, 2.0), (0.0, 0.0)])
def test_bloch_symbol_p1_equals_printed_stencil_symbol(th):
    kh = 0.9
    assert abs(d.bloch_symbol(1, kh, th)[0, 0] - q1_symbol(kh, th)) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_bloch_symbol_by_periodic_brute_force(p):
    """Bloch theorem: the eigenvalues of the assembled FE matrix on an N x N
    periodic mesh are the union of eig(A^(theta)) over theta in (2 pi / N) Z^2."""
    N, kh = 4, 0.8
    K1, M1 = fem.ref_matrices(p)
    Ae = np.kron(K1, M1) + np.kron(M1, K1) - kh * kh * np.kron(M1, M1)
    n1 = N * p
    A = np.zeros((n1 * n1, n1 * n1))
    for cy in range(N):
        for cx in range(N):
            nodes = [((cy * p + ay) % n1) * n1 + (cx * p + ax) % n1
                     for ay in range(p + 1) for ax in range(p + 1)]
            A[np.ix_(nodes, nodes)] += Ae
    ev = np.sort(np.linalg.eigvalsh(A))
    sym = []
    for jy in range(N):
        for jx in range(N):
            th = (2 * math.pi * jx / N, 2 * math.pi * jy / N)
            sym.extend(np.linalg.eigvalsh(d.bloch_symbol(p, kh, th)))
    assert np.allclose(ev, np.sort(sym), atol=1e-11)


@pytest.mark.parametrize("t", [0.0, 0.4, math.pi / 4])
def test_fine_radius_p1_closed_form(t):
    kh = 0.8
    r = d.fine_radius(1, kh, t)
    c1, c2 = math.cos(r * math.cos(t)), math.cos(r * math.sin(t))
    sigma = 8 / 3 - 2 / 3 * (c1 + c2) - 4 / 3 * c1 * c2 - kh ** 2 * (4 / 9 + 2 / 9 * (c1 + c2) + c1 * c2 / 9)
    assert abs(sigma) < 1e-13


def test_fine_radius_converges_to_k_with_order():
    kh = 2 * math.pi * 4 / 10
    errs = [abs(d.fine_radius(p, kh * p / 4, d.T1) / (kh * p / 4) - 1) for p in (2, 4)]
    assert errs[1] < errs[0] * 1e-1


@pytest.mark.parametrize("eta", [0.4, 1.0, 1.6])
def test_fit_reduces_to_qsfem_for_exact_wavenumbers(eta):
    """With the true wavenumber at both angles the fit is the QSFEM stencil."""
    assert np.allclose(d.fit_from_radii(eta, eta, eta), qsfem.q_weights(eta), rtol=1e-13)


@pytest.mark.parametrize("p,eta", [(2, 1.0), (4, 1.2)])
def test_plain_fit_matches_fine_dispersion_at_the_two_angles(p, eta):
    q = d.plain_fit(eta, p)
    kh = eta * p / 2
    for t in (d.T1, d.T2):
        zf = d.fine_radius(p, kh, t) * 2 / p
        assert abs(d.coarse_radius(q, t, eta) - zf) < 1e-12
    # and matches it better than QSFEM over all directions
    assert d.dispersion_mismatch(q, eta, p, 8) < d.dispersion_mismatch(qsfem.q_weights(eta), eta, p, 8)


# ---------------------------------------------------------------- MLP --------
@pytest.mark.parametrize("n_out", [2, 3])
def test_mlp_gradient_by_central_differences(n_out):
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(mlp.n_params(n_out)) * 0.3
    x = rng.standard_normal((7, 3))
    t = rng.standard_normal((7, n_out))
    _, g = mlp.loss_and_grad(theta, x, t)
    assert mlp.n_out_of(theta) == n_out
    idx = rng.choice(mlp.n_params(n_out), 40, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (mlp.loss_and_grad(theta + e, x, t)[0] - mlp.loss_and_grad(theta - e, x, t)[0]) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9


def test_adam_first_step_is_lr_times_sign():
    th = np.array([1.0, -2.0])
    g = np.array([0.3, -5.0])
    new, m, v = mlp.adam_step(th, g, np.zeros(2), np.zeros(2), 1, lr=0.01, eps=0.0)
    assert np.allclose(new, th - 0.01 * np.sign(g))


def test_target_transform_round_trip():
    e = np.array([-1e-3, -4e-7, -2e-12])
    assert np.allclose(mlp.errors_from_targets(mlp.targets_from_errors(e)), e, rtol=1e-12)


# ------------------------------------------------- Bloch LFA of the two-grid --
@pytest.mark.parametrize("p,N", [(2, 4), (4, 3)])
def test_two_grid_symbols_match_periodic_brute_force(p, N):
    """eig(M) on the periodic mesh = union over theta in (2 pi / N) Z^2 of
    eig(M^(theta)) (Sec. 6.1: the symbols block-diagonalise the cycle)."""
    from oracle.lfa import BlochTwoGrid
    lfa = BlochTwoGrid(p, N, kh=2 * math.pi * p / 10 * 1.0, D=0.01, alpha_s=0.2)
    ev = np.linalg.eigvals(lfa.brute_force())
    sym = np.concatenate([np.linalg.eigvals(lfa.symbol((2 * math.pi * jx / N, 2 * math.pi * jy / N)))
                          for jy in range(N) for jx in range(N)])
    # match every brute-force eigenvalue to a distinct symbol eigenvalue
    used = np.zeros(len(sym), dtype=bool)
    for z in ev:
        d_ = np.abs(sym - z) + used * 1e9
        i = int(np.argmin(d_))
        assert d_[i] < 1e-8 * max(1.0, abs(z)), (z, sym[i])
        used[i] = True


def test_lfa_convergence_factor_p4_at_10_dof_per_wavelength():
    """Sec. 6.3: for order 4 the method converges above 8 DOF per wavelength
    (alpha_s = 0.2, D = 0.01, n_s = 1, omega_c = 1)."""
    from oracle.lfa import BlochTwoGrid
    lfa = BlochTwoGrid(4, 5, kh=2 * math.pi * 4 / 10, D=0.01, alpha_s=0.2)
    rho = lfa.rho(24)
    print("rho p=4, 10 DOF/wavelength:", rho)
    assert rho < 1.0
