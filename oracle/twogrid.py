"""Two-grid step (Alg. 1), the preconditioner map and the outer Krylov method.

Follows Sec. 4 of the paper:
  TwoGridStep(u, f): n_s smoother steps; r_c = I_P^*(f - A u); solve
  A_c u_c = r_c (direct solver); u += omega_c I_P u_c; n_s smoother steps.
  The preconditioner is the map f -> TwoGridStep(0, f).

Readings (the outer Krylov method is not specified in the paper):
  * right-preconditioned GMRES from x0 = 0, modified Gram-Schmidt Arnoldi
    with the Hermitian inner product, Givens rotations, no restart unless
    asked; the preconditioned directions z_j are stored and x = sum y_j z_j
    (identical to GMRES for a fixed preconditioner, and to FGMRES);
  * a cycle ends when the recurrence residual |g_{j+1}| / ||f|| <= rtol; the
    iterate is then converged only if its true residual satisfies
    ||f - A x|| / ||f|| <= rtol, otherwise a new cycle starts from that
    residual (until maxit).
The coarse solve is a sparse LU of the quasi-FE QSFEM matrix.

Dirichlet sides (eq. Helmholtz_eq): their nodes are eliminated on both levels
and from I_P; a right-hand side that vanishes there gives iterates that vanish
there, the iteration on the remaining unknowns.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import helmholtz_matrix
from .qsfem import coarse_cell_values, coarse_matrix
from .qsfem3d import coarse_matrix_3d
from .smoother import CSDDSmoother
from .transfer import prolongation


class TwoGrid:
    def __init__(self, p, k, eps=None, alpha_s=0.5, l_dd=8, robin=None, n_dd=1,
                 n_s=1, omega_c=1.0, coarse_q=None, dirichlet=None):
        self.dim = k.ndim
        self.N = k.shape[0]
        self.p = p
        if eps is None:
            eps = np.zeros_like(k)
        if robin is None:
            robin = (True,) * (2 * self.dim)
        if dirichlet is not None:
            assert not any(r and d for r, d in zip(robin, dirichlet)), \
                "a side is either absorbing or Dirichlet"
        self.A = helmholtz_matrix(p, k, eps, robin, 0.0, dirichlet)
        self.A_s = helmholtz_matrix(p, k, eps, robin, alpha_s, dirichlet)
        self.smoother = CSDDSmoother(p, k, eps, alpha_s, l_dd, robin, n_dd,
                                     A=self.A, A_s=self.A_s, dirichlet=dirichlet)
        self.I_P = prolongation(self.N, p, self.dim, dirichlet)
        kc = coarse_cell_values(k, p)
        epsc = coarse_cell_values(eps, p)
        if self.dim == 3:
            self.A_c = coarse_matrix_3d(kc, epsc, robin, q=coarse_q, dirichlet=dirichlet)
        else:
            self.A_c = coarse_matrix(kc, epsc, robin, q=coarse_q, dirichlet=dirichlet)
        self.coarse_lu = spla.splu(self.A_c.tocsc())
        self.n_s = n_s
        self.omega_c = omega_c

    # individual steps -----------------------------------------------------
    def residual(self, u, f):
        return f - self.A @ u

    def smooth(self, u, f):
        return self.smoother.apply(u, f)

    def restrict(self, r):
        return self.I_P.T @ r

    def prolong_add(self, u, uc, omega):
        return u + omega * (self.I_P @ uc)

    def coarse_solve(self, rc):
        return self.coarse_lu.solve(rc)

    # Alg. 1 -----------------------------------------------------------------
    def twogrid_step(self, u, f):
        for _ in range(self.n_s):
            u = self.smooth(u, f)
        rc = self.restrict(self.residual(u, f))
        uc = self.coarse_solve(rc)
        u = self.prolong_add(u, uc, self.omega_c)
        for _ in range(self.n_s):
            u = self.smooth(u, f)
        return u

    def precond(self, v):
        return self.twogrid_step(np.zeros_like(v), v)

    def gmres(self, f, rtol=1e-6, maxit=300, restart=None, callback=None):
        return gmres_right(lambda x: self.A @ x, self.precond, f, rtol, maxit, restart,
                           callback)


def gmres_right(matvec, precond, f, rtol=1e-6, maxit=300, restart=None, callback=None):
    """Right-preconditioned GMRES (stored preconditioned directions), x0 = 0.

    Returns (x, iters, rel_res_history).  iters counts Arnoldi steps, i.e.
    preconditioner applications; converged means the true residual meets rtol.
    """
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape[0]
    m = maxit if restart is None else restart
    x = np.zeros(n, dtype=np.complex128)
    fnorm = np.linalg.norm(f)
    hist = [1.0]
    if fnorm == 0.0:
        return x, 0, hist
    total = 0
    r = f.copy()
    while True:
        beta = np.linalg.norm(r)
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        done = False
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # apply previous rotations
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j], rr = givens(H[j, j], H[j + 1, j])
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            rel = abs(g[j + 1]) / fnorm
            hist.append(rel)
            if callback is not None:
                callback(total, rel)
            if rel <= rtol or total >= maxit:
                done = True
                break
        y = np.zeros(j_end, dtype=np.complex128)
        for i in reversed(range(j_end)):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:j_end]) / H[i, i]
        x = x + y @ Z[:j_end]
        r = f - matvec(x)
        if np.linalg.norm(r) <= rtol * fnorm or total >= maxit:
            return x, total, hist


def givens(a, b):
    """Complex Givens rotation [c s; -conj(s) conj(c)] with c real-positive
    direction chosen so that the rotated second entry vanishes."""
    if b == 0:
        return 1.0 + 0j, 0.0 + 0j, a
    if a == 0:
        return 0.0 + 0j, np.conj(b) / abs(b), abs(b) + 0j
    t = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / t + 0j
    s = (a / abs(a)) * np.conj(b) / t
    return c, s, (a / abs(a)) * t
