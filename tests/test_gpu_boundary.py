"""GPU parity for the boundary and parameter variants, against the FP64 oracle
on the same seeded inputs:
  * homogeneous Dirichlet sides (eq. Helmholtz_eq; nodes eliminated on both
    levels, in the subdomain matrices and from I_P), mixed with absorbing and
    Neumann sides, in 2-D (both FP64 subdomain-operator layouts) and 3-D;
  * sin^2 absorbing layers (per-cell eps, the recipe of the paper's
    convergence tests);
  * the two-grid parameters of Table 1(b): n_s = 2 smoothing steps and
    omega_c = 0.8, with n_dd = 2 DD iterations per smoother step.
Bars as in the other parity tests (relative L2 error): 1e-12 for single
operator applications, 1e-13 for the transfers, 1e-11 for the coarse solve
and the two-grid step, 1e-10 for the solution after the same iteration count.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle.fem import side_mask
from oracle.twogrid import TwoGrid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


CASES = [  # (N, p, l_dd, bc): bc per side x-, x+, y-, y+(, z-, z+)
    (19, 4, 6, ("dirichlet", "robin", "neumann", "dirichlet")),      # dense operator rows
    (33, 4, 8, ("robin", "dirichlet", "dirichlet", "neumann")),      # symmetric tiles
    (7, 8, 3, ("dirichlet", "dirichlet", "robin", "robin")),
    (6, 2, 3, ("dirichlet", "robin", "neumann", "robin", "robin", "dirichlet")),
    (5, 4, 2, ("robin", "neumann", "dirichlet", "robin", "dirichlet", "robin")),
]


def problem(N, p, l_dd, bc, **kw):
    """Oracle and GPU solver for a heterogeneous medium with sin^2 absorbing
    layers (16 DOFs wide) along the absorbing sides."""
    from paper_2509_17494_amd import TwoGridSolver
    dim = len(bc) // 2
    c = syn.grf_speed(N, dim, 0.2, 1.5, 4.0, seed=N + p)
    k = syn.wavenumber_from_speed(c, p * N / 8.0)
    robin = tuple(b == "robin" for b in bc)
    dirichlet = tuple(b == "dirichlet" for b in bc)
    eps = syn.absorbing_layer_eps(k, p, robin, dofs=16.0)
    tg = TwoGrid(p, k, eps=eps, l_dd=l_dd, robin=robin, dirichlet=dirichlet, **kw)
    s = TwoGridSolver(k, eps=eps, order=p, l_dd=l_dd, bc=bc, max_rhs=2, **kw)
    mask = side_mask(N * p + 1, dim, dirichlet)
    cmask = side_mask(N * (p // 2) + 1, dim, dirichlet)
    return tg, s, mask, cmask


def ids(case):
    return f"N{case[0]}p{case[1]}d{len(case[3]) // 2}"


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_steps_with_dirichlet_sides_and_absorbing_layers(case):
    N, p, l_dd, bc = case
    print(f"case boundary steps {ids(case)} bc={bc}", flush=True)
    tg, s, mask, cmask = problem(N, p, l_dd, bc, alpha_s=0.3, n_dd=2, n_s=2, omega_c=0.8)
    n, nc = tg.A.shape[0], tg.A_c.shape[0]
    u0 = syn.random_complex((2, n), seed=31)
    f = syn.random_complex((2, n), seed=32)
    rc0 = syn.random_complex((2, nc), seed=33)
    # residual: unit rows on the eliminated nodes give f - u there
    r = to_np(s.residual(to_dev(u0), to_dev(f)))
    ref = np.stack([tg.residual(u0[i], f[i]) for i in range(2)])
    assert rel(r, ref) < 1e-12
    assert np.array_equal(r[:, mask], f[:, mask] - u0[:, mask])
    # transfers
    rc = to_np(s.restrict(to_dev(ref)))
    assert rel(rc, np.stack([tg.restrict(x) for x in ref])) < 1e-13
    assert np.all(rc[:, cmask] == 0)
    u = to_dev(u0)
    s.prolong(to_dev(rc0), u, omega=0.8)
    got = to_np(u)
    assert rel(got, np.stack([tg.prolong_add(u0[i], rc0[i], 0.8) for i in range(2)])) < 1e-13
    assert np.array_equal(got[:, mask], u0[:, mask])
    # smoother (n_dd = 2)
    u = to_dev(u0)
    s.smooth(u, to_dev(f))
    assert rel(to_np(u), np.stack([tg.smooth(u0[i], f[i]) for i in range(2)])) < 1e-12
    # coarse solve
    lu = spla.splu(tg.A_c.tocsc())
    uc = to_np(s.coarse_solve(to_dev(rc0)))
    assert rel(uc, np.stack([lu.solve(x) for x in rc0])) < 1e-11
    # two-grid step with n_s = 2, omega_c = 0.8
    u = to_dev(u0)
    s.twogrid(u, to_dev(f))
    assert rel(to_np(u), np.stack([tg.twogrid_step(u0[i], f[i]) for i in range(2)])) < 1e-11
    s.close()


@pytest.mark.parametrize("case", [CASES[0], CASES[3]], ids=ids)
def test_solve_with_dirichlet_sides_same_iterations(case):
    N, p, l_dd, bc = case
    print(f"case boundary solve {ids(case)}", flush=True)
    tg, s, mask, _ = problem(N, p, l_dd, bc, alpha_s=0.2, n_s=2, omega_c=0.8)
    dim = len(bc) // 2
    f = syn.gaussian_load(N, p, [[0.4] * dim], 2.0 / N, dim=dim)
    f[:, mask] = 0.0
    x_ref, it_ref, _ = tg.gmres(f[0], 1e-8)
    u, st = s.solve(to_dev(f), rtol=1e-8)
    x = to_np(u)[0]
    print(f"  oracle iters {it_ref}, gpu iters {st.iters}, rel err {rel(x, x_ref):.2e}", flush=True)
    assert st.status == 0 and st.iters == it_ref and st.rel_res <= 1e-8
    assert rel(x, x_ref) < 1e-10
    assert np.all(x[mask] == 0)
    s.close()


def test_mixed_precision_solve_with_dirichlet_sides():
    """BF16 subdomain operators, complex64 preconditioner, FP64 outer FGMRES:
    converges to the FP64 tolerance on the true residual, zero on the
    eliminated nodes."""
    from paper_2509_17494_amd import TwoGridSolver
    N, p = 40, 4
    bc = ("dirichlet", "robin", "dirichlet", "neumann")
    k = syn.wavenumber_from_speed(syn.grf_speed(N, 2, 0.1, 1.5, 4.0, seed=4), p * N / 10.0)
    robin = tuple(b == "robin" for b in bc)
    eps = syn.absorbing_layer_eps(k, p, robin)
    mask = side_mask(N * p + 1, 2, tuple(b == "dirichlet" for b in bc))
    s = TwoGridSolver(k, eps=eps, order=p, alpha_s=0.2, l_dd=8, bc=bc, gemm="bf16", max_rhs=4)
    f = syn.gaussian_load(N, p, [[0.3, 0.3], [0.7, 0.4], [0.5, 0.8], [0.2, 0.6]], 2.0 / N)
    f[:, mask] = 0.0
    fd = to_dev(f)
    u, st = s.solve(fd, rtol=1e-6, precond="c64")
    r = to_np(s.residual(u, fd))
    true_res = max(np.linalg.norm(r[i]) / np.linalg.norm(f[i]) for i in range(4))
    print(f"mixed: iters {st.iters}, true rel res {true_res:.2e}", flush=True)
    assert st.status == 0 and st.rel_res <= 1e-6
    assert true_res <= 1e-6 * (1 + 1e-9)   # the same FP64 residual, computed here
    assert np.all(to_np(u)[:, mask] == 0)
    s.close()
