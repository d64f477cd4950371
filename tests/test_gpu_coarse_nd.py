"""GPU parity of the two coarse factorisations (nested dissection and the
block elimination over grid lines or planes) against the oracle's coarse
matrix solved by sparse LU: relative L2 error 1e-11 for 1 to 9 right-hand
sides (every right-hand-side chunk width of the solve kernels), 2-D and 3-D,
absorbing, Neumann and Dirichlet sides."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle.qsfem import coarse_cell_values, coarse_matrix
from oracle.qsfem3d import coarse_matrix_3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def hetero_k(N, dim, p, seed, ppw=8.0):
    c = syn.grf_speed(N, dim, 0.2, 1.5, 4.0, seed=seed)
    return syn.wavenumber_from_speed(c, p * N / ppw)


CASES_2D = [  # (N, p, l_dd, nrhs, bc)
    (37, 2, 8, 1, None),
    (19, 4, 6, 3, None),
    (64, 2, 8, 9, None),                       # C1's coarse grid, 8 + 1 right-hand sides
    (50, 4, 8, 2, ("robin", "dirichlet", "neumann", "robin")),
    (7, 6, 3, 5, ("dirichlet",) * 4),
]


@pytest.mark.parametrize("solver", ["nd", "lines"])
@pytest.mark.parametrize("N,p,l_dd,nrhs,bc", CASES_2D)
def test_coarse_solvers_2d(N, p, l_dd, nrhs, bc, solver):
    from paper_2509_17494_amd import TwoGridSolver
    print(f"case coarse2d {solver} N={N} p={p} nrhs={nrhs} bc={bc}", flush=True)
    k = hetero_k(N, 2, p, seed=40 + N)
    bcs = bc or ("robin",) * 4
    robin = tuple(b == "robin" for b in bcs)
    dirichlet = tuple(b == "dirichlet" for b in bcs)
    Ac = coarse_matrix(coarse_cell_values(k, p), robin=robin, dirichlet=dirichlet)
    s = TwoGridSolver(k, order=p, l_dd=l_dd, max_rhs=nrhs, bc=bcs, coarse_solver=solver)
    info = s.info()
    assert info["coarse_solver"] == (2 if solver == "nd" else 1)
    assert 0.0 <= info["coarse_check"] < 1e-9
    rc = syn.random_complex((nrhs, Ac.shape[0]), seed=N + nrhs)
    lu = spla.splu(Ac.tocsc())
    ref = np.stack([lu.solve(x) for x in rc])
    uc = to_np(s.coarse_solve(to_dev(rc)))
    err = rel(uc, ref)
    print(f"  rel err {err:.2e}, check {info['coarse_check']:.2e}, levels {info['coarse_levels']} "
          f"refine {info['coarse_refine_exact']} (preconditioner {info['coarse_refine']}, "
          f"{info['coarse_check_pc']:.2e})", flush=True)
    if solver == "nd":  # the preconditioner's refinement reaches 1e-8 or stops at 3 steps
        assert info["coarse_refine"] <= info["coarse_refine_exact"]
        assert 0.0 <= info["coarse_check_pc"] <= 1e-8 or info["coarse_refine"] == 3
    assert err < 1e-11
    s.close()


CASES_3D = [  # (N, p, l_dd, nrhs, bc)
    (12, 2, 4, 1, None),
    (9, 4, 3, 8, None),
    (10, 2, 5, 3, ("robin", "dirichlet", "neumann", "robin", "dirichlet", "robin")),
]


@pytest.mark.parametrize("solver", ["nd", "lines"])
@pytest.mark.parametrize("N,p,l_dd,nrhs,bc", CASES_3D)
def test_coarse_solvers_3d(N, p, l_dd, nrhs, bc, solver):
    from paper_2509_17494_amd import TwoGridSolver
    print(f"case coarse3d {solver} N={N} p={p} nrhs={nrhs} bc={bc}", flush=True)
    k = hetero_k(N, 3, p, seed=50 + N)
    bcs = bc or ("robin",) * 6
    robin = tuple(b == "robin" for b in bcs)
    dirichlet = tuple(b == "dirichlet" for b in bcs)
    Ac = coarse_matrix_3d(coarse_cell_values(k, p), robin=robin, dirichlet=dirichlet)
    s = TwoGridSolver(k, order=p, l_dd=l_dd, max_rhs=nrhs, bc=bcs, coarse_solver=solver)
    info = s.info()
    assert info["coarse_solver"] == (2 if solver == "nd" else 1)
    rc = syn.random_complex((nrhs, Ac.shape[0]), seed=N + 7 * nrhs)
    lu = spla.splu(Ac.tocsc())
    ref = np.stack([lu.solve(x) for x in rc])
    uc = to_np(s.coarse_solve(to_dev(rc)))
    err = rel(uc, ref)
    print(f"  rel err {err:.2e}, check {info['coarse_check']:.2e}", flush=True)
    assert err < 1e-11
    s.close()


def test_nd_and_lines_solve_c1_alike():
    """A full C1 solve with nested dissection and with the line elimination
    takes the same iterations and agrees to 1e-10."""
    from paper_2509_17494_amd import TwoGridSolver
    cfg = syn.config("C1")
    f = syn.gaussian_load(cfg["n"], cfg["p"], cfg["centres"], cfg["sigma"])
    out = {}
    for solver in ("nd", "lines"):
        s = TwoGridSolver(cfg["k"], order=cfg["p"], l_dd=cfg["l_dd"], alpha_s=cfg["alpha_s"],
                          coarse_solver=solver)
        u, st = s.solve(to_dev(f))
        out[solver] = (s.info()["coarse_solver"], to_np(u), st)
        s.close()
    assert out["nd"][0] == 2 and out["lines"][0] == 1
    st_nd, st_ln = out["nd"][2], out["lines"][2]
    assert st_nd.status == 0 and st_ln.status == 0
    assert st_nd.iters == st_ln.iters
    assert rel(out["nd"][1], out["lines"][1]) < 1e-10


def test_automatic_choice_follows_the_time_model():
    """The automatic choice: the line elimination for C1's small grid and one
    right-hand side (a few launches beat the dissection tree's levels), nested
    dissection for C3's 64 right-hand sides (complex64 preconditioner, no
    refinement) and for C2's large grid."""
    from paper_2509_17494_amd import TwoGridSolver
    got = {}
    for name, kw in (("C1", {}), ("C3", dict(max_rhs=64, gemm="bf16")), ("C2", {})):
        cfg = syn.config(name)
        s = TwoGridSolver(cfg["k"], order=cfg["p"], l_dd=cfg["l_dd"], alpha_s=cfg["alpha_s"], **kw)
        got[name] = s.info()["coarse_solver"]
        s.close()
    print(f"automatic coarse solver: {got}", flush=True)
    assert got == {"C1": 1, "C3": 2, "C2": 2}



def test_nd_calls_of_changing_width():
    """One context, calls of changing width: 64 right-hand sides (eight passes
    of 8), then 3, 17, 1 and 64 again; every call matches sparse LU to 1e-11."""
    from paper_2509_17494_amd import TwoGridSolver
    N, p = 64, 2
    k = hetero_k(N, 2, p, seed=77)
    Ac = coarse_matrix(coarse_cell_values(k, p), robin=(True,) * 4, dirichlet=(False,) * 4)
    lu = spla.splu(Ac.tocsc())
    s = TwoGridSolver(k, order=p, l_dd=8, max_rhs=64, coarse_solver="nd")
    assert s.info()["coarse_solver"] == 2
    for i, nrhs in enumerate((64, 3, 17, 1, 64)):
        print(f"case nd call {i} nrhs={nrhs}", flush=True)
        rc = syn.random_complex((nrhs, Ac.shape[0]), seed=300 + i)
        ref = np.stack([lu.solve(x) for x in rc])
        err = rel(to_np(s.coarse_solve(to_dev(rc))), ref)
        print(f"  rel err {err:.2e}", flush=True)
        assert err < 1e-11
    s.close()
