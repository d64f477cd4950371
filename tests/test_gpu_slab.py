"""GPU parity of the slab-factor layout of the subdomain solves (block
factorisation of A_s^(i) over slabs of P node layers, forward and backward
sweeps) against the FP64 oracle's exact subdomain solves, in 2-D and 3-D,
with absorbing, Neumann and Dirichlet sides.  Bars as in the other parity
tests: 1e-12 (FP64) and 1e-5 (FP32 storage) for the smoother, 1e-11 for the
two-grid step, 1e-10 for a solve after the same iteration count."""
import numpy as np
import pytest

import synthetic as syn
from oracle.smoother import CSDDSmoother
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


def medium(N, p, dim, seed):
    c = syn.grf_speed(N, dim, 0.2, 1.5, 4.0, seed=seed)
    return syn.wavenumber_from_speed(c, p * N / 8.0)


def solver(k, p, l_dd, **kw):
    from paper_2509_17494_amd import TwoGridSolver
    s = TwoGridSolver(k, order=p, l_dd=l_dd, layout="slab", **kw)
    assert s.info()["smoother_layout"] == 3
    return s


# (N, p, l_dd): several subdomain sizes, ragged blocks, every order; l_dd = 1
# gives subdomains of 2 and 3 slabs (a middle slab with one or two chains of
# a single slab), N = 1 a single subdomain of one slab (the middle alone, no
# chain), l_dd = 8 at N = 37 up to 10 slabs
CASES_2D = [(19, 4, 6), (33, 4, 8), (7, 6, 3), (5, 8, 2), (37, 2, 8), (12, 2, 5), (9, 4, 1),
            (1, 4, 1), (1, 2, 1)]


@pytest.mark.parametrize("packed", ["1", "0"])
@pytest.mark.parametrize("N,p,l_dd", CASES_2D)
def test_smooth_slab_2d(N, p, l_dd, packed, monkeypatch):
    """Both storages of G_t: packed (lower block triangle as skewed tiles and
    a dense strip; slabs of fewer than 64 rows are all strip) and whole."""
    print(f"case slab smooth N={N} p={p} l_dd={l_dd} packed={packed}", flush=True)
    monkeypatch.setenv("TH_SLAB_PACKED", packed)
    k = medium(N, p, 2, seed=N)
    sm = CSDDSmoother(p, k, None, 0.5, l_dd)
    s = solver(k, p, l_dd, max_rhs=3, coarse=None)
    assert s.info()["slab_packed"] == int(packed)
    u0 = syn.random_complex((3, sm.n_nodes), seed=1)
    f = syn.random_complex((3, sm.n_nodes), seed=2)
    ref = np.stack([sm.apply(u0[i], f[i]) for i in range(3)])
    u = to_dev(u0)
    s.smooth(u, to_dev(f))
    err = rel(to_np(u), ref)
    print(f"  rel err {err:.2e}", flush=True)
    assert err < 1e-12
    s.close()


def test_smooth_slab_ndd2_neumann_and_f32():
    N, p, l_dd = 18, 4, 5
    k = medium(N, p, 2, seed=3)
    robin = (True, False, True, False)
    bc = ("robin", "neumann", "robin", "neumann")
    sm = CSDDSmoother(p, k, None, 0.3, l_dd, robin=robin, n_dd=2)
    u0 = syn.random_complex((2, sm.n_nodes), seed=4)
    f = syn.random_complex((2, sm.n_nodes), seed=5)
    ref = np.stack([sm.apply(u0[i], f[i]) for i in range(2)])
    s = solver(k, p, l_dd, alpha_s=0.3, n_dd=2, bc=bc, max_rhs=2, coarse=None)
    u = to_dev(u0)
    s.smooth(u, to_dev(f))
    assert rel(to_np(u), ref) < 1e-12
    s.close()
    s32 = solver(k, p, l_dd, alpha_s=0.3, n_dd=2, bc=bc, max_rhs=2, coarse=None, gemm="f32")
    u = to_dev(u0, torch.complex64)
    s32.smooth(u, to_dev(f, torch.complex64))
    assert rel(to_np(u), ref) < 1e-5
    s32.close()


@pytest.mark.parametrize("N,p,l_dd,packed", [(6, 2, 3, "1"), (6, 2, 3, "0"), (5, 4, 2, None),
                                              (7, 2, 4, None)])
def test_smooth_slab_3d(N, p, l_dd, packed, monkeypatch):
    """3-D slabs; (6, 2, 3) also with packed G_t (slabs of 162 and 243 rows:
    two and three 64-row blocks of tiles, strips of 34 and 51 rows; one
    right-hand side per chunk)."""
    print(f"case slab smooth 3-D N={N} p={p} packed={packed}", flush=True)
    if packed is not None:
        monkeypatch.setenv("TH_SLAB_PACKED", packed)
    k = medium(N, p, 3, seed=N + 1)
    sm = CSDDSmoother(p, k, None, 0.5, l_dd)
    s = solver(k, p, l_dd, max_rhs=2, coarse=None)
    if packed is not None:
        assert s.info()["slab_packed"] == int(packed)
    u0 = syn.random_complex((2, sm.n_nodes), seed=6)
    f = syn.random_complex((2, sm.n_nodes), seed=7)
    ref = np.stack([sm.apply(u0[i], f[i]) for i in range(2)])
    u = to_dev(u0)
    s.smooth(u, to_dev(f))
    assert rel(to_np(u), ref) < 1e-12
    s.close()


@pytest.mark.parametrize("N,p,l_dd,bc", [
    (19, 4, 6, ("dirichlet", "robin", "neumann", "dirichlet")),
    (5, 4, 2, ("robin", "neumann", "dirichlet", "robin", "dirichlet", "robin")),
])
def test_twogrid_slab_dirichlet_and_layers(N, p, l_dd, bc):
    """Two-grid step (n_s = 2, omega_c = 0.8) with Dirichlet sides and sin^2
    absorbing layers along the absorbing sides."""
    print(f"case slab twogrid N={N} p={p} bc={bc}", flush=True)
    dim = len(bc) // 2
    k = medium(N, p, dim, seed=N + p)
    robin = tuple(b == "robin" for b in bc)
    dirichlet = tuple(b == "dirichlet" for b in bc)
    eps = syn.absorbing_layer_eps(k, p, robin, dofs=16.0)
    tg = TwoGrid(p, k, eps=eps, alpha_s=0.3, l_dd=l_dd, robin=robin, dirichlet=dirichlet,
                 n_s=2, omega_c=0.8)
    s = solver(k, p, l_dd, eps=eps, alpha_s=0.3, bc=bc, n_s=2, omega_c=0.8, max_rhs=1)
    n = tg.A.shape[0]
    u0 = syn.random_complex(n, seed=8)
    f = syn.random_complex(n, seed=9)
    ref = tg.twogrid_step(u0, f)
    u = to_dev(u0[None])
    s.twogrid(u, to_dev(f[None]))
    assert rel(to_np(u)[0], ref) < 1e-11
    s.close()


def test_solve_c1_slab_same_iterations():
    cfg = syn.config("C1")
    p, N = cfg["p"], cfg["n"]
    f = syn.gaussian_load(N, p, cfg["centres"], cfg["sigma"])
    tg = TwoGrid(p, cfg["k"], alpha_s=cfg["alpha_s"], l_dd=cfg["l_dd"])
    x_ref, it_ref, _ = tg.gmres(f[0], 1e-6)
    s = solver(cfg["k"], p, cfg["l_dd"], alpha_s=cfg["alpha_s"], max_rhs=1)
    u, st = s.solve(to_dev(f))
    print(f"C1 slab: oracle iters {it_ref}, gpu iters {st.iters}", flush=True)
    assert st.status == 0 and st.iters == it_ref and st.rel_res <= 1e-6
    assert rel(to_np(u)[0], x_ref) < 1e-10
    s.close()


def test_slab_layout_rejected_where_unsupported():
    from paper_2509_17494_amd import THError, TwoGridSolver, _lib as L
    k = np.full((8, 8), 8.0)
    with pytest.raises(THError) as e:
        TwoGridSolver(k, order=2, l_dd=4, gemm="bf16", layout="slab")
    assert e.value.status == L.TH_EINVAL
