"""GPU parity at the full C2 size (Q4, 200 x 200 cells, 641,601 DOF, 169
subdomains, the launch configuration bench.py times), on sampled outputs.

The expected values were written by tests/golden/make_c2_samples.py, which
calls only the FP64 oracle: every step of the path at 256 sampled fine nodes
(and 256 coarse vertices) for seeded random inputs, and the full GMRES solve
of the C2 load (iteration count and sampled solution).  Bars, relative to the
largest entry of the oracle's full output vector: 1e-12 for single fine
operator applications, 1e-13 for the restriction, 1e-11 for the coarse solve
and the two-grid step, 1e-10 for the solution after the same iteration count.
"""
import json
import os

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c2_samples.json")


def load_gold():
    d = json.load(open(GOLD))
    c = lambda v: np.array([a + 1j * b for a, b in v])
    for key in ("residual", "smooth", "restrict", "coarse_solve", "twogrid"):
        d[key] = c(d[key])
    d["solve"]["x"] = c(d["solve"]["x"])
    return d


@pytest.fixture(scope="module")
def c2():
    from paper_2509_17494_amd import TwoGridSolver
    cfg = syn.config("C2")
    print("case C2 full size: setup", flush=True)
    s = TwoGridSolver(cfg["k"], order=cfg["p"], alpha_s=cfg["alpha_s"], l_dd=cfg["l_dd"],
                      max_rhs=1)
    yield cfg, s, load_gold()
    s.close()
    torch.cuda.synchronize()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)[None]).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()[0]


def check(name, got, gold, tol):
    err = np.max(np.abs(got - gold[name])) / gold["norms_inf"][name]
    print(f"  {name}: max sampled error / max entry = {err:.2e}", flush=True)
    assert err < tol


def test_c2_steps_at_sampled_nodes(c2):
    cfg, s, g = c2
    n, nc = s.n_fine, s.n_coarse
    u = syn.random_complex(n, g["seeds"]["u"])
    f = syn.random_complex(n, g["seeds"]["f"])
    rc = syn.random_complex(nc, g["seeds"]["rc"])
    idx, idc = np.array(g["idx"]), np.array(g["idc"])
    ud, fd = dev(u), dev(f)
    r = host(s.residual(ud, fd))
    check("residual", r[idx], g, 1e-12)
    rcv = host(s.restrict(dev(r)))
    check("restrict", rcv[idc], g, 1e-13)
    sm = dev(u)
    s.smooth(sm, fd)
    check("smooth", host(sm)[idx], g, 1e-12)
    check("coarse_solve", host(s.coarse_solve(dev(rc)))[idc], g, 1e-11)
    tw = dev(u)
    s.twogrid(tw, fd)
    check("twogrid", host(tw)[idx], g, 1e-11)


def test_c2_solve_same_iterations_and_sampled_solution(c2):
    cfg, s, g = c2
    f = syn.gaussian_load(cfg["n"], cfg["p"], cfg["centres"], cfg["sigma"])
    u, st = s.solve(torch.from_numpy(f).to("cuda"), rtol=g["solve"]["rtol"])
    x = u.cpu().numpy()[0]
    err = np.max(np.abs(x[np.array(g["idx"])] - g["solve"]["x"])) / g["solve"]["x_norm_inf"]
    print(f"C2 full size: iters {st.iters} (oracle {g['solve']['iters']}), rel res {st.rel_res:.2e}, "
          f"sampled solution error {err:.2e}", flush=True)
    assert st.status == 0 and st.iters == g["solve"]["iters"]
    assert st.rel_res <= 1e-6
    assert err < 1e-10
