"""Write tests/golden/c2_samples.json: outputs of the FP64 oracle on the full
C2 workload (Q4, 200 x 200 cells, 641,601 DOF) at sampled nodes, for the
full-size GPU parity test.  Calls only oracle/ and synthetic/ (about five
minutes on one core).

Usage: python tests/golden/make_c2_samples.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthetic as syn  # noqa: E402
from oracle.transfer import restriction  # noqa: E402
from oracle.twogrid import TwoGrid  # noqa: E402

SEED_U, SEED_F, SEED_RC, SEED_IDX = 101, 102, 103, 104
N_SAMPLES = 256


def cplx(z):
    return [[float(v.real), float(v.imag)] for v in np.asarray(z)]


def main():
    cfg = syn.config("C2")
    p, N = cfg["p"], cfg["n"]
    t0 = time.time()
    tg = TwoGrid(p, cfg["k"], alpha_s=cfg["alpha_s"], l_dd=cfg["l_dd"])
    print(f"oracle setup {time.time() - t0:.1f} s", flush=True)
    n = tg.A.shape[0]
    nc = tg.A_c.shape[0]
    rng = np.random.Generator(np.random.PCG64(SEED_IDX))
    idx = np.sort(rng.choice(n, N_SAMPLES, replace=False))
    idc = np.sort(rng.choice(nc, N_SAMPLES, replace=False))
    u = syn.random_complex(n, SEED_U)
    f = syn.random_complex(n, SEED_F)
    rc = syn.random_complex(nc, SEED_RC)
    r = tg.residual(u, f)
    sm = tg.smooth(u, f)
    rr = restriction(N, p) @ r
    uc = tg.coarse_solve(rc)
    two = tg.twogrid_step(u, f)
    load = syn.gaussian_load(N, p, cfg["centres"], cfg["sigma"])[0]
    t0 = time.time()
    x, iters, hist = tg.gmres(load, 1e-6)
    print(f"oracle GMRES {iters} iterations, {time.time() - t0:.1f} s", flush=True)
    out = {
        "description": "FP64 oracle on the C2 workload at sampled nodes; random vectors are "
                       "synthetic.random_complex(n, seed)",
        "seeds": {"u": SEED_U, "f": SEED_F, "rc": SEED_RC},
        "idx": idx.tolist(), "idc": idc.tolist(),
        "residual": cplx(r[idx]), "smooth": cplx(sm[idx]), "restrict": cplx(rr[idc]),
        "coarse_solve": cplx(uc[idc]), "twogrid": cplx(two[idx]),
        "solve": {"rtol": 1e-6, "iters": int(iters), "x": cplx(x[idx]),
                  "x_norm_inf": float(np.max(np.abs(x)))},
        "norms_inf": {"residual": float(np.max(np.abs(r))), "smooth": float(np.max(np.abs(sm))),
                      "restrict": float(np.max(np.abs(rr))),
                      "coarse_solve": float(np.max(np.abs(uc))),
                      "twogrid": float(np.max(np.abs(two)))},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_samples.json")
    json.dump(out, open(path, "w"))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
