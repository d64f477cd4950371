#!/usr/bin/env python3
"""Benchmark of the two-grid Helmholtz solve on one MI355X.

A step is one complete solve A u = f to a relative residual of 1e-6 (GMRES
with the two-grid preconditioner: fine residuals, CSDD smoothing, restriction,
coarse solve, prolongation, orthogonalisation) on the default workload:

  C2: 2-D unit square, Q4, 200 x 200 cells (801^2 = 641,601 DOF), seeded
      Gaussian-random-field speed (l = 0.05, 1.5..4.0) with 80 wavelengths at
      the slowest speed (10 DOF per wavelength there), absorbing boundary, one
      Gaussian source (sigma = 2h) at the centre, 16x16-cell subdomains,
      alpha_s = 0.5, complex128 two-grid preconditioner under FP64 GMRES.

value = fine DOF x two-grid cycles / second (setup excluded), summed over the
right-hand sides; ms_per_step is the time to the 1e-6 residual.  Inputs are in
HBM before the timed region starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0   # dense matrix cores
FP64_PEAK_TFLOPS = 78.6     # matrix and vector
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def sources_sha256(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3", "C4", "C5"])
    ap.add_argument("--precond", default=None, choices=["c128", "c64"])
    ap.add_argument("--alpha-s", type=float, default=None,
                    help="smoother shift alpha_s (default: the workload's, 0.5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="leave the 3-D C4 variant out")
    ap.add_argument("--no-graph", action="store_true",
                    help="no HIP-graph replay of the preconditioner (profiling runs)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--study", default=None, choices=["table1"],
                    help="instead of the benchmark, print the iteration counts of a parameter "
                         "study (table1: the two-grid parameters of Table 1)")
    return ap.parse_args()


def workload(name):
    import synthetic as syn
    cfg = syn.config(name)
    spec = dict(l_dd=cfg["l_dd"], alpha_s=cfg["alpha_s"], gemm="f64", precond="c128",
                coarse="qsfem")
    if name == "C3":
        spec.update(gemm="bf16", precond="c64")
    if name == "C4":  # FP32 slab factors, complex64 preconditioner, dispersion-matched 27-point
        spec.update(gemm="f32", precond="c64", coarse="plainfit", restart=30)
    return cfg, spec


def dd_apply_bytes(info_sub, nrhs, mat_bytes, vec_bytes, symmetric=False):
    """Algorithmic bytes of one batched subdomain apply: every stored B_i entry
    once (with the symmetric layout the U x U block counts n_U (n_U + 1) / 2
    entries), the gathered patch X_i and the output rows Y_i once per
    right-hand side."""
    if symmetric:
        b = sum(nu * (nu + 1) // 2 + nu * (no - nu) for nu, no in info_sub) * mat_bytes
    else:
        b = sum(nu * no for nu, no in info_sub) * mat_bytes
    v = sum(no + nu for nu, no in info_sub) * vec_bytes * nrhs
    return b + v


def subdomain_sizes(N, p, l_dd, dim=2):
    """(n_U, n_Omega) of every subdomain: balanced blocks of about l_dd cells,
    Omega = U grown by one cell layer clipped to the domain."""
    import itertools
    import math
    M = math.ceil(N / l_dd)
    base, rem = divmod(N, M)
    sizes = [base + 1] * rem + [base] * (M - rem)
    starts = [0]
    for s in sizes:
        starts.append(starts[-1] + s)
    nu1 = [sizes[b] * p + 1 for b in range(M)]
    no1 = [(min(starts[b + 1] + 1, N) - max(starts[b] - 1, 0)) * p + 1 for b in range(M)]
    out = []
    for idx in itertools.product(range(M), repeat=dim):
        out.append((math.prod(nu1[b] for b in idx), math.prod(no1[b] for b in idx)))
    return out


def slab_apply_bytes(N, p, l_dd, dim, nrhs, mat_bytes, vec_bytes, packed=False):
    """Algorithmic bytes and flops of one application in the slab-factor
    layout with the twisted elimination (middle slab M = (nsl - 1) // 2):
    every G_t read by the forward sweep (whole, or with packed storage its
    m (m + 1) / 2 distinct entries, G_t being symmetric); the backward sweep reads E_t
    (rows of slab t x first layer of t + 1) for the lower slabs t < M and the
    first-layer rows of G_t for the upper slabs t > M; the coupling bands of
    slabs 1 .. nsl - 1 once in the forward sweep and those of the upper slabs
    again in the backward one; the patch X_i and the output rows Y_i once per
    right-hand side."""
    import itertools
    import math
    M = math.ceil(N / l_dd)
    base, rem = divmod(N, M)
    sizes = [base + 1] * rem + [base] * (M - rem)
    starts = [0]
    for x in sizes:
        starts.append(starts[-1] + x)
    ocells = [min(starts[b + 1] + 1, N) - max(starts[b] - 1, 0) for b in range(M)]
    cb = ((2 * p + 1) ** (dim - 1)) * p
    g_entries, band_entries, vec, mul_entries = 0, 0, 0, 0
    for idx in itertools.product(range(M), repeat=dim):
        no = [ocells[b] * p + 1 for b in idx]      # x first
        nu = [sizes[b] * p + 1 for b in idx]
        nsl, lsz = ocells[idx[-1]], math.prod(no[:-1])
        m, ml = p * lsz, (p + 1) * lsz
        mid = (nsl - 1) // 2
        nup = nsl - 1 - mid
        full = (nsl - 1) * m * m + ml * ml                   # G_t, forward
        g_entries += (nsl - 1) * m * (m + 1) // 2 + ml * (ml + 1) // 2 if packed else full
        mul_entries += full - ((nsl - 1) * m * (m + 1) // 2 + ml * (ml + 1) // 2 if packed else full)
        g_entries += mid * m * lsz                           # E_t, lower chain
        g_entries += (nup - 1) * m * lsz + ml * lsz if nup else 0  # G_t rows, upper chain
        band_entries += (nsl - 1 + nup) * lsz * cb
        vec += math.prod(no) + math.prod(nu)
    byts = (g_entries + band_entries) * mat_bytes + vec * vec_bytes * nrhs
    # flops: every entry of every G_t multiplies once (a stored off-diagonal
    # entry of a packed G_t twice)
    return byts, 8.0 * (g_entries + mul_entries + band_entries) * nrhs


def traffic_cfg(key):
    """The matrix-core smoother configuration a counter entry was taken with
    (None when the entry names none)."""
    try:
        return json.load(open(TRAFFIC_FILE)).get(key, {}).get("smoother_cfg")
    except Exception:
        return None


def traffic_entry(key):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE counter runs scaled by
    a device copy of known size) from the committed summary, or None when the
    kernel sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        e = json.load(open(TRAFFIC_FILE)).get(key)
        if not e or e.get("kernel_sha256") != sources_sha256(e["sources"]):
            return None
        return e.get("hbm_bytes_per_launch", e.get("hbm_bytes_per_solve"))
    except Exception:
        return None


def host_description():
    """The host the oracle runs on: usable cores and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "logical_cpus": os.cpu_count(), "cpu_model": model}


def timed_oracle_solves(tg, f, threads, min_seconds=8.0):
    """Repeat the oracle's GMRES solve for about min_seconds of CPU work with
    the BLAS thread pools limited to `threads` (the sparse LU solves of the
    coarse level are serial either way)."""
    from threadpoolctl import threadpool_limits
    its = reps = 0
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        while True:
            _, k, _ = tg.gmres(f, 1e-6)
            its += k
            reps += 1
            if time.perf_counter() - t0 >= min_seconds:
                break
        t = time.perf_counter() - t0
    return its, t, reps


def _baseline(tg, f, ndof, t_setup, what):
    host = host_description()
    runs = {}
    for threads in (1, host["nproc"]):
        its, t, reps = timed_oracle_solves(tg, f, threads)
        runs[threads] = (ndof * its / t, its, t, reps)
    best = max(runs, key=lambda k: runs[k][0])
    v, its, t, reps = runs[best]
    return {"value": v, "unit": "DOF*cycles/s", "cores": best, "kind": "oracle",
            "sample": f"{what}: oracle GMRES to 1e-6 repeated {reps} times, {its} cycles in "
                      f"{t:.2f} s with {best} BLAS thread(s) (setup {t_setup:.1f} s excluded); "
                      f"numpy/scipy FP64",
            "single_thread_value": runs[1][0], "all_cores_value": runs[host["nproc"]][0],
            "host": host}


def cpu_baseline_3d():
    """The oracle on the reduced 3-D cube: C4's recipe (GRF correlation 0.1,
    speeds 1.5..4, 10 points per minimum wavelength, Q2, 8-cell subdomains,
    8 sources at {1/4, 3/4}^3) on 16^3 cells, one source, solved to 1e-6."""
    import synthetic as syn
    from oracle.twogrid import TwoGrid
    n, p = 16, 2
    k = syn.wavenumber_from_speed(syn.grf_speed(n, 3, 0.1, 1.5, 4.0, seed=0), n * p / 10.0)
    t0 = time.perf_counter()
    tg = TwoGrid(p, k, alpha_s=0.5, l_dd=8)
    t_setup = time.perf_counter() - t0
    f = syn.gaussian_load(n, p, [[0.25, 0.25, 0.25]], 2.0 / n, dim=3)[0]
    ndof = (n * p + 1) ** 3
    return _baseline(tg, f, ndof, t_setup,
                     f"C4 recipe on a 16^3-cell cube ({ndof} DOF), Q2, l_dd=8, one source, "
                     f"exact-wavenumber 27-point coarse stencil")


def cpu_baseline(cfg_name):
    """The FP64 oracle timed on this host on a bounded sample: a 96x96-cell
    window of the same medium, order and k h with the same subdomain size,
    solved to 1e-6 by the oracle's GMRES; rate = DOF x cycles / solve time,
    with one BLAS thread and with all usable cores (the faster is the value)."""
    if cfg_name == "C4":
        return cpu_baseline_3d()
    import numpy as np
    import synthetic as syn
    from oracle.twogrid import TwoGrid
    cfg = syn.config(cfg_name)
    n = min(96, cfg["n"])
    # a physical window of side n/N keeps k h (DOF per wavelength) of the workload
    k = np.ascontiguousarray(cfg["k"][:n, :n]) * (n / cfg["n"])
    p = cfg["p"]
    t0 = time.perf_counter()
    tg = TwoGrid(p, k, alpha_s=cfg["alpha_s"], l_dd=cfg["l_dd"])
    t_setup = time.perf_counter() - t0
    f = syn.gaussian_load(n, p, [[0.5, 0.5]], 2.0 / n)[0]
    ndof = (n * p + 1) ** 2
    return _baseline(tg, f, ndof, t_setup,
                     f"{cfg_name} medium, order and k*h on a {n}x{n}-cell window ({ndof} DOF), "
                     f"l_dd={cfg['l_dd']}")


def run_workload(name, steps, warmup, precond=None, graph=False, timing=True, verbose=False,
                 gemm=None, alpha_s=None, coarse=None, coarse_q=None):
    """Set up one workload, then time `steps` solves to 1e-6 after `warmup`
    untimed ones.  With timing, HIP events record every kernel class over the
    timed region (graph replay is off then); without it a separate one-solve
    timing pass follows the timed region."""
    import torch
    import synthetic as syn
    from paper_2509_17494_amd import TwoGridSolver

    cfg, spec = workload(name)
    precond = precond or spec["precond"]
    kry = {k: spec[k] for k in ("restart", "maxit") if k in spec}
    if gemm:
        spec["gemm"] = gemm
    if alpha_s is not None:
        spec["alpha_s"] = alpha_s
    if coarse is not None:
        spec["coarse"] = coarse
    N, p, dim = cfg["n"], cfg["p"], cfg.get("dim", 2)
    f_host = syn.gaussian_load(N, p, cfg["centres"], cfg["sigma"], dim=dim)
    R = f_host.shape[0]
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        s = TwoGridSolver(cfg["k"], order=p, alpha_s=spec["alpha_s"], l_dd=spec["l_dd"],
                          gemm=spec["gemm"], max_rhs=R, coarse=spec["coarse"], coarse_q=coarse_q)
        t_setup = time.perf_counter() - t0
        info = s.info()
        f = torch.from_numpy(f_host).to("cuda")
        u = torch.empty_like(f)
        if verbose:
            print(f"{name}: setup {t_setup:.2f} s (fine {info['t_setup_fine_s']:.2f}, coarse "
                  f"{info['t_setup_coarse_s']:.2f}); B {info['b_bytes'] / 1e9:.3f} GB",
                  flush=True)
        for _ in range(warmup):
            s.solve(f, u, precond=precond, graph=graph, **kry)
        torch.cuda.synchronize()
        if timing:
            s.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cycles, iters, worst = 0, [], 0.0
        for _ in range(steps):
            _, st = s.solve(f, u, precond=precond, graph=graph, **kry)
            cycles += st.n_precond
            iters.append(st.iters)
            worst = max(worst, st.rel_res)
            if st.status != 0:
                raise RuntimeError(f"{name}: solve did not converge: {st}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if not timing:
            s.timing(True)
            s.solve(f, u, precond=precond, graph=False, **kry)
            torch.cuda.synchronize()
        kt = s.kernel_times()
        s.timing(False)
        ksteps = steps if timing else 1
    elapsed = t1 - t0
    mat_bytes = {"f64": 16, "f32": 8, "bf16": 4}[spec["gemm"]]
    vec_bytes = 16 if precond == "c128" else 8
    subs = subdomain_sizes(N, p, spec["l_dd"], dim)
    sym = info["smoother_layout"] == 1
    alg = dd_apply_bytes(subs, R, mat_bytes, vec_bytes, symmetric=sym)
    flops = 8.0 * sum(nu * no for nu, no in subs) * R
    if info["smoother_layout"] == 3:
        alg, flops = slab_apply_bytes(N, p, spec["l_dd"], dim, R, mat_bytes, vec_bytes,
                                      packed=bool(info["slab_packed"]))
    dd_ms, dd_n = kt["dd_apply"]
    avg_ms = dd_ms / max(dd_n, 1)
    # coarse solve: one per two-grid cycle; bytes streamed per solve by the
    # nested dissection (factors once per solve and refinement step, the
    # refinement residual reads the stencil) or the line elimination (its
    # factors once per pass of right-hand sides)
    c_ms, _ = kt["coarse"]
    c_avg = c_ms / max(sum(iters) if timing else iters[-1], 1)  # one coarse solve per iteration
    S = 27 if dim == 3 else 9
    st_bytes = info["n_coarse"] * S * 16
    refine = info["coarse_refine"] if precond == "c128" else 0
    if info["coarse_solver"] == 2:
        c_bytes = (info["coarse_bytes"] - st_bytes) * (1 + refine) + refine * st_bytes
    else:
        c_bytes = info["coarse_bytes"]
    res = {
        "name": name, "precond": precond, "gemm": spec["gemm"], "graph": graph, "R": R,
        "n_fine": info["n_fine"], "value": info["n_fine"] * cycles / elapsed,
        "ms_per_step": elapsed / steps * 1e3, "gmres_iters": iters[-1], "max_rel_res": worst,
        "setup_s": t_setup, "info": info,
        "kernel_ms_per_step": {k: round(v[0] / ksteps, 4) for k, v in kt.items()},
        "layout": ["dense", "symmetric", "matrix-core", "slab"][info["smoother_layout"]],
        "dd": {"alg_bytes": alg, "flops": flops, "avg_ms": avg_ms, "launches": dd_n,
               "gbs": alg / (avg_ms * 1e-3) / 1e9, "tflops": flops / (avg_ms * 1e-3) / 1e12},
        "coarse": {"solver": {1: "lines", 2: "nested dissection"}[info["coarse_solver"]],
                   "levels": info["coarse_levels"], "refine_steps": refine,
                   "probe_error": info["coarse_check_pc"] if precond == "c128" else None,
                   "factor_bytes": info["coarse_bytes"],
                   "bytes_per_solve": c_bytes, "avg_ms_per_solve": round(c_avg, 4),
                   "gbs": c_bytes / max(c_avg * 1e-3, 1e-12) / 1e9},
        "desc": f"{name}: {dim}-D Q{p}, {N}^{dim} cells ({info['n_fine']} DOF), {R} RHS, "
                f"l_dd={spec['l_dd']}, alpha_s={spec['alpha_s']}, B_i {spec['gemm']}, "
                f"preconditioner {precond}, coarse {spec['coarse']}"
                + (", HIP-graph replay" if graph else ""),
    }
    del s
    torch.cuda.synchronize()
    return res


def study_table1(wavelengths=16.0, rtol=1e-6):
    """GMRES iteration counts of the two-grid method for the parameter grid of
    Table 1: constant k on the unit square, absorbing boundary on all sides,
    a Gaussian source (sigma = 2h) off the centre, QSFEM coarse level.  The
    paper states neither domain size nor tolerance: about 16 wavelengths
    across the domain and a 1e-6 relative residual are used.  Prints one JSON
    line per part."""
    import math

    import numpy as np
    import torch

    import synthetic as syn
    from paper_2509_17494_amd import TwoGridSolver

    def iters(p, ppw, **kw):
        N = max(2, round(ppw * wavelengths / p))
        k = np.full((N, N), 2.0 * math.pi * p * N / ppw)  # ppw DOFs per wavelength
        f = syn.gaussian_load(N, p, [[0.41, 0.57]], 2.0 / N)
        s = TwoGridSolver(k, order=p, max_rhs=1, **kw)
        _, st = s.solve(torch.from_numpy(f).to("cuda"), rtol=rtol, maxit=400)
        s.close()
        return st.iters if st.status == 0 else None

    part_a = {}
    for p, ppw in ((4, 10), (6, 8)):
        for l_dd in (4, 6):
            for n_dd in (1, 2):
                row = [iters(p, ppw, alpha_s=a, l_dd=l_dd, n_dd=n_dd)
                       for a in (0.1, 0.15, 0.2, 0.3, 0.4)]
                part_a[f"p={p} ppw={ppw} subdomsize={l_dd} n_dd={n_dd}"] = row
                print(f"table1a p={p} l_dd={l_dd} n_dd={n_dd}: {row}", file=sys.stderr,
                      flush=True)
    print(json.dumps({"study": "table1a", "columns": "alpha_s = 0.1, 0.15, 0.2, 0.3, 0.4",
                      "wavelengths": wavelengths, "rtol": rtol, "iters": part_a}), flush=True)
    part_b = {}
    for n_s in (1, 2):
        for om in (1.0, 0.8, 0.6):
            row = {}
            for p, ppws in ((4, (8, 10, 14)), (6, (6, 8, 10, 14))):
                for ppw in ppws:
                    row[f"p={p} ppw={ppw}"] = iters(p, ppw, alpha_s=0.2, l_dd=4, n_s=n_s,
                                                    omega_c=om)
            part_b[f"n_s={n_s} omega_c={om}"] = row
            print(f"table1b n_s={n_s} omega_c={om}: {list(row.values())}", file=sys.stderr,
                  flush=True)
    print(json.dumps({"study": "table1b", "alpha_s": 0.2, "subdomsize": 4,
                      "wavelengths": wavelengths, "rtol": rtol, "iters": part_b}), flush=True)


def roofline_hbm(v, kernel, mfma_peak=None, traffic_key=None):
    """Roofline object of a variant's smoother application (HBM bound):
    algorithmic bytes per launch over the average launch time from HIP
    events; with mfma_peak, the matrix-core rate of the same launch too."""
    d = v["dd"]
    r = {"bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(d["gbs"] / HBM_PEAK_GBS, 4),
         "traffic": traffic_entry(traffic_key) if traffic_key else None, "kernel": kernel,
         "alg_bytes_per_launch": d["alg_bytes"], "avg_launch_ms": round(d["avg_ms"], 4),
         "launches": d["launches"]}
    if mfma_peak:
        r["mfma_TFLOPs"] = round(d["tflops"], 2)
        r["mfma_frac"] = round(d["tflops"] / mfma_peak, 4)
    return r


def mfma_kernel_name(cfg):
    """The BF16 matrix-core smoother form of an autotuner configuration."""
    if cfg < 5:
        return f"k_dd_mfma (persistent, configuration {cfg}; BF16 B_i, FP32 accumulation)"
    if cfg < 12:
        return f"k_dd_mfx (staged patch in LDS, configuration {cfg}; BF16 B_i, FP32 accumulation)"
    return (f"k_mfp_gather + k_mfp_gemm (two-pass, configuration {cfg}; BF16 B_i, FP32 "
            f"accumulation)")


def roofline_fp64(v):
    """The FP64 batched smoother is a dense complex GEMM (arithmetic intensity
    above the FP64 ridge of 9.8 flop/B): bound by the FP64 matrix cores."""
    d = v["dd"]
    return {"bound": "mfma", "achieved": round(d["tflops"], 2), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(d["tflops"] / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": "k_dd_gatherx + k_dd_mfma64 (FP64 matrix cores, v_mfma_f64_16x16x4f64)",
            "flops_per_launch": d["flops"], "avg_launch_ms": round(d["avg_ms"], 4),
            "launches": d["launches"]}


def coarse_roofline(v, traffic_key=None):
    c = v["coarse"]
    return {"bound": "hbm", "achieved": round(c["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(c["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic_entry(traffic_key) if traffic_key else None,
            "kernel": "coarse solve (" + c["solver"] + ")",
            "alg_bytes_per_solve": c["bytes_per_solve"], "avg_ms_per_solve": c["avg_ms_per_solve"]}


def variant_entry(v, roof):
    return {"workload": v["desc"], "value": v["value"], "unit": "DOF*cycles/s",
            "time_to_1e-6_ms": v["ms_per_step"], "gmres_iters": v["gmres_iters"],
            "max_rel_res": v["max_rel_res"], "setup_s": round(v["setup_s"], 3),
            "kernel_ms_per_step": v["kernel_ms_per_step"], "coarse": v["coarse"],
            "roofline": roof}


def c5_variant(steps, verbose):
    """C5: the surrogate network trained on the device (1e5 seeded samples of
    the plain fit, 30 epochs), then the C5 solve with per-cell network
    stencils (fallback threshold 1e-3 on the zero-set mismatch) against the
    plain fit computed per cell on the host."""
    import synthetic as syn
    from paper_2509_17494_amd import CoarseStencilMLP
    t0 = time.perf_counter()
    net = CoarseStencilMLP(syn.mlp_init(seed=2))
    st = net.train(syn.mlp_samples(100_000, seed=1), epochs=30, batch=1024, lr=2e-3, bf16=True)
    t_train = time.perf_counter() - t0
    out = {"training": {"samples": 100000, "epochs": 30, "steps": st.steps,
                        "loss_first": st.loss_first, "loss_last": st.loss_last,
                        "t_targets_s": round(st.t_targets_s, 3),
                        "t_device_train_s": round(st.t_train_s, 3), "t_total_s": round(t_train, 3)}}
    for key, coarse, q in (("plainfit", "plainfit", None), ("mlp", "mlp", (net, 1e-3))):
        v = run_workload("C5", steps, 1, graph=False, timing=True, verbose=verbose,
                         coarse=coarse, coarse_q=q)
        out[key] = {"workload": v["desc"], "value": v["value"], "unit": "DOF*cycles/s",
                    "time_to_1e-6_ms": v["ms_per_step"], "gmres_iters": v["gmres_iters"],
                    "max_rel_res": v["max_rel_res"],
                    "stencil_time_ms": round(v["info"]["t_stencil_s"] * 1e3, 3),
                    "fallback_cells": v["info"]["n_fallback_cells"],
                    "coarse_setup_s": round(v["info"]["t_setup_coarse_s"], 3)}
    net.close()
    return out


def main():
    a = parse()
    if a.verbose:
        os.environ.setdefault("TH_PROGRESS", "1")  # library progress lines during long setups
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if a.study == "table1":
        study_table1()
        return
    mixed = a.workload in ("C3", "C4")
    prim = run_workload(a.workload, a.steps, a.warmup, precond=a.precond,
                        graph=mixed and not a.no_graph, timing=not mixed, verbose=a.verbose,
                        alpha_s=a.alpha_s)
    d = prim["dd"]
    traffic = traffic_entry(a.workload)
    roof = {"bound": "hbm", "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": {"dense": "k_dd_apply", "symmetric": "k_dd_sym + k_dd_symred",
                       "matrix-core": "k_dd_mfma",
                       "slab": ("k_slab_gather + k_slab_fwd_chain + k_slab_fwd_pk (middles) + "
                                "k_slab_bwd_chain + k_slab_extract (one smoother application, "
                                "packed G_t)" if prim["info"]["slab_packed"] else
                                "k_slab_gather + k_slab_fwd + k_slab_bwd + k_slab_extract "
                                "(one smoother application)")}[prim["layout"]],
            "alg_bytes_per_launch": d["alg_bytes"], "avg_launch_ms": round(d["avg_ms"], 4),
            "launches": d["launches"]}
    info = prim["info"]
    out = {
        "metric": "fine DOF*cycles/s and time-to-1e-6 residual, mixed+batched vs FP64, 1 GPU",
        "value": prim["value"],
        "unit": "DOF*cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prim["precond"] == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": prim["desc"],
                   "time_to_1e-6_ms": prim["ms_per_step"], "gmres_iters": prim["gmres_iters"],
                   "max_rel_res": prim["max_rel_res"], "setup_s": round(prim["setup_s"], 3),
                   "setup_fine_s": round(info["t_setup_fine_s"], 3),
                   "setup_coarse_s": round(info["t_setup_coarse_s"], 3),
                   "b_bytes": info["b_bytes"], "coarse_bytes": info["coarse_bytes"],
                   "coarse_lines_per_block": info["coarse_lines"],
                   "kernel_ms_per_step": prim["kernel_ms_per_step"]},
        "roofline": roof,
    }
    out["config"]["coarse"] = prim["coarse"]
    out["coarse_roofline"] = coarse_roofline(
        prim, traffic_key="C2_coarse" if a.workload == "C2" and prim["coarse"]["solver"] ==
        "nested dissection" else None)
    if not a.no_variants and a.workload == "C2":
        variants = {}
        v_mixed = run_workload("C3", max(3, a.steps), 1, graph=True, timing=False,
                               verbose=a.verbose)
        variants["C3_mixed_bf16_batched64_graph"] = variant_entry(
            v_mixed, roofline_hbm(v_mixed, mfma_kernel_name(v_mixed["info"]["smoother_cfg"]),
                                  mfma_peak=BF16_PEAK_TFLOPS,
                                  traffic_key=next((k for k in ("C3", "C3_cfg12")
                                                    if traffic_cfg(k) ==
                                                    v_mixed["info"]["smoother_cfg"]), None)))
        v_fp64 = run_workload("C3", max(3, a.steps), 1, precond="c128", gemm="f64", graph=False,
                              timing=True, verbose=a.verbose)
        variants["C3_fp64_batched64_control"] = variant_entry(v_fp64, roofline_fp64(v_fp64))
        variants["C3_mixed_vs_fp64"] = {
            "value_ratio": v_mixed["value"] / v_fp64["value"],
            "time_ratio": v_fp64["ms_per_step"] / v_mixed["ms_per_step"],
            "note": "the same 64 sources; FP64 control runs its subdomain GEMMs on the FP64 "
                    "matrix cores"}
        v1 = run_workload("C1", max(3, a.steps), 1, graph=False, timing=True, verbose=a.verbose)
        variants["C1_fp64"] = variant_entry(v1, roofline_hbm(v1, "k_dd_apply (dense rows)"))
        variants["C5_learned_stencils"] = c5_variant(max(3, a.steps), a.verbose)
        if not a.no_c4:
            v4 = run_workload("C4", 2, 1, graph=True, timing=False, verbose=a.verbose)
            variants["C4_3d_mixed_f32slab_8rhs_graph"] = variant_entry(
                v4, roofline_hbm(v4, "k_slab_gather + k_slab_fwd + k_slab_bwd + k_slab_extract "
                                     "(one smoother application, FP32 slab factors)"))
        out["config"]["variants"] = variants
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline("C2" if a.workload == "C2" else a.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
