"""MI355X two-grid solver for finite-element Helmholtz problems.

Thin Python binding over the C ABI of libth.so (include/th.h): it checks
shapes, dtypes and devices of torch tensors on the host and passes raw device
pointers and the current HIP stream.  Every step of the method runs in the
library's HIP kernels; there is no Python or CPU fallback, and importing the
binding without the built library raises ImportError.

Method: Stolk, "A two-grid method with dispersion matching for finite-element
Helmholtz problems" (arXiv 2509.17494): Q_p Galerkin fine level (Sec. 3.1),
complex-shifted DD smoother (Alg. 2), QSFEM coarse level (Sec. 3.2-3.3),
Q_{p/2} interpolation (Sec. 4.2), two-grid step (Alg. 1) inside FP64 GMRES.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

__all__ = ["TwoGridSolver", "THError", "SolveStats", "load_library", "CoarseStencilMLP", "plain_fit",
           "plain_fit3d"]


class THError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


@dataclass
class SolveStats:
    iters: int
    rel_res: float
    t_solve_s: float
    n_precond: int
    status: int
    t_cycle_s: float = 0.0
    n_fallback_cells: int = 0


def load_library():
    return L.load()


_BC = {"robin": L.TH_BC_ROBIN, "neumann": L.TH_BC_NEUMANN, "dirichlet": L.TH_BC_DIRICHLET}
_GEMM = {"f64": L.TH_GEMM_F64, "f32": L.TH_GEMM_F32, "bf16": L.TH_GEMM_BF16}
_CSOLVE = {None: L.TH_CSOLVE_AUTO, "auto": L.TH_CSOLVE_AUTO, "lines": L.TH_CSOLVE_LINES,
           "nd": L.TH_CSOLVE_ND}
_LAYOUT = {None: L.TH_LAYOUT_AUTO, "auto": L.TH_LAYOUT_AUTO, "dense": L.TH_LAYOUT_DENSE,
           "symmetric": L.TH_LAYOUT_SYMMETRIC, "slab": L.TH_LAYOUT_SLAB}
LAYOUT_NAMES = {0: "dense", 1: "symmetric", 2: "matrix-core", 3: "slab"}


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.complex128:
        return L.TH_C128
    if t.dtype == torch.complex64:
        return L.TH_C64
    raise TypeError(f"vectors must be complex128 or complex64, got {t.dtype}")


class TwoGridSolver:
    """One fine problem (unit square or cube, N^d cells, order p) on one GPU.

    k, eps: per-cell arrays of shape (N, N) indexed [y][x], or (N, N, N)
    indexed [z][y][x] (host, float64); bc lists the sides x-, x+, y-, y+(, z-, z+),
    each "robin" (absorbing), "neumann" or "dirichlet".  layout: storage of the
    FP64/FP32 subdomain solves ("dense", "symmetric", "slab"; None = automatic).
    Vectors are torch tensors on the solver's device of shape (nrhs, ndof)
    (or (ndof,) for one right-hand side), complex128 or complex64, contiguous.
    """

    def __init__(self, k, eps=None, order: int = 2, alpha_s: float = 0.5, l_dd: int = 8,
                 n_dd: int = 1, n_s: int = 1, omega_c: float = 1.0, bc=None,
                 gemm: str = "f64", max_rhs: int = 1, device: int | None = None,
                 coarse: str | None = "qsfem", coarse_q=None, layout: str | None = None,
                 coarse_solver: str | None = None):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64))
        if k.ndim not in (2, 3) or len(set(k.shape)) != 1:
            raise ValueError("k must have shape (N, N) or (N, N, N)")
        self.N = k.shape[0]
        self.p = int(order)
        self.dim = k.ndim
        self.n1 = self.N * self.p + 1
        self.nc1 = self.N * (self.p // 2) + 1
        self.n_fine = self.n1 ** self.dim
        self.n_coarse = self.nc1 ** self.dim
        if bc is None:
            bc = ("robin",) * (2 * self.dim)
        if len(bc) != 2 * self.dim:
            raise ValueError(f"bc needs {2 * self.dim} entries")
        self.max_rhs = int(max_rhs)
        self.omega_c = float(omega_c)
        self._k = k
        self._eps = None if eps is None else np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
        if self._eps is not None and self._eps.shape != k.shape:
            raise ValueError("eps must have the shape of k")
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            st = self._lib.th_create(C.byref(h), self.device.index, C.c_void_p(self._stream.cuda_stream))
            if st != 0:
                raise THError(st, "th_create failed")
            self._h = h
            d = L.FineDesc()
            d.dim, d.n, d.order = self.dim, self.N, self.p
            d.k = k.ctypes.data_as(C.POINTER(C.c_double))
            d.eps = (self._eps.ctypes.data_as(C.POINTER(C.c_double)) if self._eps is not None
                     else C.POINTER(C.c_double)())
            for i, b in enumerate(bc):
                d.bc[i] = _BC[b]
            d.alpha_s, d.l_dd, d.n_dd, d.n_s, d.omega_c = alpha_s, l_dd, n_dd, n_s, omega_c
            d.gemm = _GEMM[gemm]
            d.max_rhs = self.max_rhs
            d.layout = _LAYOUT[layout]
            self._check(self._lib.th_setup_fine(self._h, C.byref(d)))
            if coarse is not None:
                self.setup_coarse(coarse, coarse_q, solver=coarse_solver)

    # ------------------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            msg = self._lib.th_last_error(self._h)
            raise THError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.th_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup_coarse(self, scheme: str = "qsfem", q=None, solver: str | None = None):
        """Coarse operator and its factorisation; solver: "nd" (nested
        dissection), "lines" (block elimination over grid lines or planes) or
        None (automatic)."""
        d = L.CoarseDesc()
        d.solver = _CSOLVE[solver]
        if scheme == "qsfem":
            d.scheme = L.TH_COARSE_QSFEM
            d.q = C.POINTER(C.c_double)()
        elif scheme == "plainfit":
            d.scheme = L.TH_COARSE_PLAINFIT
            d.q = C.POINTER(C.c_double)()
        elif scheme == "mlp":
            net, tau = q
            d.scheme = L.TH_COARSE_MLP
            d.q = C.POINTER(C.c_double)()
            d.mlp = net._h
            d.fallback_tau = float(tau)
            self._mlp_ref = net
        elif scheme == "weights":
            q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
            nc = self.N * (self.p // 2)
            want = (nc,) * self.dim + (3 if self.dim == 2 else 4,)
            if q.shape != want:
                raise ValueError(f"q must have shape {want}")
            self._q = q
            d.scheme = L.TH_COARSE_WEIGHTS
            d.q = q.ctypes.data_as(C.POINTER(C.c_double))
        else:
            raise ValueError(scheme)
        with torch.cuda.device(self.device):
            self._check(self._lib.th_setup_coarse(self._h, C.byref(d)))

    def timing(self, enable: bool):
        """Start (and clear) or stop per-kernel-class event timing."""
        self._check(self._lib.th_timing_enable(self._h, 1 if enable else 0))

    def kernel_times(self) -> dict:
        """{class: (total_ms, launches)} since timing was enabled."""
        out = {}
        for i, name in enumerate(L.KERNEL_CLASSES):
            ms, n = C.c_double(), C.c_longlong()
            self._check(self._lib.th_timing_get(self._h, i, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def info(self) -> dict:
        inf = L.Info()
        self._check(self._lib.th_get_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in L.Info._fields_}

    # ------------------------------------------------------------------
    def _vec(self, t: torch.Tensor, n: int, name: str, dtype=None):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.shape[-1] != n or t.dim() not in (1, 2):
            raise ValueError(f"{name} must have shape (nrhs, {n}) or ({n},)")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")
        nrhs = 1 if t.dim() == 1 else t.shape[0]
        if nrhs < 1 or nrhs > self.max_rhs:
            raise ValueError(f"nrhs={nrhs} outside [1, max_rhs={self.max_rhs}]")
        return nrhs

    def _ordered(self, fn, *args):
        """Run a stream-ordered library call on the solver's stream, ordered
        after the caller's current stream and before its later work."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self._stream:
            self._stream.wait_stream(cur)
        st = fn(*args)
        if cur != self._stream:
            cur.wait_stream(self._stream)
        return st

    @staticmethod
    def _p(t):
        return C.c_void_p(t.data_ptr())

    def empty_fine(self, nrhs=1, dtype=torch.complex128):
        return torch.zeros((nrhs, self.n_fine), dtype=dtype, device=self.device)

    def empty_coarse(self, nrhs=1, dtype=torch.complex128):
        return torch.zeros((nrhs, self.n_coarse), dtype=dtype, device=self.device)

    def residual(self, u, f, r=None):
        """r = f - A u."""
        nrhs = self._vec(u, self.n_fine, "u")
        self._vec(f, self.n_fine, "f", u.dtype)
        if f.shape != u.shape:
            raise ValueError("u and f must have the same shape")
        r = torch.empty_like(u) if r is None else r
        self._vec(r, self.n_fine, "r", u.dtype)
        self._check(self._ordered(self._lib.th_residual, self._h, self._p(u), self._p(f), self._p(r), nrhs, _dt(u)))
        return r

    def smooth(self, u, f):
        """u <- CSDDSmoother(u, f) in place."""
        nrhs = self._vec(u, self.n_fine, "u")
        self._vec(f, self.n_fine, "f", u.dtype)
        if f.shape != u.shape:
            raise ValueError("u and f must have the same shape")
        self._check(self._ordered(self._lib.th_smooth, self._h, self._p(u), self._p(f), nrhs, _dt(u)))
        return u

    def restrict(self, r, rc=None):
        """rc = I_P^T r."""
        nrhs = self._vec(r, self.n_fine, "r")
        shape = (self.n_coarse,) if r.dim() == 1 else (nrhs, self.n_coarse)
        rc = torch.empty(shape, dtype=r.dtype, device=self.device) if rc is None else rc
        self._vec(rc, self.n_coarse, "rc", r.dtype)
        self._check(self._ordered(self._lib.th_restrict, self._h, self._p(r), self._p(rc), nrhs, _dt(r)))
        return rc

    def prolong(self, uc, u, omega=None):
        """u += omega I_P uc in place."""
        nrhs = self._vec(u, self.n_fine, "u")
        nrc = self._vec(uc, self.n_coarse, "uc", u.dtype)
        if nrc != nrhs:
            raise ValueError("uc and u must hold the same number of vectors")
        om = self.omega_c if omega is None else float(omega)
        self._check(self._ordered(self._lib.th_prolong, self._h, self._p(uc), self._p(u), om, nrhs, _dt(u)))
        return u

    def coarse_solve(self, rc, uc=None):
        """uc = A_c^{-1} rc (FP64 factors)."""
        nrhs = self._vec(rc, self.n_coarse, "rc")
        uc = torch.empty_like(rc) if uc is None else uc
        self._vec(uc, self.n_coarse, "uc", rc.dtype)
        if uc.data_ptr() == rc.data_ptr():
            raise ValueError("rc and uc must not alias")
        self._check(self._ordered(self._lib.th_coarse_solve, self._h, self._p(rc), self._p(uc), nrhs, _dt(rc)))
        return uc

    def coarse_solve_noalloc(self, rc, uc):
        """uc = A_c^{-1} rc with the library's fixed per-GPU scratch array
        instead of the context's work buffers (allocates nothing)."""
        nrhs = self._vec(rc, self.n_coarse, "rc")
        self._vec(uc, self.n_coarse, "uc", rc.dtype)
        if uc.data_ptr() == rc.data_ptr():
            raise ValueError("rc and uc must not alias")
        self._check(self._ordered(self._lib.th_coarse_solve_noalloc, self._h, self._p(rc),
                                  self._p(uc), nrhs, _dt(rc)))
        return uc

    def twogrid(self, u, f):
        """u <- TwoGridStep(u, f) in place."""
        nrhs = self._vec(u, self.n_fine, "u")
        self._vec(f, self.n_fine, "f", u.dtype)
        if f.shape != u.shape:
            raise ValueError("u and f must have the same shape")
        self._check(self._ordered(self._lib.th_twogrid, self._h, self._p(u), self._p(f), nrhs, _dt(u)))
        return u

    def solve(self, f, u=None, rtol=1e-6, maxit=300, restart=0, precond="c128",
              method="gmres", raise_on_notconv=False, graph=False):
        """Solve A u = f (complex128 vectors) with the two-grid preconditioner.

        Converged means ||f - A u|| / ||f|| <= rtol on the true FP64 residual
        of every right-hand side.  restart <= 0: no restart.
        method: "gmres" / "fgmres" (the same flexible iteration) or
        "stationary".  precond: "c128" (FP64 two-grid step) or "c64"
        (complex64 step under FP64 flexible GMRES).  graph: replay the preconditioner from a HIP
        graph (needs the solver to run on a non-default stream).
        Returns (u, SolveStats)."""
        nrhs = self._vec(f, self.n_fine, "f", torch.complex128)
        u = torch.empty_like(f) if u is None else u
        self._vec(u, self.n_fine, "u", torch.complex128)
        o = L.SolveOpts()
        methods = {"gmres": L.TH_KRYLOV_GMRES_RIGHT, "fgmres": L.TH_KRYLOV_FGMRES,
                   "stationary": L.TH_KRYLOV_STATIONARY}
        if method not in methods:
            raise ValueError(f"method must be one of {sorted(methods)}")
        o.krylov = methods[method]
        o.rtol, o.maxit, o.restart = float(rtol), int(maxit), int(restart)
        o.precond_dtype = L.TH_C128 if precond == "c128" else L.TH_C64
        o.use_graph = 1 if graph else 0
        st = L.SolveStats()
        status = self._ordered(self._lib.th_solve, self._h, self._p(f), self._p(u), nrhs, C.byref(o), C.byref(st))
        if status not in (0, L.TH_ENOTCONV) or (status and raise_on_notconv):
            self._check(status)
        return u, SolveStats(st.iters, st.rel_res, st.t_solve_s, st.n_precond, status,
                             st.t_cycle_s, st.n_fallback_cells)


def plain_fit(samples):
    """Plain dispersion-matching fit (host, through the C ABI): samples (n, 3)
    rows (eta_c, p, shift) -> (e (n, 2) fine dispersion errors at pi/16 and
    3 pi/16, q (n, 3) coarse weights)."""
    lib = L.load()
    x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64).reshape(-1, 3))
    n = x.shape[0]
    e = np.zeros((n, 2))
    q = np.zeros((n, 3))
    st = lib.th_plain_fit(x.ctypes.data, n, e.ctypes.data, q.ctypes.data)
    if st != 0:
        raise THError(st, "th_plain_fit rejected the samples (eta_c > 0, p in 1..8, kh < pi)")
    return e, q


def plain_fit3d(samples):
    """3-D compact 27-point plain fit (host, through the C ABI): samples (n, 3)
    rows (eta_c, p, shift) -> (e (n, 3) fine dispersion errors along the three
    fit directions, q (n, 4) weights (q0, q_face, q_edge, q_corner))."""
    lib = L.load()
    x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64).reshape(-1, 3))
    n = x.shape[0]
    e = np.zeros((n, 3))
    q = np.zeros((n, 4))
    st = lib.th_plain_fit3d(x.ctypes.data, n, e.ctypes.data, q.ctypes.data)
    if st != 0:
        raise THError(st, "th_plain_fit3d rejected the samples (eta_c > 0, p in 1..8, kh < pi)")
    return e, q


@dataclass
class TrainStats:
    loss_first: float
    loss_last: float
    steps: int
    t_targets_s: float
    t_train_s: float


class CoarseStencilMLP:
    """Surrogate network for the per-cell dispersion errors of the fine scheme
    (3 -> 64 -> 64 -> n_out, SiLU; n_out = 2 for the 9-point family of 2-D
    problems, 3 for the 27-point family of 3-D problems), trained and
    evaluated by the library's HIP kernels (FP32 master weights, BF16 copy,
    FP32 accumulation)."""

    def __init__(self, weights=None, device: int | None = None, dim: int = 2):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            st = self._lib.th_mlp_create_family(C.byref(h), self.device.index,
                                                C.c_void_p(self._stream.cuda_stream), int(dim))
            if st != 0:
                raise THError(st, "th_mlp_create_family failed")
            self._h = h
        d, n = C.c_int(), C.c_int()
        self._check(self._lib.th_mlp_info(self._h, C.byref(d), C.byref(n)))
        self.dim, self.n_params = d.value, n.value
        self.n_out = 3 if self.dim == 3 else 2
        if weights is not None:
            self.set_weights(weights)

    def _check(self, st):
        if st != 0:
            msg = self._lib.th_mlp_last_error(self._h)
            raise THError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.th_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, theta):
        w = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
        self._check(self._lib.th_mlp_set_weights(self._h, w.ctypes.data, w.size))

    def weights(self):
        w = np.zeros(self.n_params, dtype=np.float32)
        self._check(self._lib.th_mlp_get_weights(self._h, w.ctypes.data, w.size))
        return w

    def set_scaling(self, in_mean, in_std, out_mean, out_std):
        a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in
             (in_mean, in_std, out_mean, out_std)]
        self._check(self._lib.th_mlp_set_scaling(self._h, *[v.ctypes.data for v in a]))
        self._keep = a

    def scaling(self):
        a = [np.zeros(3), np.zeros(3), np.zeros(self.n_out), np.zeros(self.n_out)]
        self._check(self._lib.th_mlp_get_scaling(self._h, *[v.ctypes.data for v in a]))
        return a

    def loss_grad(self, x_std, y_std, bf16=False):
        x = np.ascontiguousarray(np.asarray(x_std, dtype=np.float32))
        y = np.ascontiguousarray(np.asarray(y_std, dtype=np.float32))
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_double()
        self._check(self._lib.th_mlp_loss_grad(self._h, x.ctypes.data, y.ctypes.data, x.shape[0],
                                               1 if bf16 else 0, C.byref(loss), g.ctypes.data))
        return loss.value, g

    def train(self, samples, epochs=20, batch=1024, lr=2e-3, bf16=True) -> TrainStats:
        x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64))
        o = L.MlpTrainOpts(epochs, batch, lr, 1 if bf16 else 0)
        st = L.MlpTrainStats()
        self._check(self._lib.th_mlp_train(self._h, x.ctypes.data, x.shape[0], C.byref(o),
                                           C.byref(st)))
        return TrainStats(st.loss_first, st.loss_last, st.steps, st.t_targets_s, st.t_train_s)

    def predict(self, samples, bf16=True):
        x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64))
        e = np.zeros((x.shape[0], self.n_out))
        self._check(self._lib.th_mlp_predict(self._h, x.ctypes.data, x.shape[0],
                                             1 if bf16 else 0, e.ctypes.data))
        return e

    def stencils(self, samples):
        """(q, mismatch): per-sample coarse weights from the network and the
        distance (relative to eta) of their zero set from the fine dispersion
        curve over the sector of wave directions, computed on the device."""
        x = np.ascontiguousarray(np.asarray(samples, dtype=np.float64))
        q = np.zeros((x.shape[0], 4 if self.n_out == 3 else 3))
        mis = np.zeros(x.shape[0])
        self._check(self._lib.th_mlp_stencils(self._h, x.ctypes.data, x.shape[0], q.ctypes.data,
                                              mis.ctypes.data))
        return q, mis
