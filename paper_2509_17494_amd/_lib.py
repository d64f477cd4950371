"""ctypes declarations of the C ABI in include/th.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libth.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "th.h")

TH_OK, TH_EINVAL, TH_ESTATE, TH_ENOMEM, TH_EHIP, TH_ENOTCONV, TH_ENUMERIC, TH_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "TH_OK", -1: "TH_EINVAL", -2: "TH_ESTATE", -3: "TH_ENOMEM", -4: "TH_EHIP",
                -5: "TH_ENOTCONV", -6: "TH_ENUMERIC", -7: "TH_EUNSUPPORTED"}
TH_BC_ROBIN, TH_BC_NEUMANN, TH_BC_DIRICHLET = 0, 1, 2
TH_LAYOUT_AUTO, TH_LAYOUT_DENSE, TH_LAYOUT_SYMMETRIC, TH_LAYOUT_SLAB = 0, 1, 2, 3
TH_C128, TH_C64 = 0, 1
TH_GEMM_F64, TH_GEMM_F32, TH_GEMM_BF16 = 0, 1, 2
TH_COARSE_QSFEM, TH_COARSE_PLAINFIT, TH_COARSE_MLP, TH_COARSE_WEIGHTS = 0, 1, 2, 3
TH_KRYLOV_GMRES_RIGHT, TH_KRYLOV_FGMRES, TH_KRYLOV_STATIONARY = 0, 1, 2
TH_CSOLVE_AUTO, TH_CSOLVE_LINES, TH_CSOLVE_ND = 0, 1, 2
KERNEL_CLASSES = ["dd_apply", "dd_accum", "operator", "restrict", "prolong", "coarse", "krylov"]


class FineDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("order", C.c_int),
                ("k", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
                ("bc", C.c_int * 6), ("alpha_s", C.c_double), ("l_dd", C.c_int),
                ("n_dd", C.c_int), ("n_s", C.c_int), ("omega_c", C.c_double),
                ("gemm", C.c_int), ("max_rhs", C.c_int), ("layout", C.c_int)]


class CoarseDesc(C.Structure):
    _fields_ = [("scheme", C.c_int), ("q", C.POINTER(C.c_double)), ("mlp", C.c_void_p),
                ("fallback_tau", C.c_double), ("solver", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("krylov", C.c_int), ("rtol", C.c_double), ("maxit", C.c_int),
                ("restart", C.c_int), ("precond_dtype", C.c_int), ("use_graph", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res", C.c_double), ("t_solve_s", C.c_double),
                ("n_precond", C.c_longlong), ("t_cycle_s", C.c_double),
                ("n_fallback_cells", C.c_int)]


class Info(C.Structure):
    _fields_ = [("n_fine", C.c_longlong), ("n_coarse", C.c_longlong), ("n_sub", C.c_int),
                ("b_entries", C.c_longlong), ("b_bytes", C.c_longlong),
                ("coarse_bytes", C.c_longlong), ("t_setup_fine_s", C.c_double),
                ("t_setup_coarse_s", C.c_double), ("smoother_cfg", C.c_int),
                ("smoother_grid", C.c_int), ("coarse_lines", C.c_int),
                ("n_fallback_cells", C.c_int), ("t_stencil_s", C.c_double),
                ("smoother_layout", C.c_int), ("coarse_solver", C.c_int),
                ("coarse_levels", C.c_int), ("coarse_refine", C.c_int),
                ("coarse_check", C.c_double),
                ("slab_packed", C.c_int),
                ("coarse_refine_exact", C.c_int),
                ("coarse_check_pc", C.c_double)]


_lib = None


def declared_functions(header: str = HEADER):
    """Names of the functions declared in the public header."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(th_[a-z_]+)\s*\(", text)))


def load():
    """Load libth.so; raises ImportError when the HIP library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2509_17494_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    sig = {
        "th_create": ([C.POINTER(vp), i, vp], i),
        "th_destroy": ([vp], None),
        "th_last_error": ([vp], C.c_char_p),
        "th_get_info": ([vp, C.POINTER(Info)], i),
        "th_setup_fine": ([vp, C.POINTER(FineDesc)], i),
        "th_setup_coarse": ([vp, C.POINTER(CoarseDesc)], i),
        "th_residual": ([vp, vp, vp, vp, i, i], i),
        "th_smooth": ([vp, vp, vp, i, i], i),
        "th_restrict": ([vp, vp, vp, i, i], i),
        "th_prolong": ([vp, vp, vp, d, i, i], i),
        "th_coarse_solve": ([vp, vp, vp, i, i], i),
        "th_coarse_solve_noalloc": ([vp, vp, vp, i, i], i),
        "th_twogrid": ([vp, vp, vp, i, i], i),
        "th_solve": ([vp, vp, vp, i, C.POINTER(SolveOpts), C.POINTER(SolveStats)], i),
        "th_timing_enable": ([vp, i], i),
        "th_timing_get": ([vp, i, C.POINTER(C.c_double), C.POINTER(C.c_longlong)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    load_mlp(lib)
    _lib = lib
    return lib


class MlpTrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("bf16", C.c_int)]


class MlpTrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("steps", C.c_int),
                ("t_targets_s", C.c_double), ("t_train_s", C.c_double)]


def load_mlp(lib):
    """Declare the surrogate-network entry points on an already loaded library."""
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    sig = {
        "th_plain_fit": ([vp, i, vp, vp], i),
        "th_plain_fit3d": ([vp, i, vp, vp], i),
        "th_mlp_num_params": ([C.POINTER(i)], i),
        "th_mlp_create": ([C.POINTER(vp), i, vp], i),
        "th_mlp_create_family": ([C.POINTER(vp), i, vp, i], i),
        "th_mlp_info": ([vp, C.POINTER(i), C.POINTER(i)], i),
        "th_mlp_destroy": ([vp], None),
        "th_mlp_last_error": ([vp], C.c_char_p),
        "th_mlp_set_weights": ([vp, vp, i], i),
        "th_mlp_get_weights": ([vp, vp, i], i),
        "th_mlp_set_scaling": ([vp, vp, vp, vp, vp], i),
        "th_mlp_get_scaling": ([vp, vp, vp, vp, vp], i),
        "th_mlp_loss_grad": ([vp, vp, vp, i, i, C.POINTER(d), vp], i),
        "th_mlp_train": ([vp, vp, i, C.POINTER(MlpTrainOpts), C.POINTER(MlpTrainStats)], i),
        "th_mlp_predict": ([vp, vp, i, i, vp], i),
        "th_mlp_stencils": ([vp, vp, i, vp, vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib
