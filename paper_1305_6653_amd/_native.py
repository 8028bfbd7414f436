"""ctypes binding of libfdebvm.so (include/fdebvm.h): argument marshalling only.

The library is loaded from this package directory; there is no fallback.  A missing or
unloadable library raises ``NativeLibraryMissing`` on first use.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDE_LIB_PATH selects another build of the same library (the host-sanitizer build of
# `python -m paper_1305_6653_amd.build --sanitize`); by default the in-tree library.
LIB_PATH = os.environ.get("FDE_LIB_PATH") or os.path.join(_HERE, "libfdebvm.so")

FDE_OK, FDE_EINVAL, FDE_ENOMEM, FDE_ESINGULAR, FDE_ENOCONV, FDE_EDEVICE, FDE_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "FDE_OK", -1: "FDE_EINVAL", -2: "FDE_ENOMEM", -3: "FDE_ESINGULAR",
                -4: "FDE_ENOCONV", -5: "FDE_EDEVICE", -6: "FDE_EUNSUPPORTED"}
FDE_BVM_TRAPEZOIDAL, FDE_BVM_GBDF3, FDE_BVM_CUSTOM, FDE_BVM_GAM5 = 0, 1, 2, 3
FDE_FP64, FDE_MIXED_C32 = 0, 1
FDE_MEM_HOST, FDE_MEM_DEVICE = 0, 1
FDE_COPY_H2D, FDE_COPY_D2H, FDE_COPY_D2D = 0, 1, 2

_dp = C.POINTER(C.c_double)


class FdeBvmFormula(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int),
                ("alpha", _dp), ("beta", _dp),
                ("alpha_init", _dp), ("beta_init", _dp),
                ("alpha_fin", _dp), ("beta_fin", _dp)]


class FdeProblem(C.Structure):
    _fields_ = [("alpha", C.c_double), ("xL", C.c_double), ("xR", C.c_double),
                ("t0", C.c_double), ("T", C.c_double), ("m", C.c_int), ("s", C.c_int),
                ("d_plus", _dp), ("d_minus", _dp), ("kind", C.c_int),
                ("custom", C.POINTER(FdeBvmFormula))]


FDE_X0_SOLUTION, FDE_X0_LOWRANK = 0, 1
FDE_OPT_GRAPHS, FDE_OPT_AUTOTUNE, FDE_OPT_TRSV_W, FDE_OPT_TRSV_W_IN_USE, FDE_OPT_GRAPHS_IN_USE = 0, 1, 2, 3, 4
FDE_OPT_PRECOND, FDE_OPT_SIDE, FDE_OPT_BLOCKS, FDE_OPT_ORTHO = 5, 6, 7, 8
FDE_ORTHO_MGS, FDE_ORTHO_CGS2 = 0, 1
FDE_BLOCKS_LU, FDE_BLOCKS_HESSENBERG, FDE_BLOCKS_BAND, FDE_BLOCKS_AUTO = 0, 1, 2, 3
FDE_OPT_BLOCKS_IN_USE = 9
FDE_OPT_X0_GATE, FDE_OPT_X0_KEPT = 10, 11
FDE_SIDE_RIGHT, FDE_SIDE_LEFT = 0, 1
FDE_PC_STRANG, FDE_PC_BCCB, FDE_PC_BCCB_SHIFTED, FDE_PC_NONE = 0, 1, 2, 3


class FdeSolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int),
                ("x0", C.c_void_p), ("mem_space", C.c_int), ("x0_kind", C.c_int)]


class FdeSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("precision", C.c_int), ("true_relres", C.c_double), ("est_relres", C.c_double),
                ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FdeNnConfig(C.Structure):
    _fields_ = [("m", C.c_int), ("s", C.c_int), ("max_batch", C.c_int),
                ("conv_ch", C.c_int * 3), ("fc", C.c_int * 2), ("nx", C.c_int), ("nt", C.c_int),
                ("seed", C.c_int)]


class NativeLibraryMissing(ImportError):
    pass


class FdeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


# (name, restype, argtypes) for every symbol declared in include/fdebvm.h
_VP = C.c_void_p
SIGNATURES = [
    ("fde_bvm_setup", C.c_int, [C.POINTER(FdeProblem), C.POINTER(_VP)]),
    ("fde_precond_factor", C.c_int, [_VP, C.c_int]),
    ("fde_bvm_solve", C.c_int, [_VP, _VP, _VP, _VP, C.POINTER(FdeSolveOpts), C.POINTER(FdeSolveInfo)]),
    ("fde_precond_factor_batch", C.c_int, [C.POINTER(_VP), C.c_int, C.c_int]),
    ("fde_bvm_solve_batch", C.c_int, [C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(_VP),
                                      C.POINTER(_VP), C.POINTER(FdeSolveOpts), C.POINTER(FdeSolveInfo)]),
    ("fde_bvm_solve_batch_x0", C.c_int, [C.POINTER(_VP), C.c_int, C.POINTER(_VP), C.POINTER(_VP),
                                         C.POINTER(_VP), C.POINTER(_VP), C.POINTER(FdeSolveOpts),
                                         C.POINTER(FdeSolveInfo)]),
    ("fde_bvm_destroy", None, [_VP]),
    ("fde_last_error", C.c_char_p, []),
    ("fde_set_stream", C.c_int, [_VP, _VP]),
    ("fde_get_dims", C.c_int, [_VP, C.POINTER(C.c_int)]),
    ("fde_bvm_set_option", C.c_int, [_VP, C.c_int, C.c_int]),
    ("fde_bvm_get_option", C.c_int, [_VP, C.c_int, C.POINTER(C.c_int)]),
    ("fde_autotune_report", C.c_int, [C.c_char_p, C.c_int]),
    ("fde_device_alloc", C.c_int, [C.c_size_t, C.POINTER(_VP)]),
    ("fde_device_free", C.c_int, [_VP]),
    ("fde_memcpy", C.c_int, [_VP, _VP, C.c_size_t, C.c_int]),
    ("fde_device_synchronize", C.c_int, []),
    ("fde_read_bandwidth_probe", C.c_int, [C.c_size_t, C.c_int, _dp]),
    ("fde_mfma_peak_probe", C.c_int, [C.c_int, C.c_int, _dp]),
    ("fde_build_rhs", C.c_int, [_VP, _VP, _VP, _VP, C.c_int]),
    ("fde_apply_matvec", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_toeplitz_apply", C.c_int, [_VP, _VP, _VP, C.c_int, C.c_int]),
    ("fde_time_rfft", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_apply_precond", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_apply_precond_noalloc", C.c_int, [_VP, _VP, _VP]),
    ("fde_get_factor_block", C.c_int, [_VP, C.c_int, _VP]),
    ("fde_get_hessenberg", C.c_int, [_VP, _VP, _VP]),
    ("fde_profile_enable", C.c_int, [_VP, C.c_int]),
    ("fde_profile_query", C.c_int, [_VP, C.c_char_p, _dp, C.POINTER(C.c_int), _dp]),
    ("fde_bvm_set_coefficients", C.c_int, [_VP, C.c_double, _dp, _dp]),
    ("fde_bvm_strang_apply", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_bvm_lowrank_correction", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_nn_set_basis", C.c_int, [_VP, _VP]),
    ("fde_nn_create", C.c_int, [C.POINTER(FdeNnConfig), C.POINTER(_VP)]),
    ("fde_nn_destroy", None, [_VP]),
    ("fde_nn_last_error", C.c_char_p, []),
    ("fde_nn_num_params", C.c_int, [_VP, C.POINTER(C.c_longlong)]),
    ("fde_nn_set_params", C.c_int, [_VP, _VP]),
    ("fde_nn_get_params", C.c_int, [_VP, _VP, C.c_int]),
    ("fde_nn_set_state", C.c_int, [_VP, _VP, _VP, C.c_int]),
    ("fde_nn_get_step", C.c_int, [_VP, C.POINTER(C.c_int)]),
    ("fde_nn_features", C.c_int, [_VP, C.c_int, C.POINTER(_VP), C.POINTER(_VP), C.POINTER(_VP),
                                  _dp, _VP, _VP]),
    ("fde_nn_loss_grad", C.c_int, [_VP, _VP, _VP, _VP, C.POINTER(C.c_int), C.c_int,
                                   C.POINTER(C.c_float)]),
    ("fde_nn_adam", C.c_int, [_VP, C.c_float, C.c_float, C.c_float, C.c_float]),
    ("fde_nn_predict", C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_int), C.c_int, C.POINTER(_VP)]),
    ("fde_nn_output", C.c_int, [_VP, _VP, C.c_int]),
    ("fde_nn_sync", C.c_int, [_VP]),
]

_lib = None


def _bind_runtime_first():
    """Make the HIP runtime that torch ships the only one in the process.

    torch's libamdhip64.so carries the same SONAME (libamdhip64.so.7) as the system ROCm
    runtime this library is linked against, and torch resolves its own copy through its
    RPATH, so the first of the two to be loaded decides which runtime this library binds
    to.  Importing torch first maps torch's runtime (and its HSA runtime) once; this library
    then binds to it by SONAME and no second runtime is ever mapped.  With FDE_NO_TORCH=1
    torch is not imported and the library binds to the system runtime instead (a process
    that must not map torch's copy, e.g. one whose profiler preloads the system runtime);
    torch must then not be imported later in that process."""
    if os.environ.get("FDE_NO_TORCH", "0") == "1":
        return
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load libfdebvm.so once; raise NativeLibraryMissing if it is absent or broken."""
    global _lib
    if _lib is not None:
        return _lib
    _bind_runtime_first()
    if not os.path.exists(LIB_PATH):
        raise NativeLibraryMissing(
            f"{LIB_PATH} is not built; run `python -m paper_1305_6653_amd.build` (hipcc, gfx950)")
    try:
        L = C.CDLL(LIB_PATH)
    except OSError as e:
        raise NativeLibraryMissing(f"cannot load {LIB_PATH}: {e}") from e
    for name, res, args in SIGNATURES:
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int) -> int:
    if status != FDE_OK:
        raise FdeError(status, lib().fde_last_error().decode(errors="replace"))
    return status


def check_nn(status: int) -> int:
    if status != FDE_OK:
        raise FdeError(status, lib().fde_nn_last_error().decode(errors="replace"))
    return status
