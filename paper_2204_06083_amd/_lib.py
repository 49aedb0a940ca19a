"""ctypes binding of libebamg.so (the C ABI declared in include/ebamg.h).

Argument marshalling only.  Loading fails loudly if the HIP library has not
been built: there is no CPU fallback anywhere in the product path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebamg.so")

EB_OK, EB_EINVAL, EB_EDOMAIN, EB_ENOSPC, EB_ENOTSPD, EB_ENAN, EB_ENOCONV, EB_EHIP, EB_ENOTIMPL, EB_EGEOM = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
EB_BC_LINE, EB_BC_MIXED, EB_BC_RBF = 0, 1, 2
BC_MODES = {"line": EB_BC_LINE, "mixed": EB_BC_MIXED, "rbf": EB_BC_RBF}

EXPORTS = [
    "eb_assemble_diag", "eb_assemble_diag_mode", "eb_assemble_diag_beta", "eb_assemble_rhs", "eb_assemble_rhs_islands",
    "amg_setup_beta", "amg_setup_islands", "stencil_apply_beta", "eb_wave_rhs_beta", "eb_stencil_combine_beta", "stencil_apply", "amg_setup", "pcg_solve", "pcg_solve_batched",
    "amg_vcycle_apply", "amg_vcycle_apply_fp32", "amg_vcycle_apply_prec", "amg_set_level_weight", "amg_num_levels", "amg_level_info", "amg_fine_nodes", "amg_free",
    "eb_strerror", "eb_last_error", "eb_abi_version", "eb_timing_select", "eb_timing_read",
    "eb_release_cached_memory", "eb_smoother_net_size", "eb_smoother_forward", "eb_smoother_backward",
    "eb_smoother_scratch_floats", "eb_adam_step", "amg_set_fine_weights", "amg_clear_fine_weights",
    "amg_smoother_samples", "amg_smoother_loss_grad", "eb_wave_rhs", "eb_stencil_combine",
    "pcg_solve_islands", "pcg_batched_set_launch_shape", "pcg_batched_launch_shape", "eb_set_iteration_graphs",
    "eb_check_spd", "eb_segment_dots", "eb_segment_dots_noalloc",
]

KERNEL_IDS = {"pcg_spmv": 0, "pcg_xr_down": 1, "fine_down": 2, "fine_restrict": 3, "fine_up": 4,
              "fine_post": 5}


class EbGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("x0", C.c_double * 3), ("h", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class AmgParams(C.Structure):
    _fields_ = [("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("min_reduction", C.c_double),
                ("dense_limit", C.c_int32), ("reserved", C.c_int32), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p)]


class PcgParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("x0_given", C.c_int32),
                ("check_every", C.c_int32), ("precision", C.c_int32)]


PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}


class PcgResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("restarts", C.c_int32),
                ("levels", C.c_int32), ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double),
                ("solve_ms", C.c_double), ("reserved", C.c_double)]


class LevelInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_p", C.c_int64), ("nnz_r", C.c_int64),
                ("rho", C.c_double), ("omega", C.c_double), ("is_coarsest", C.c_int32),
                ("max_comp", C.c_int32), ("ext", C.c_int32 * 3), ("nnz_ap", C.c_int32),
                ("a_rowptr", C.c_void_p), ("a_col", C.c_void_p), ("a_val", C.c_void_p),
                ("p_rowptr", C.c_void_p), ("p_col", C.c_void_p), ("p_val", C.c_void_p),
                ("r_rowptr", C.c_void_p), ("r_col", C.c_void_p), ("r_val", C.c_void_p),
                ("agg", C.c_void_p), ("coords", C.c_void_p), ("dense_inv", C.c_void_p)]


CUT_DTYPE = np.dtype([("node", "<i8"), ("dir", "<i4"), ("steps", "<i4"), ("q", "<f8"),
                      ("c", "<f8"), ("xg", "<f8", (3,))])
assert CUT_DTYPE.itemsize == 56


class EbError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libebamg.so (once); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2204_06083_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.eb_assemble_diag.argtypes = [C.POINTER(EbGrid), vp, vp, vp, vp, i64, C.POINTER(i64), C.POINTER(i64), vp]
    L.eb_assemble_diag_mode.argtypes = [C.POINTER(EbGrid), vp, i32, vp, vp, vp, i64, C.POINTER(i64),
                                        C.POINTER(i64), vp]
    L.eb_assemble_diag_mode.restype = i32
    L.eb_assemble_diag_beta.argtypes = [C.POINTER(EbGrid), vp, vp, i32, vp, vp, vp, i64, C.POINTER(i64),
                                        C.POINTER(i64), vp]
    L.eb_assemble_diag_beta.restype = i32
    L.eb_assemble_rhs.argtypes = [C.POINTER(EbGrid), vp, vp, vp, i64, vp, vp, vp]
    L.eb_assemble_rhs_islands.argtypes = [C.POINTER(EbGrid), vp, vp, vp, i64, vp, i32, C.POINTER(i32),
                                          C.POINTER(dbl), vp, vp]
    L.eb_assemble_rhs_islands.restype = i32
    L.eb_check_spd.argtypes = [C.POINTER(EbGrid), vp, vp, i64, C.POINTER(i64), C.POINTER(i64), vp]
    L.eb_check_spd.restype = i32
    L.stencil_apply.argtypes = [C.POINTER(EbGrid), vp, vp, dbl, vp, vp, vp]
    L.eb_wave_rhs.argtypes = [C.POINTER(EbGrid), vp, vp, dbl, dbl, dbl, vp, vp, vp, vp]
    L.eb_stencil_combine.argtypes = [C.POINTER(EbGrid), vp, vp, dbl, dbl, vp, dbl, vp, dbl, vp, vp, vp]
    L.stencil_apply_beta.argtypes = [C.POINTER(EbGrid), vp, vp, vp, dbl, vp, vp, vp]
    L.eb_wave_rhs_beta.argtypes = [C.POINTER(EbGrid), vp, vp, vp, dbl, dbl, dbl, vp, vp, vp, vp]
    L.eb_stencil_combine_beta.argtypes = [C.POINTER(EbGrid), vp, vp, vp, dbl, dbl, vp, dbl, vp, dbl, vp, vp, vp]
    for name in ("stencil_apply_beta", "eb_wave_rhs_beta", "eb_stencil_combine_beta"):
        getattr(L, name).restype = i32
    L.eb_segment_dots.argtypes = [vp, vp, C.c_int32, i64, i64, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dbl), vp]
    L.eb_segment_dots_noalloc.argtypes = L.eb_segment_dots.argtypes
    L.amg_setup.argtypes = [C.POINTER(EbGrid), vp, vp, dbl, C.POINTER(AmgParams), C.POINTER(vp), vp]
    L.amg_setup_beta.argtypes = [C.POINTER(EbGrid), vp, vp, vp, dbl, C.POINTER(AmgParams), C.POINTER(vp), vp]
    L.amg_setup_beta.restype = i32
    L.amg_setup_islands.argtypes = [C.POINTER(EbGrid), vp, vp, dbl, i32, C.POINTER(i32), C.POINTER(AmgParams),
                                    C.POINTER(vp), vp]
    L.amg_setup_islands.restype = i32
    L.pcg_solve.argtypes = [vp, vp, vp, C.POINTER(PcgParams), C.POINTER(PcgResult), vp]
    L.pcg_solve_batched.argtypes = [vp, C.c_int32, vp, vp, C.POINTER(PcgParams), C.POINTER(PcgResult), vp]
    L.pcg_solve_islands.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int32), vp, vp, C.POINTER(PcgParams),
                                    C.POINTER(PcgResult), vp]
    L.pcg_batched_set_launch_shape.argtypes = [C.c_int32, C.c_int32]
    L.eb_set_iteration_graphs.argtypes = [C.c_int32]
    i32p = C.POINTER(C.c_int32)
    L.pcg_batched_launch_shape.argtypes = [vp, i32p, i32p, i32p, i32p, i32p, C.POINTER(C.c_float)]
    L.amg_vcycle_apply.argtypes = [vp, vp, vp, vp]
    L.amg_vcycle_apply_fp32.argtypes = [vp, vp, vp, vp]
    L.amg_vcycle_apply_prec.argtypes = [vp, vp, vp, i32, vp]
    L.amg_set_level_weight.argtypes = [vp, i32, dbl, vp]
    L.amg_set_level_weight.restype = i32
    L.amg_num_levels.argtypes = [vp]
    L.amg_level_info.argtypes = [vp, C.c_int, C.POINTER(LevelInfo)]
    L.amg_fine_nodes.argtypes = [vp]
    L.amg_fine_nodes.restype = vp
    L.amg_free.argtypes = [vp]
    L.amg_free.restype = None
    L.eb_timing_select.argtypes = [vp, C.c_int]
    L.eb_timing_read.argtypes = [vp, C.POINTER(i64), C.POINTER(dbl)]
    L.eb_release_cached_memory.argtypes = []
    L.eb_release_cached_memory.restype = None
    L.eb_smoother_net_size.argtypes = [i32]
    L.eb_smoother_net_size.restype = i64
    L.eb_smoother_forward.argtypes = [C.POINTER(EbGrid), vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp]
    L.eb_smoother_backward.argtypes = [C.POINTER(EbGrid), vp, vp, vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp]
    L.eb_smoother_scratch_floats.argtypes = [C.POINTER(EbGrid)]
    L.eb_smoother_scratch_floats.restype = i64
    L.eb_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, C.c_float, vp]
    L.amg_set_fine_weights.argtypes = [vp, vp, vp]
    L.amg_clear_fine_weights.argtypes = [vp]
    L.amg_smoother_samples.argtypes = [vp, i32, i32, vp, vp, vp]
    L.amg_smoother_loss_grad.argtypes = [vp, i32, vp, C.POINTER(dbl), vp, vp]
    L.eb_strerror.argtypes = [C.c_int]
    L.eb_strerror.restype = C.c_char_p
    L.eb_last_error.restype = C.c_char_p
    for name in ("eb_assemble_diag", "eb_assemble_rhs", "stencil_apply", "amg_setup", "pcg_solve", "pcg_solve_batched",
                 "amg_vcycle_apply", "amg_vcycle_apply_fp32", "amg_vcycle_apply_prec", "amg_num_levels", "amg_level_info", "eb_abi_version",
                 "eb_timing_select", "eb_timing_read", "eb_smoother_forward", "eb_smoother_backward",
                 "eb_adam_step", "amg_set_fine_weights", "amg_clear_fine_weights", "amg_smoother_samples",
                 "amg_smoother_loss_grad"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(code, where, ok=(EB_OK,)):
    if code not in ok:
        L = lib()
        raise EbError(code, where, L.eb_last_error().decode() or L.eb_strerror(code).decode())
    return code


def make_grid(grid) -> EbGrid:
    """EbGrid from a workloads.Grid-like object (dim, n, x0, h)."""
    g = EbGrid()
    g.dim = int(grid.dim)
    for a in range(3):
        g.n[a] = int(grid.n[a]) if a < grid.dim else 0
        g.x0[a] = float(grid.x0[a]) if a < grid.dim else 0.0
    g.h = float(grid.h)
    return g


_hip = None


def hip_runtime():
    """libamdhip64 for raw device copies of library-owned arrays."""
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64.so not found")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


def copy_device_to_host(ptr: int, nbytes: int, out: np.ndarray):
    """Blocking copy of nbytes from a device pointer into a host numpy array."""
    if nbytes == 0:
        return out
    assert out.nbytes >= nbytes
    rc = hip_runtime().hipMemcpy(out.ctypes.data, C.c_void_p(ptr), nbytes, 4)  # hipMemcpyDefault
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
    return out
