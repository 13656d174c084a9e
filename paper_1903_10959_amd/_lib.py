"""ctypes declarations of the C ABI in include/chfsi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchfsi.so")

FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}

OK, ERR_ARG, ERR_STATE, ERR_OOM, ERR_HIP, ERR_NOT_SPD, ERR_NONFINITE = 0, -1, -2, -3, -4, -5, -6
WARN_NOT_CONVERGED = 1


class Opts(C.Structure):
    _fields_ = [("nstates", C.c_int), ("nblock", C.c_int), ("degree", C.c_int), ("max_iter", C.c_int),
                ("block_width", C.c_int), ("tol", C.c_double), ("ladder", C.c_int * 4), ("n_ladder", C.c_int),
                ("ladder_tol", C.c_double * 4), ("mixed_cholgs", C.c_int)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int), ("status", C.c_int), ("rung", C.c_int), ("t_filter", C.c_double),
                ("t_cholgs", C.c_double), ("t_rr", C.c_double), ("max_resid", C.c_double),
                ("dofvecs", C.c_int64)]


_vp, _dp, _i64, _int, _dbl = C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_double

SIGNATURES = {
    "chfsi_create": (_int, [C.POINTER(C.c_void_p), _int, _vp]),
    "chfsi_destroy": (_int, [_vp]),
    "chfsi_set_mesh": (_int, [_vp, _dbl, _int, _int]),
    "chfsi_get_sizes": (_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
    "chfsi_get_cell_dof_map": (_int, [_vp, _vp]),
    "chfsi_get_cell_colors": (_int, [_vp, _vp]),
    "chfsi_get_dof_coords": (_int, [_vp, _vp]),
    "chfsi_get_mass": (_int, [_vp, _vp]),
    "chfsi_get_cell_matrix": (_int, [_vp, _vp]),
    "chfsi_set_potential": (_int, [_vp, _vp, _i64, _int]),
    "chfsi_get_upper_bound": (_int, [_vp, C.POINTER(C.c_double)]),
    "chfsi_apply": (_int, [_vp, _dp, _dp, _i64, _int, _int]),
    "chfsi_cheb_step": (_int, [_vp, _dp, _dp, _dp, _i64, _int, _dbl, _dbl, _dbl]),
    "chfsi_chebyshev_filter": (_int, [_vp, _dp, _i64, _int, _int, _dbl, _dbl, _dbl, _int, _int]),
    "chfsi_orthonormalize": (_int, [_vp, _dp, _i64, _int, _int]),
    "chfsi_rayleigh_ritz": (_int, [_vp, _dp, _i64, _int, _vp, _vp, _dp]),
    "chfsi_solve": (_int, [_vp, C.POINTER(Opts), _dp, _i64, _vp, _vp, C.POINTER(Report)]),
    "chfsi_solve_batch": (_int, [_vp, _int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "chfsi_batch_create": (_int, [C.POINTER(C.c_void_p), _int]),
    "chfsi_batch_destroy": (_int, [_vp]),
    "chfsi_batch_add": (_int, [_vp, _vp, C.POINTER(Opts), _dp, _i64, _vp, _vp]),
    "chfsi_batch_pass": (_int, [_vp, _vp, C.POINTER(C.c_int), _int]),
    "chfsi_batch_report": (_int, [_vp, _int, C.POINTER(Report)]),
    "chfsi_batch_last_error": (C.c_char_p, [_vp]),
    "chfsi_footprint_bytes": (C.c_size_t, [_int, _int, _int, _int, _int]),
    "chfsi_status_string": (C.c_char_p, [_int]),
    "chfsi_last_error": (C.c_char_p, [_vp]),
    "chfsi_rayleigh_ritz_split": (_int, [_vp, _vp, _i64, _int, _int, _int, _vp, _i64, _vp, _vp]),
    "chfsi_fermi_level": (_int, [_vp, _int, _int, _dbl, _dbl, _vp]),
    "chfsi_set_mesh_periodic": (_int, [_vp, _dbl, _int, _int]),
    "chfsi_set_kpoint": (_int, [_vp, _dbl, _dbl, _dbl]),
    "chfsi_apply_complex": (_int, [_vp, _vp, _vp, _i64, _int]),
    "chfsi_set_kpoints": (_int, [_vp, _int, _vp]),
    "chfsi_poisson_apply": (_int, [_vp, _vp, _vp]),
    "chfsi_poisson_solve": (_int, [_vp, _vp, _int, _vp, _vp, _vp, _dbl, _int, _vp, _vp]),
    "chfsi_apply_complex_kpoints": (_int, [_vp, _vp, _vp, _i64, _int, _i64]),
    "chfsi_density": (_int, [_vp, _vp, _i64, _int, _vp, _i64, _int, _vp, _dbl, _dbl, _vp]),
    "chfsi_set_timing": (_int, [_vp, _int]),
    "chfsi_set_tile_variant": (_int, [_vp, _int]),
    "chfsi_set_cells_per_tile": (_int, [_vp, _int]),
    "chfsi_set_rr_residual": (_int, [_vp, _int]),
    "chfsi_reset_timing": (_int, [_vp]),
    "chfsi_last_filter_timing": (_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)]),
    "chfsi_set_jacobi_sweeps": (_int, [_vp, _int]),
    "chfsi_batch_set_threads": (_int, [_vp, _int]),
    "chfsi_batch_footprint_bytes": (C.c_size_t, [_int, _int, _int]),
    "chfsi_device_bytes": (_int, [_vp, C.POINTER(C.c_size_t)]),
    "chfsi_orthonormalize_noalloc": (_int, [_vp, _dp, _i64, _int, _int]),
    "chfsi_get_upper_bound_k": (_int, [_vp, C.POINTER(C.c_double)]),
    "chfsi_chebyshev_filter_complex": (_int, [_vp, _vp, _i64, _int, _int, _dbl, _dbl, _dbl, _int]),
    "chfsi_orthonormalize_complex": (_int, [_vp, _vp, _i64, _int]),
    "chfsi_rayleigh_ritz_complex": (_int, [_vp, _vp, _i64, _int, _vp, _vp, _vp]),
    "chfsi_solve_complex": (_int, [_vp, C.POINTER(Opts), _vp, _i64, _vp, _vp, C.POINTER(Report)]),
}

_LIB = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (no fallback).

    torch is imported first: its bundled HIP runtime is then already resident
    under the soname libamdhip64.so.7, and the library's own dependency on that
    soname binds to it, so one process never holds two HIP (or HSA) runtimes
    (torch's libraries name the runtime without the version suffix and would
    otherwise load a second copy next to /opt/rocm's)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with "
                           f"`python -m paper_1903_10959_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
