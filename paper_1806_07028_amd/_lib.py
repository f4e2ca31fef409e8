"""ctypes binding of libpcamg.so (the C ABI in include/pcamg.h).

Argument marshalling only: torch tensors supply device memory (their data
pointers) and the current HIP stream; every step of the method runs in the
library's HIP kernels.  If the library is missing this module raises -- there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcamg.so")
_lib = None

_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u64 = C.c_uint64


class Params(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("theta", C.c_double),
        ("max_iter", _i32),
        ("outer", _i32),
        ("cycle_prec", _i32),
        ("coarse_max", _i32),
        ("relax_sweeps", _i32),
        ("rebuild_vcycles", _i32),
        ("rebuild_source", _i32),
        ("p1_mode", _i32),
        ("coarse_solve", _i32),
        ("a2_hub_cap", _i32),
        ("max_rebuilds", _i32),
        ("max_levels", _i32),
        ("numW", _i32),
        ("iterW", _i32),
        ("iterV", _i32),
        ("rebuild_rule", _i32),
        ("keep_setup", _i32),
        ("validate", _i32),
        ("tail_max_n", _i32),
        ("use_graphs", _i32),
        ("row_lanes", _i32),
        ("w_dense", _i32),
        ("first_sweeps", _i32),
        ("dense_max_n", _i32),
        ("long_row_min", _i32),
        ("v_dense_max_n", _i32),
        ("seed", _u64),
        ("colour_seed", _u64),
        ("case3", _i32),
        ("block_sweep_min_colours", _i32),
        ("init", _i32),
        ("top_dense_max_n", _i32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", _i32),
        ("rebuilds", _i32),
        ("levels", _i32),
        ("status", _i32),
        ("relres", C.c_double),
        ("true_relres", C.c_double),
        ("rho_geo", C.c_double),
        ("convr_last10", C.c_double),
        ("op_complexity", C.c_double),
        ("t_setup_ms", C.c_double),
        ("t_solve_ms", C.c_double),
        ("t_rebuild_ms", C.c_double),
        ("t_approx_ms", C.c_double),
        ("t_build_ms", C.c_double),
        ("vcycles64", _i32),
        ("vcycles32", _i32),
        ("wcycles", _i32),
        ("hist_len", _i32),
        ("relres_hist", C.POINTER(C.c_double)),
        ("hist_cap", _i32),
        ("learned_builds", _i32),
        ("fallback_builds", _i32),
    ]


class Graph(C.Structure):
    _fields_ = [("n", _i32), ("nnz", _i32), ("row_ptr", _p), ("col_idx", _p), ("weight", _p)]


STATUS = {0: "ok", -1: "EINVAL", -2: "ENOTSYM", -3: "ESELFLOOP", -4: "EDUPEDGE", -5: "EWEIGHT",
          -6: "EDISCONNECTED", -7: "ERHS", -8: "ENOMEM", -9: "EHIP", -10: "ENOCONV", -11: "EBREAKDOWN",
          -12: "ENAN", -13: "EUNSUPPORTED"}


class PcamgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_SIGS = {
    "pcamg_status_str": ([_i32], C.c_char_p),
    "pcamg_last_error": ([], C.c_char_p),
    "pcamg_params_default": ([C.POINTER(Params)], _i32),
    "pcamg_setup": ([C.POINTER(Graph), _p, C.POINTER(Params), _p, C.POINTER(_p)], _i32),
    "pcamg_set_rhs": ([_p, _p], _i32),
    "pcamg_solve": ([_p, _p, C.POINTER(Stats)], _i32),
    "pcamg_rebuild": ([_p, _p], _i32),
    "pcamg_destroy": ([_p], None),
    "pcamg_net_num_params": ([], _i32),
    "pcamg_net_create": ([C.POINTER(_p)], _i32),
    "pcamg_net_destroy": ([_p], None),
    "pcamg_net_set_params": ([_p, _p, _p], _i32),
    "pcamg_net_get_params": ([_p, _p, _p], _i32),
    "pcamg_net_init": ([_p, _u64, _p], _i32),
    "pcamg_net_forward": ([_p, C.POINTER(Graph), _p, _p, _p], _i32),
    "pcamg_net_loss_grad": ([_p, C.POINTER(Graph), _p, _p, C.POINTER(C.c_double), _p, _p], _i32),
    "pcamg_net_adam_step": ([_p, C.c_float, _p], _i32),
    "pcamg_relax_vector": ([C.POINTER(Graph), C.POINTER(Params), _i32, _p, _p, _p], _i32),
    "pcamg_start_vector": ([C.POINTER(Graph), C.POINTER(Params), _i32, _p, _p], _i32),
    "pcamg_setup_learned": ([C.POINTER(Graph), _p, C.POINTER(Params), _p, _p, C.POINTER(_p)], _i32),
    "pcamg_batch_solve": ([C.POINTER(Graph), C.POINTER(_p), C.POINTER(_p), _i32, C.POINTER(Params), _i32,
                           C.POINTER(Stats)], _i32),
    "pcamg_num_hierarchies": ([_p, C.POINTER(_i32)], _i32),
    "pcamg_num_levels": ([_p, _i32, C.POINTER(_i32)], _i32),
    "pcamg_level_info": ([_p, _i32, _i32, C.POINTER(_i64)], _i32),
    "pcamg_level_get": ([_p, _i32, _i32, C.c_char_p, _p], _i32),
    "pcamg_cycle": ([_p, _i32, _p, _p, _i32], _i32),
    "pcamg_cycle32": ([_p, _i32, _p, _p, _i32], _i32),
    "pcamg_approx_error": ([_p, _i32, _p, _p], _i32),
    "pcamg_initial_error": ([_p, _p], _i32),
    "pcamg_bench_smoother": ([_p, _i32, _i32, C.POINTER(C.c_double), C.POINTER(_i64), C.POINTER(C.c_double)], _i32),
    "pcamg_bench_level": ([_p, _i32, _i32, _i32, _i64, C.POINTER(C.c_double), C.POINTER(_i64),
                           C.POINTER(C.c_double)], _i32),
    "pcamg_bench_copy": ([_i64, _i32, _p, C.POINTER(C.c_double)], _i32),
    "pcamg_bench_gemm": ([_i32, _i32, _i32, _i32, _i32, _p, C.POINTER(C.c_double)], _i32),
    "pcamg_laplacian": ([_i32, _p, _p, _p, _p, _p, _p, _p], _i32),
    "pcamg_colour": ([_i32, _p, _p, _u64, _i32, _p, C.POINTER(_i32), _p], _i32),
    "pcamg_gs": ([_i32, _p, _p, _p, _p, _p, _i32, _p, _p, _i32, _i32, _p], _i32),
    "pcamg_residual": ([_i32, _p, _p, _p, _p, _p, _p, _p, _p], _i32),
    "pcamg_a2_count": ([_i32, _p, _p, _i32, _p, C.POINTER(_i64), _p], _i32),
    "pcamg_a2_fill": ([_i32, _p, _p, _i32, _p, _p, _p], _i32),
    "pcamg_sort_edges": ([_i32, _p, _p, _p, _p, _p, _p], _i32),
    "pcamg_path_cover": ([_i32, _i32, _p, _p, _p, _p], _i32),
    "pcamg_orient": ([_i32, _p, _p, _p, _p, _p], _i32),
    "pcamg_orient_noalloc": ([_i32, _p, _p, _p, _p, _p], _i32),
    "pcamg_aggregate": ([_i32, _p, _p, _p, _p, _p, _p, C.POINTER(_i32), _p, _p], _i32),
    "pcamg_mwm_aggregate": ([_i32, _p, _p, _p, _p, C.POINTER(_i32), _p, _p], _i32),
    "pcamg_galerkin_count": ([_i32, _p, _p, _i32, _p, _p, C.POINTER(_i64), _p], _i32),
    "pcamg_galerkin_fill": ([_i32, _p, _p, _p, _p, _i32, _p, _p, _p, _p, _p, _p, _p], _i32),
    "pcamg_shorten": ([_i32, _p, _i32, _p, _p, _p], _i32),
}

EXPORTED = sorted(_SIGS)


def lib():
    """Load libpcamg.so (built by paper_1806_07028_amd/build.py).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_1806_07028_amd/build.py` "
                           "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int):
    if status != 0:
        raise PcamgError(status, lib().pcamg_last_error().decode())


def default_params(**kw) -> Params:
    p = Params()
    check(lib().pcamg_params_default(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def stats_dict(st: Stats, hist: np.ndarray | None = None) -> dict:
    d = {f: getattr(st, f) for f, _ in Stats._fields_ if f not in ("relres_hist", "hist_cap")}
    if hist is not None:
        d["relres_hist"] = hist[: st.hist_len].copy()
    return d
