"""CPU oracle for PC-alphaAMG -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper over ``liboracle.so`` (built from ``pcamg_oracle.cpp`` by
``oracle/build.py``).  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the HIP library never
does.  See ``pcamg_oracle.cpp`` for the algorithm and the readings of the paper.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force, invariants stated in the paper and hand
worked examples, except the iteration/rebuild *counts* of the adaptive loop,
which the paper's tables do not fix for these readings (parity unpinned; only
the final answer of the loop is pinned, against a dense pseudo-inverse solve).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


class OracleParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("theta", C.c_double),
        ("max_iter", C.c_int),
        ("outer", C.c_int),
        ("cycle_prec", C.c_int),
        ("coarse_max", C.c_int),
        ("relax_sweeps", C.c_int),
        ("rebuild_vcycles", C.c_int),
        ("rebuild_source", C.c_int),
        ("p1_mode", C.c_int),
        ("coarse_solve", C.c_int),
        ("a2_hub_cap", C.c_int),
        ("max_rebuilds", C.c_int),
        ("max_levels", C.c_int),
        ("numW", C.c_int),
        ("iterW", C.c_int),
        ("iterV", C.c_int),
        ("rebuild_rule", C.c_int),
        ("seed", C.c_ulonglong),
        ("colour_seed", C.c_ulonglong),
        ("case3", C.c_int),
        ("init", C.c_int),
    ]


DEFAULTS = dict(tol=1e-8, theta=0.4, max_iter=2500, outer=0, cycle_prec=0, coarse_max=64, relax_sweeps=3,
                rebuild_vcycles=2, rebuild_source=0, p1_mode=0, coarse_solve=0, a2_hub_cap=0, max_rebuilds=50,
                max_levels=64, numW=2, iterW=7, iterV=4, rebuild_rule=0, seed=0x5EED, colour_seed=0xC010,
                case3=0, init=0)


def params(**kw) -> OracleParams:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return OracleParams(**d)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (oracle/build.py)
        _b.build()
    L = C.CDLL(_LIB_PATH)
    L.or_last_error.restype = C.c_char_p
    L.or_xi.argtypes = [C.c_int, C.c_ulonglong, C.c_int, _f64p]
    L.or_colour_priority.argtypes = [C.c_ulonglong, C.c_int, C.c_int]
    L.or_colour_priority.restype = C.c_ulonglong
    L.or_colour_key.argtypes = [C.c_ulonglong, C.c_int, C.c_int, C.c_int]
    L.or_colour_key.restype = C.c_ulonglong
    L.or_laplacian.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
    L.or_colour.argtypes = [C.c_int, _i32p, _i32p, C.c_ulonglong, C.c_int, _i32p]
    L.or_colour.restype = C.c_int
    L.or_colour_greedy.argtypes = [C.c_int, _i32p, _i32p, C.c_ulonglong, C.c_int, _i32p]
    L.or_colour_greedy.restype = C.c_int
    L.or_gs.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _i32p, C.c_int, _f64p, _f64p, C.c_int, C.c_int]
    L.or_gs32.argtypes = [C.c_int, _i32p, _i32p, _f32p, _f32p, _i32p, C.c_int, _f32p, _f32p, C.c_int]
    L.or_residual.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
    L.or_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
    L.or_smooth_error.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_ulonglong, C.c_ulonglong, C.c_int, _f64p]
    L.or_a2_count.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p]
    L.or_a2_count.restype = C.c_longlong
    L.or_a2_fill.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p]
    L.or_sorted_edges.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p]
    L.or_path_cover.argtypes = [C.c_int, C.c_int, _i32p, _i32p, _i32p]
    L.or_orient.argtypes = [C.c_int, _i32p, _i32p, _i32p, _i32p]
    L.or_orient.restype = C.c_int
    L.or_aggregate.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, _i32p, C.c_int, _i32p, _i32p]
    L.or_aggregate.restype = C.c_int
    L.or_mwm_aggregate.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p]
    L.or_mwm_aggregate.restype = C.c_int
    L.or_hier_build.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_void_p, C.POINTER(OracleParams)]
    L.or_hier_build.restype = C.c_void_p
    L.or_hier_free.argtypes = [C.c_void_p]
    L.or_hier_levels.argtypes = [C.c_void_p]
    L.or_hier_levels.restype = C.c_int
    L.or_hier_info.argtypes = [C.c_void_p, C.c_int, _i64p]
    L.or_hier_oc.argtypes = [C.c_void_p]
    L.or_hier_oc.restype = C.c_double
    L.or_hier_get_int.argtypes = [C.c_void_p, C.c_int, C.c_char_p, _i32p]
    L.or_hier_get_int.restype = C.c_int
    L.or_hier_get_dbl.argtypes = [C.c_void_p, C.c_int, C.c_char_p, _f64p]
    L.or_hier_get_dbl.restype = C.c_int
    L.or_hier_vcycle.argtypes = [C.c_void_p, _f64p, _f64p]
    L.or_hier_vcycle32.argtypes = [C.c_void_p, _f32p, _f32p]
    L.or_hier_coarsest_solve.argtypes = [C.c_void_p, _f64p, _f64p]
    L.or_hier_cycle.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int]
    L.or_hier_cycle32.argtypes = [C.c_void_p, _f32p, _f32p, C.c_int]
    L.or_approx_error.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(OracleParams), _f64p, _f64p]
    L.or_hier_relax_error.argtypes = [C.c_void_p, C.POINTER(OracleParams), C.c_int, _f64p]
    L.or_galerkin.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, _i32p, _f64p, _i32p, C.c_void_p,
                              C.c_void_p, C.c_void_p]
    L.or_galerkin.restype = C.c_longlong
    L.or_shorten.argtypes = [C.c_int, _i32p, C.c_int, _i32p, _i32p]
    L.or_solve.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.POINTER(OracleParams), C.c_void_p, _f64p,
                           _f64p, _f64p, C.c_int, _i32p, C.c_int]
    L.or_solve.restype = C.c_int
    _lib = L
    return L


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _err():
    return lib().or_last_error().decode()


# ----------------------------------------------------------------------------
# Stage functions
# ----------------------------------------------------------------------------

def xi(n: int, seed: int, r: int) -> np.ndarray:
    out = np.empty(n)
    lib().or_xi(n, seed, r, out)
    return out


def colour_priority(seed: int, level: int, v: int) -> int:
    return int(lib().or_colour_priority(seed, level, v))


def colour_key(seed: int, level: int, v: int, deg: int) -> int:
    return int(lib().or_colour_key(seed, level, v, deg))


def laplacian(g):
    n, rp, ci, w = g
    a = np.empty(len(ci))
    d = np.empty(n)
    dinv = np.empty(n)
    lib().or_laplacian(n, _i32(rp), _i32(ci), _f64(w), a, d, dinv)
    return a, d, dinv


def colour(n, rp, ci, seed: int, level: int = 0):
    """The smoother's colouring of a level graph: red-black on a connected
    bipartite graph, greedy first-fit in priority order otherwise."""
    c = np.empty(n, dtype=np.int32)
    nc = lib().or_colour(n, _i32(rp), _i32(ci), seed, level, c)
    return c, nc


def colour_greedy(n, rp, ci, seed: int, level: int = 0):
    """Greedy first-fit in descending (key, id) order, whatever the graph
    (key: degree, then the random word)."""
    c = np.empty(n, dtype=np.int32)
    nc = lib().or_colour_greedy(n, _i32(rp), _i32(ci), seed, level, c)
    return c, nc


def gs(n, rp, ci, aval, dinv, colour_, ncol, b, x, forward=True, count=1):
    x = _f64(x).copy()
    lib().or_gs(n, _i32(rp), _i32(ci), _f64(aval), _f64(dinv), _i32(colour_), ncol, _f64(b), x, int(forward), count)
    return x


def gs32(n, rp, ci, aval32, dinv32, colour_, ncol, b32, x32, forward=True):
    x = np.ascontiguousarray(x32, dtype=np.float32).copy()
    lib().or_gs32(n, _i32(rp), _i32(ci), np.ascontiguousarray(aval32, np.float32),
                  np.ascontiguousarray(dinv32, np.float32), _i32(colour_), ncol,
                  np.ascontiguousarray(b32, np.float32), x, int(forward))
    return x


def residual(n, rp, ci, aval, d, b, x):
    r = np.empty(n)
    lib().or_residual(n, _i32(rp), _i32(ci), _f64(aval), _f64(d), _f64(b), _f64(x), r)
    return r


def spmv(n, rp, ci, aval, d, p):
    q = np.empty(n)
    lib().or_spmv(n, _i32(rp), _i32(ci), _f64(aval), _f64(d), _f64(p), q)
    return q


def smooth_error(g, colour_seed: int, seed: int, sweeps: int = 3) -> np.ndarray:
    n, rp, ci, w = g
    e = np.empty(n)
    lib().or_smooth_error(n, _i32(rp), _i32(ci), _f64(w), colour_seed, seed, sweeps, e)
    return e


def a2_pattern(n, rp, ci, cap: int = 0):
    rp2 = np.empty(n + 1, dtype=np.int32)
    nnz2 = lib().or_a2_count(n, _i32(rp), _i32(ci), cap, rp2)
    ci2 = np.empty(nnz2, dtype=np.int32)
    lib().or_a2_fill(n, _i32(rp), _i32(ci), cap, ci2)
    return rp2, ci2


def sorted_edges(n, rp2, ci2, e):
    m = int((np.asarray(ci2) > np.repeat(np.arange(n), np.diff(rp2))).sum())
    su = np.empty(m, dtype=np.int32)
    sv = np.empty(m, dtype=np.int32)
    lib().or_sorted_edges(n, _i32(rp2), _i32(ci2), _f64(e), su, sv)
    return su, sv


def path_cover(n, su, sv):
    nb = np.empty(2 * n, dtype=np.int32)
    lib().or_path_cover(n, len(su), _i32(su), _i32(sv), nb)
    return nb.reshape(n, 2)


def orient(nb):
    nb = _i32(np.asarray(nb).reshape(-1))
    n = len(nb) // 2
    pid = np.empty(n, dtype=np.int32)
    pos = np.empty(n, dtype=np.int32)
    plen = np.empty(n, dtype=np.int32)
    np_ = lib().or_orient(n, nb, pid, pos, plen)
    return pid, pos, plen, np_


def aggregate(n, grp, gci, gw, nb, gkey=None, case3: int = 0):
    """Alg. 3 on one level.  case3 = 0: the connected reading of Case 3 (v
    stays when taking it out would split its aggregate; u joins there);
    case3 = 1: Step 17 as printed (v always leaves)."""
    agg = np.empty(n, dtype=np.int32)
    stats = np.empty(6, dtype=np.int32)
    keyp = None
    if gkey is not None:
        gkey = _f64(gkey)
        keyp = gkey.ctypes.data_as(C.c_void_p)
    nc = lib().or_aggregate(n, _i32(grp), _i32(gci), _f64(gw), keyp, _i32(np.asarray(nb).reshape(-1)), case3,
                            agg, stats)
    return agg, nc, dict(zip(["n_unagg", "case1", "case2", "case3", "middle", "singleton"], stats.tolist()))


def mwm_aggregate(n, rp, ci, aval):
    """MWM aggregation (Sec. 2.1) of a level with off-diagonal entries aval
    (weights -aval): (agg, nc, stats)."""
    agg = np.empty(n, dtype=np.int32)
    stats = np.empty(3, dtype=np.int32)
    nc = lib().or_mwm_aggregate(n, _i32(rp), _i32(ci), _f64(aval), agg, stats)
    return agg, nc, dict(zip(["n_unagg", "joined", "singleton"], stats.tolist()))


def galerkin(n, rp, ci, aval, d, nc, agg, pval):
    """Coarse operator P^T A P: (rp_c, ci_c, off-diagonal values, diagonal)."""
    rpc = np.empty(nc + 1, dtype=np.int32)
    args = (n, _i32(rp), _i32(ci), _f64(aval), _f64(d), nc, _i32(agg), _f64(pval))
    nnz = lib().or_galerkin(*args, rpc, None, None, None)
    cic = np.empty(max(nnz, 1), dtype=np.int32)
    vc = np.empty(max(nnz, 1))
    dc = np.empty(nc)
    lib().or_galerkin(*args, rpc, cic.ctypes.data_as(C.c_void_p), vc.ctypes.data_as(C.c_void_p),
                      dc.ctypes.data_as(C.c_void_p))
    return rpc, cic[:nnz], vc[:nnz], dc


def shorten(nb, nc, agg):
    nb = _i32(np.asarray(nb).reshape(-1))
    n = len(nb) // 2
    out = np.empty(2 * nc, dtype=np.int32)
    lib().or_shorten(n, nb, nc, _i32(agg), out)
    return out.reshape(nc, 2)


# ----------------------------------------------------------------------------
# Hierarchy
# ----------------------------------------------------------------------------

INFO_KEYS = ["n", "nnz", "ncolours", "nc", "nnz_G", "npaths", "n_unagg", "case1", "case2", "case3", "middle",
             "singleton", "p1_fallback", "grounded", "coarse_fallback", "n_path_vertices"]


class Hierarchy:
    """An oracle hierarchy built from a graph and a smooth error (or the first-build error)."""

    def __init__(self, g, e=None, **kw):
        n, rp, ci, w = g
        self.n = n
        self.p = params(**kw)
        self._keep = (_i32(rp), _i32(ci), _f64(w))
        ep = None
        if e is not None:
            self._e = _f64(e)
            ep = self._e.ctypes.data_as(C.c_void_p)
        h = lib().or_hier_build(n, self._keep[0], self._keep[1], self._keep[2], ep, C.byref(self.p))
        if not h:
            raise RuntimeError("oracle build failed: " + _err())
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_hier_free(h)
            self.h = None

    @property
    def nlevels(self) -> int:
        return lib().or_hier_levels(self.h)

    @property
    def op_complexity(self) -> float:
        return lib().or_hier_oc(self.h)

    def info(self, level: int) -> dict:
        out = np.empty(16, dtype=np.int64)
        lib().or_hier_info(self.h, level, out)
        return dict(zip(INFO_KEYS, out.tolist()))

    def _size(self, level, name):
        inf = self.info(level)
        n, nnz, nc, nG = inf["n"], inf["nnz"], inf["nc"], inf["nnz_G"]
        return {"colour": n, "agg": n if nc else 0, "path_id": n, "pos": n, "nb": 2 * n, "A_rp": n + 1,
                "A_ci": nnz, "G_rp": n + 1, "G_ci": nG, "moff": nc + 1 if nc else 0, "mem": n if nc else 0,
                "A_v": nnz, "d": n, "dinv": n, "pval": n if nc else 0, "G_v": nG, "gkey": nG if level == 0 else 0,
                "e": self.n}[name]

    def get_int(self, level: int, name: str) -> np.ndarray:
        out = np.empty(max(self._size(level, name), 1), dtype=np.int32)
        k = lib().or_hier_get_int(self.h, level, name.encode(), out)
        if k < 0:
            raise KeyError(name)
        return out[:k]

    def get_dbl(self, level: int, name: str) -> np.ndarray:
        out = np.empty(max(self._size(level, name), 1))
        k = lib().or_hier_get_dbl(self.h, level, name.encode(), out)
        if k < 0:
            raise KeyError(name)
        return out[:k]

    def level_matrix(self, level: int):
        """(rp, ci, off-diagonal values, diagonal) of A_level."""
        return (self.get_int(level, "A_rp"), self.get_int(level, "A_ci"), self.get_dbl(level, "A_v"),
                self.get_dbl(level, "d"))

    def vcycle(self, b, x=None) -> np.ndarray:
        x = np.zeros(self.n) if x is None else _f64(x).copy()
        lib().or_hier_vcycle(self.h, _f64(b), x)
        return x

    def vcycle32(self, b32, x32=None) -> np.ndarray:
        x = np.zeros(self.n, np.float32) if x32 is None else np.ascontiguousarray(x32, np.float32).copy()
        lib().or_hier_vcycle32(self.h, np.ascontiguousarray(b32, np.float32), x)
        return x

    def coarsest_solve(self, b) -> np.ndarray:
        b = _f64(b)
        x = np.zeros(len(b))
        lib().or_hier_coarsest_solve(self.h, b, x)
        return x

    def cycle(self, b, x=None, gamma: int = 1) -> np.ndarray:
        x = np.zeros(self.n) if x is None else _f64(x).copy()
        lib().or_hier_cycle(self.h, _f64(b), x, gamma)
        return x

    def cycle32(self, b32, x32=None, gamma: int = 1) -> np.ndarray:
        x = np.zeros(self.n, np.float32) if x32 is None else np.ascontiguousarray(x32, np.float32).copy()
        lib().or_hier_cycle32(self.h, np.ascontiguousarray(b32, np.float32), x, gamma)
        return x

    def relax_error(self, r: int) -> np.ndarray:
        """Homogeneous rebuild vector of build r (fresh start, V-cycles on A e = 0, sweeps)."""
        e = np.empty(self.n)
        lib().or_hier_relax_error(self.h, C.byref(self.p), r, e)
        return e


def approximate_error(hierarchies, r, **kw) -> np.ndarray:
    """Alg. 2 with ``hierarchies`` as the history (Re = len(hierarchies))."""
    p = params(**kw)
    arr = (C.c_void_p * len(hierarchies))(*[h.h for h in hierarchies])
    e = np.empty(hierarchies[0].n)
    lib().or_approx_error(arr, len(hierarchies), C.byref(p), _f64(r), e)
    return e


STAT_KEYS = ["iterations", "rebuilds", "status", "levels", "relres", "true_relres", "rho_geo", "convr_last10",
             "oc_mean", "t_setup", "t_solve", "first_levels", "first_oc"]


@dataclass
class SolveResult:
    x: np.ndarray
    stats: dict
    relres_hist: np.ndarray
    rebuild_at: np.ndarray


def solve(g, b, x0=None, **kw) -> SolveResult:
    """Adaptive solve from x0 (default 0).  init=1 starts from the MWM
    hierarchy; rebuild_source=2 with rebuild_rule=1 and b = 0 is Alg. 6."""
    n, rp, ci, w = g
    p = params(**kw)
    x = np.empty(n)
    st = np.zeros(13)
    cap = p.max_iter + 2
    hist = np.zeros(cap)
    rb = np.full(p.max_rebuilds + 1, -1, dtype=np.int32)
    x0p = None
    if x0 is not None:
        x0 = _f64(x0)
        x0p = x0.ctypes.data_as(C.c_void_p)
    rc = lib().or_solve(n, _i32(rp), _i32(ci), _f64(w), _f64(b), C.byref(p), x0p, x, st, hist, cap, rb, len(rb))
    if rc != 0:
        raise RuntimeError("oracle solve failed: " + _err())
    stats = dict(zip(STAT_KEYS, st.tolist()))
    for k in ("iterations", "rebuilds", "status", "levels", "first_levels"):
        stats[k] = int(stats[k])
    it = stats["iterations"]
    return SolveResult(x, stats, hist[: it + 1], rb[: stats["rebuilds"]])
