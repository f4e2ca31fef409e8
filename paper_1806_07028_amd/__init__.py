"""PC-alphaAMG on MI355X: path-cover adaptive AMG for weighted graph Laplacians.

Python front end of libpcamg.so (HIP kernels for gfx950 behind a C ABI,
include/pcamg.h).  Torch tensors provide device memory and the current stream;
nothing here computes -- every step runs in the library.

    from paper_1806_07028_amd import Solver
    s = Solver(row_ptr, col_idx, weight, rhs, outer="fcg", cycle_prec="f32", theta=0.5)
    x, stats = s.solve()
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import PcamgError, default_params, lib

__all__ = ["Solver", "batch_solve", "PcamgError", "lib", "default_params", "stages", "learned"]

_OUTER = {"vcycle": 0, "fcg": 1}
_PREC = {"f64": 0, "f32": 1}
_P1 = {"smooth": 0, "const": 1}
_COARSE = {"auto": 0, "grounded": 1, "full": 2}
_SOURCE = {"error": 0, "relax": 1, "iterate": 2}
_INIT = {"relax": 0, "mwm": 1}


def _ptr(t: torch.Tensor | None, dtype: torch.dtype | None = None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _params(kw: dict) -> _lib.Params:
    maps = {"outer": _OUTER, "cycle_prec": _PREC, "p1_mode": _P1, "coarse_solve": _COARSE,
            "rebuild_source": _SOURCE, "init": _INIT}
    conv = {}
    for k, v in kw.items():
        if k in maps and isinstance(v, str):
            v = maps[k][v]
        conv[k] = v
    return default_params(**conv)


def _dev(a, dtype) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


class Solver:
    """One graph Laplacian: setup on construction (first hierarchy), then solve."""

    def __init__(self, row_ptr, col_idx, weight, rhs=None, net=None, **params):
        """net: a learned.Net whose proposal replaces the first build's relaxation."""
        self.row_ptr = _dev(row_ptr, torch.int32)
        self.col_idx = _dev(col_idx, torch.int32)
        self.weight = _dev(weight, torch.float64)
        self.n = self.row_ptr.numel() - 1
        self.p = _params(params)
        g = _lib.Graph(self.n, self.col_idx.numel(), _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.weight))
        self.rhs = None if rhs is None else _dev(rhs, torch.float64)
        h = C.c_void_p()
        if net is None:
            _lib.check(lib().pcamg_setup(C.byref(g), _ptr(self.rhs), C.byref(self.p), _stream(), C.byref(h)))
        else:
            _lib.check(lib().pcamg_setup_learned(C.byref(g), _ptr(self.rhs), C.byref(self.p), net.h, _stream(),
                                                 C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().pcamg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_rhs(self, rhs):
        self.rhs = _dev(rhs, torch.float64)
        _lib.check(lib().pcamg_set_rhs(self.h, _ptr(self.rhs)))

    def solve(self, x0=None, raise_on_noconv: bool = True):
        x = torch.zeros(self.n, dtype=torch.float64, device="cuda") if x0 is None else _dev(x0, torch.float64).clone()
        st = _lib.Stats()
        cap = self.p.max_iter + 2
        hist = np.zeros(cap)
        st.relres_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        st.hist_cap = cap
        status = lib().pcamg_solve(self.h, _ptr(x), C.byref(st))
        if status != 0 and (raise_on_noconv or status != -10):
            _lib.check(status)
        return x, _lib.stats_dict(st, hist)

    def rebuild(self, e=None):
        et = None if e is None else _dev(e, torch.float64)
        _lib.check(lib().pcamg_rebuild(self.h, _ptr(et)))

    @property
    def num_hierarchies(self) -> int:
        c = C.c_int32()
        _lib.check(lib().pcamg_num_hierarchies(self.h, C.byref(c)))
        return c.value

    def num_levels(self, h: int = -1) -> int:
        h = self._h(h)
        c = C.c_int32()
        _lib.check(lib().pcamg_num_levels(self.h, h, C.byref(c)))
        return c.value

    def _h(self, h):
        return self.num_hierarchies + h if h < 0 else h

    INFO_KEYS = ["n", "nnz", "ncolours", "nc", "nnz_G", "npaths", "n_unagg", "case1", "case2", "case3", "middle",
                 "singleton", "p1_fallback", "grounded", "coarse_fallback", "n_path_vertices"]

    def level_info(self, level: int, h: int = -1) -> dict:
        out = (C.c_int64 * 16)()
        _lib.check(lib().pcamg_level_info(self.h, self._h(h), level, out))
        return dict(zip(self.INFO_KEYS, list(out)))

    _INT_NAMES = {"colour", "agg", "A_rp", "A_ci", "path_id", "pos", "nb", "G_rp", "G_ci"}

    def level_get(self, level: int, name: str, h: int = -1) -> np.ndarray:
        inf = self.level_info(level, h)
        n, nnz, nG = inf["n"], inf["nnz"], inf["nnz_G"]
        size = {"colour": n, "agg": n, "A_rp": n + 1, "A_ci": nnz, "path_id": n, "pos": n, "nb": 2 * n,
                "G_rp": n + 1, "G_ci": nG, "A_v": nnz, "d": n, "dinv": n, "pval": n, "G_v": nG, "gkey": nG,
                "source": n}[name]
        out = np.empty(max(size, 1), dtype=np.int32 if name in self._INT_NAMES else np.float64)
        _lib.check(lib().pcamg_level_get(self.h, self._h(h), level, name.encode(), out.ctypes.data))
        return out[:size]

    def cycle(self, b, x=None, gamma: int = 1, h: int = -1) -> torch.Tensor:
        b = _dev(b, torch.float64)
        x = torch.zeros_like(b) if x is None else _dev(x, torch.float64).clone()
        _lib.check(lib().pcamg_cycle(self.h, self._h(h), _ptr(b), _ptr(x), gamma))
        return x

    def cycle32(self, b, x=None, gamma: int = 1, h: int = -1) -> torch.Tensor:
        b = _dev(b, torch.float32)
        x = torch.zeros_like(b) if x is None else _dev(x, torch.float32).clone()
        _lib.check(lib().pcamg_cycle32(self.h, self._h(h), _ptr(b), _ptr(x), gamma))
        return x

    def approx_error(self, r, count: int | None = None) -> torch.Tensor:
        r = _dev(r, torch.float64)
        e = torch.empty_like(r)
        _lib.check(lib().pcamg_approx_error(self.h, count or self.num_hierarchies, _ptr(r), _ptr(e)))
        return e

    def initial_error(self) -> torch.Tensor:
        e = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _lib.check(lib().pcamg_initial_error(self.h, _ptr(e)))
        return e


def batch_solve(graphs, rhs, x0=None, workers: int = 1, raise_on_error: bool = True, **params):
    """Set up and solve many independent graphs (pcamg_batch_solve): graphs is a
    list of (row_ptr, col_idx, weight), rhs a list of right-hand sides.
    workers must be 1 (the default): the graphs are solved one after another on
    the calling thread; several workers are refused by the library.
    Returns (list of solutions, list of statistics dicts)."""
    count = len(graphs)
    p = _params(params)
    keep = []
    garr = (_lib.Graph * max(count, 1))()
    barr = (C.c_void_p * max(count, 1))()
    xarr = (C.c_void_p * max(count, 1))()
    xs = []
    hists = []
    starr = (_lib.Stats * max(count, 1))()
    for g, ((rp, ci, w), b) in enumerate(zip(graphs, rhs)):
        rp, ci, w, b = _dev(rp, torch.int32), _dev(ci, torch.int32), _dev(w, torch.float64), _dev(b, torch.float64)
        n = rp.numel() - 1
        x = torch.zeros(n, dtype=torch.float64, device="cuda") if x0 is None else _dev(x0[g], torch.float64).clone()
        keep += [rp, ci, w, b]
        xs.append(x)
        garr[g] = _lib.Graph(n, ci.numel(), _ptr(rp), _ptr(ci), _ptr(w))
        barr[g] = _ptr(b)
        xarr[g] = _ptr(x)
        hist = np.zeros(p.max_iter + 2)
        hists.append(hist)
        starr[g].relres_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        starr[g].hist_cap = p.max_iter + 2
    torch.cuda.synchronize()  # inputs are read on the library's own streams
    status = lib().pcamg_batch_solve(garr, barr, xarr, count, C.byref(p), workers, starr)
    if status != 0 and raise_on_error:
        _lib.check(status)
    return xs, [_lib.stats_dict(starr[g], hists[g]) for g in range(count)]


from . import learned, stages  # noqa: E402
