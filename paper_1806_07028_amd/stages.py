"""Single steps of the method on caller tensors (parity tests and benchmarks).

Each function marshals torch tensors into one stage entry point of the C ABI
(include/pcamg.h) and returns device tensors; natural vertex order throughout.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import lib

i32, f64 = torch.int32, torch.float64


def _s():
    return torch.cuda.current_stream().cuda_stream


def _d(a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(a, dtype=dtype, device="cuda").contiguous()


def _e(n, dtype):
    return torch.empty(max(int(n), 1), dtype=dtype, device="cuda")


def laplacian(rp, ci, w):
    rp, ci, w = _d(rp, i32), _d(ci, i32), _d(w, f64)
    n = rp.numel() - 1
    a, d, dinv = _e(ci.numel(), f64), _e(n, f64), _e(n, f64)
    _lib.check(lib().pcamg_laplacian(n, rp.data_ptr(), ci.data_ptr(), w.data_ptr(), a.data_ptr(), d.data_ptr(),
                                     dinv.data_ptr(), _s()))
    return a[: ci.numel()], d[:n], dinv[:n]


def colour(rp, ci, seed: int, level: int = 0):
    rp, ci = _d(rp, i32), _d(ci, i32)
    n = rp.numel() - 1
    c = _e(n, i32)
    nc = C.c_int32()
    _lib.check(lib().pcamg_colour(n, rp.data_ptr(), ci.data_ptr(), seed, level, c.data_ptr(), C.byref(nc), _s()))
    return c[:n], nc.value


def gs(rp, ci, aval, dinv, col, ncol: int, b, x, forward=True, count=1):
    rp, ci, aval, dinv, col = _d(rp, i32), _d(ci, i32), _d(aval, f64), _d(dinv, f64), _d(col, i32)
    b = _d(b, f64)
    x = _d(x, f64).clone()
    n = rp.numel() - 1
    _lib.check(lib().pcamg_gs(n, rp.data_ptr(), ci.data_ptr(), aval.data_ptr(), dinv.data_ptr(), col.data_ptr(),
                              ncol, b.data_ptr(), x.data_ptr(), int(forward), count, _s()))
    return x


def residual(rp, ci, aval, d, b, x):
    rp, ci, aval, d, b, x = _d(rp, i32), _d(ci, i32), _d(aval, f64), _d(d, f64), _d(b, f64), _d(x, f64)
    n = rp.numel() - 1
    r = _e(n, f64)
    _lib.check(lib().pcamg_residual(n, rp.data_ptr(), ci.data_ptr(), aval.data_ptr(), d.data_ptr(), b.data_ptr(),
                                    x.data_ptr(), r.data_ptr(), _s()))
    return r[:n]


def a2_pattern(rp, ci, hub_cap: int = 0):
    rp, ci = _d(rp, i32), _d(ci, i32)
    n = rp.numel() - 1
    rp2 = _e(n + 1, i32)
    nnz2 = C.c_int64()
    _lib.check(lib().pcamg_a2_count(n, rp.data_ptr(), ci.data_ptr(), hub_cap, rp2.data_ptr(), C.byref(nnz2), _s()))
    ci2 = _e(nnz2.value, i32)
    _lib.check(lib().pcamg_a2_fill(n, rp.data_ptr(), ci.data_ptr(), hub_cap, rp2.data_ptr(), ci2.data_ptr(), _s()))
    return rp2, ci2[: nnz2.value]


def sort_edges(rp2, ci2, e):
    rp2, ci2, e = _d(rp2, i32), _d(ci2, i32), _d(e, f64)
    n = rp2.numel() - 1
    m = ci2.numel() // 2
    su, sv = _e(m, i32), _e(m, i32)
    _lib.check(lib().pcamg_sort_edges(n, rp2.data_ptr(), ci2.data_ptr(), e.data_ptr(), su.data_ptr(), sv.data_ptr(),
                                      _s()))
    return su[:m], sv[:m]


def path_cover(n: int, su, sv):
    su, sv = _d(su, i32), _d(sv, i32)
    nb = _e(2 * n, i32)
    _lib.check(lib().pcamg_path_cover(n, su.numel(), su.data_ptr(), sv.data_ptr(), nb.data_ptr(), _s()))
    return nb[: 2 * n].view(n, 2)


def orient(nb):
    nb = _d(nb, i32).reshape(-1)
    n = nb.numel() // 2
    pid, pos, plen = _e(n, i32), _e(n, i32), _e(n, i32)
    _lib.check(lib().pcamg_orient(n, nb.data_ptr(), pid.data_ptr(), pos.data_ptr(), plen.data_ptr(), _s()))
    return pid[:n], pos[:n], plen[:n]


def aggregate(grp, gci, gw, nb, gkey=None):
    grp, gci, gw = _d(grp, i32), _d(gci, i32), _d(gw, f64)
    nb = _d(nb, i32).reshape(-1)
    n = grp.numel() - 1
    gk = None if gkey is None else _d(gkey, f64)
    agg = _e(n, i32)
    nc = C.c_int32()
    stats = (C.c_int32 * 6)()
    _lib.check(lib().pcamg_aggregate(n, grp.data_ptr(), gci.data_ptr(), gw.data_ptr(),
                                     None if gk is None else gk.data_ptr(), nb.data_ptr(), agg.data_ptr(),
                                     C.byref(nc), stats, _s()))
    keys = ["n_unagg", "case1", "case2", "case3", "middle", "singleton"]
    return agg[:n], nc.value, dict(zip(keys, list(stats)))


def galerkin(rp, ci, aval, d, nc: int, agg, pval):
    rp, ci, aval, d, agg, pval = _d(rp, i32), _d(ci, i32), _d(aval, f64), _d(d, f64), _d(agg, i32), _d(pval, f64)
    n = rp.numel() - 1
    rpc = _e(nc + 1, i32)
    nnzc = C.c_int64()
    _lib.check(lib().pcamg_galerkin_count(n, rp.data_ptr(), ci.data_ptr(), nc, agg.data_ptr(), rpc.data_ptr(),
                                          C.byref(nnzc), _s()))
    cic, vc, dc = _e(nnzc.value, i32), _e(nnzc.value, f64), _e(nc, f64)
    _lib.check(lib().pcamg_galerkin_fill(n, rp.data_ptr(), ci.data_ptr(), aval.data_ptr(), d.data_ptr(), nc,
                                         agg.data_ptr(), pval.data_ptr(), rpc.data_ptr(), cic.data_ptr(),
                                         vc.data_ptr(), dc.data_ptr(), _s()))
    k = nnzc.value
    return rpc[: nc + 1], cic[:k], vc[:k], dc[:nc]


def shorten(nb, nc: int, agg):
    nb = _d(nb, i32).reshape(-1)
    agg = _d(agg, i32)
    n = nb.numel() // 2
    nbc = _e(2 * nc, i32)
    _lib.check(lib().pcamg_shorten(n, nb.data_ptr(), nc, agg.data_ptr(), nbc.data_ptr(), _s()))
    return nbc[: 2 * nc].view(nc, 2)


def mwm_aggregate(rp, ci, aval):
    """MWM aggregation (Sec. 2.1) of a level with off-diagonal entries aval."""
    rp, ci, aval = _d(rp, i32), _d(ci, i32), _d(aval, f64)
    n = rp.numel() - 1
    agg = _e(n, i32)
    nc = C.c_int32()
    stats = (C.c_int32 * 3)()
    _lib.check(lib().pcamg_mwm_aggregate(n, rp.data_ptr(), ci.data_ptr(), aval.data_ptr(), agg.data_ptr(),
                                         C.byref(nc), stats, _s()))
    return agg[:n], nc.value, dict(zip(["n_unagg", "joined", "singleton"], list(stats)))
