"""The C-ABI library loads and exports every function include/pcamg.h declares
(no GPU needed: no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "pcamg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcamg_[a-z0-9_]+)\s*\(", src)))


def test_header_matches_binding():
    from paper_1806_07028_amd import _lib

    assert declared() == _lib.EXPORTED


def test_library_exports_everything():
    from paper_1806_07028_amd import _lib

    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [f for f in declared() if not hasattr(L, f)]
    assert not missing, missing


def test_params_default_and_struct_layout():
    from paper_1806_07028_amd import _lib

    p = _lib.default_params()
    assert p.tol == 1e-8 and p.max_iter == 2500 and p.coarse_max == 64 and p.relax_sweeps == 3
    assert (p.numW, p.iterW, p.iterV) == (2, 7, 4)
    assert p.seed == 0x5EED and p.colour_seed == 0xC010
    assert ctypes.sizeof(_lib.Params) == 8 + 8 + 26 * 4 + 8 + 8 + 4 * 4
    assert p.case3 == 0 and p.init == 0 and p.block_sweep_min_colours == 0
    assert p.v_dense_max_n == 4096 and p.top_dense_max_n == 0
    assert p.first_sweeps == -1 and p.dense_max_n == 12288 and p.long_row_min == 256 and p.max_levels == 64
    assert p.tail_max_n == 2048 and p.use_graphs == 1 and p.row_lanes == 0 and p.w_dense == 1
    assert _lib.lib().pcamg_status_str(-6) == b"graph not connected"
