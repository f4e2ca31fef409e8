"""Parity at the benchmark's full size: the 7-point 128^3 weighted grid
(2,097,152 vertices, weights 10^(-3+6u)) with the benchmark's settings and
launch configuration -- FCG with FP32 cycles, red-black finest level on its
sliced-ELL copy, XCD-contiguous tiles, single-workgroup tail, captured graphs
and the dense W operator built from the coarsest up.

Bars: the first hierarchy and an FP32 V-cycle (recursive) bit for bit against
the oracle (the oracle builds the 128^3 hierarchy in about ten seconds); the
FP32 W-cycle and the default FP32 V-cycle through their dense operators within
1e-5 relative of the oracle's FP32 recursion (a dense operator changes the
rounding order only)."""
import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I
from test_gpu_parity import compare_hierarchy, host, same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full(gpu, oracle):
    g, b = I.config2(side=128)
    n, rp, ci, w = g
    print(f"fullsize: 128^3 grid, n={n}, edges={len(ci) // 2}", flush=True)
    # V-cycles recurse here (bit for bit); the default dense V operator below
    s = gpu.Solver(rp, ci, w, b, outer="fcg", cycle_prec="f32", theta=0.5, keep_setup=1, v_dense_max_n=0)
    H = oracle.Hierarchy(g, None)
    return g, b, s, H


def test_fullsize_first_hierarchy(full):
    g, b, s, H = full
    same(host(s.initial_error()), H.get_dbl(0, "e"))
    compare_hierarchy(s, H)


def test_fullsize_finest_level_red_black(full):
    g, b, s, H = full
    info = s.level_info(0)
    assert info["n"] == 128 ** 3 and info["ncolours"] == 2
    col = s.level_get(0, "colour")
    v = np.arange(128 ** 3)
    assert np.array_equal(col, (v % 128 + (v // 128) % 128 + v // 16384) % 2)


def test_fullsize_vcycle32(full):
    g, b, s, H = full
    b32 = b.astype(np.float32)
    same(host(s.cycle32(b32)), H.vcycle32(b32))


def test_fullsize_wcycle32_dense(full):
    g, b, s, H = full
    b32 = b.astype(np.float32)
    got = host(s.cycle32(b32, None, 2)).astype(np.float64)
    ref = H.cycle32(b32, None, 2).astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def test_fullsize_vcycle32_dense(full):
    """The benchmark's default: the V-cycle below the first level of at most
    2048 vertices applied as one dense operator, within 1e-5 relative of the
    oracle's FP32 recursion."""
    g, b, s, H = full
    import paper_1806_07028_amd as P
    n, rp, ci, w = g
    sd = P.Solver(rp, ci, w, b, outer="fcg", cycle_prec="f32", theta=0.5)
    b32 = b.astype(np.float32)
    got = host(sd.cycle32(b32)).astype(np.float64)
    ref = H.vcycle32(b32).astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    assert not np.array_equal(got, ref)
