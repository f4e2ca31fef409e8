"""Pins of the seeded input generators shared by the oracle and the HIP path.

The generators hold none of the method's arithmetic; these tests check that
they produce the workloads stated for them: the published SplitMix64 stream,
the grid sizes of the 2D 64x64 and 3D 128^3 problems, the CSR invariants every
graph is handed over with, and the shape of the random families (mean degree
of the geometric graphs, the Barabasi-Albert edge count, the heavy tail of the
Chung-Lu degrees, the weight ranges and the zero-mean right-hand sides).
"""
import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I


def test_splitmix64_published_stream():
    # first outputs of SplitMix64 seeded with 1234567 (Vigna's reference
    # implementation): word k is mix(seed + k * golden gamma), k = 1, 2, ...
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [int(x) for x in I.stream_words(1234567, 5)] == want
    # counters address the same stream
    assert [int(x) for x in I.stream_words(1234567, 2, start=3)] == want[3:]
    u = I.uniform_at(1234567, np.arange(1, 6, dtype=np.uint64))
    assert np.array_equal(u, I.uniform(1234567, 5))
    assert np.array_equal(u, (np.array(want, dtype=np.uint64) >> np.uint64(11)) * 2.0 ** -53)


def test_uniform_and_normal_moments():
    u = I.uniform(7, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    z = I.normal(7, 200_001)
    assert z.shape == (200_001,) and np.isfinite(z).all()
    assert abs(z.mean()) < 1e-2 and abs(z.var() - 1.0) < 2e-2
    assert abs(np.mean(z ** 4) - 3.0) < 0.1  # Gaussian kurtosis
    b = I.zero_mean_normal_rhs(7, 1001)
    assert abs(b.sum()) < 1e-10


def check_csr(n, rp, ci, w):
    rp, ci, w = np.asarray(rp), np.asarray(ci), np.asarray(w)
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and w.dtype == np.float64
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == len(ci) == len(w)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert (ci != rows).all(), "diagonal entry"
    assert ((ci >= 0) & (ci < n)).all()
    same_row = rows[1:] == rows[:-1]
    assert (ci[1:][same_row] > ci[:-1][same_row]).all(), "columns not strictly ascending"
    # symmetric, weights bitwise equal on both halves
    fwd = np.lexsort((ci, rows))
    bwd = np.lexsort((rows, ci))
    assert np.array_equal(rows[fwd], ci[bwd]) and np.array_equal(ci[fwd], rows[bwd])
    assert np.array_equal(w[fwd].view(np.uint64), w[bwd].view(np.uint64))
    assert (w > 0).all() and np.isfinite(w).all()
    return rows


def test_grid_workload_sizes():
    (n, rp, ci, w), b = I.config1()
    assert n == 4096 and len(ci) == 2 * 8064  # 2 * 64 * 63 edges
    check_csr(n, rp, ci, w)
    assert (w == 1.0).all() and abs(b.sum()) < 1e-9
    deg = np.diff(rp)
    assert sorted(np.unique(deg).tolist()) == [2, 3, 4]
    # 128^3 7-point grid: 3 * 128^2 * 127 edges
    nv, a, bb = I.grid3d_edges(128, 128, 128)
    assert nv == 2_097_152 and len(a) == 6_242_304
    # a smaller cube through the full CSR path: degrees 3..6, weights in range
    n, rp, ci, w = I.grid3d(9, 8, 7, weight_seed=3)
    assert n == 9 * 8 * 7 and len(ci) == 2 * (8 * 8 * 7 + 9 * 7 * 7 + 9 * 8 * 6)
    check_csr(n, rp, ci, w)
    assert set(np.diff(rp).tolist()) == {3, 4, 5, 6}
    assert w.min() >= 1e-3 and w.max() < 1e3


def test_path_and_ring():
    n, rp, ci, w = I.path(50)
    rows = check_csr(n, rp, ci, w)
    assert len(ci) == 98 and (np.abs(ci - rows) == 1).all()
    n, rp, ci, w = I.ring(40, 4)
    check_csr(n, rp, ci, w)
    assert (np.diff(rp) == 4).all()


def test_random_geometric_mean_degree():
    n, a, b = I.rgg_edges(20_000, 3)
    assert 0.95 * 20_000 < n <= 20_000  # largest component of a supercritical RGG
    assert 7.5 < 2 * len(a) / n < 8.5
    g = I.rgg(5000, 11)
    check_csr(*g)


def test_barabasi_albert_edge_count():
    m = 4
    for n in (10, 3000):
        nv, a, b = I.ba_edges(n, 5, m)
        # K_{m+1} seed plus m distinct targets per later vertex
        assert nv == n and len(a) == (m + 1) * m // 2 + m * (n - m - 1)
        deg = np.bincount(np.concatenate([a, b]), minlength=n)
        assert deg.min() >= m


def test_chung_lu_power_law_shape():
    n0 = 50_000
    n, a, b = I.chung_lu_edges(n0, 1)
    assert 0.9 * n0 < n <= n0
    deg = np.bincount(np.concatenate([a, b]), minlength=n)
    assert deg.min() >= 1  # largest component only
    assert 14.0 < deg.mean() < 18.5
    kmax = np.sqrt(16.0 * n0)  # expected degree of the heaviest vertex
    assert 0.5 * kmax < deg.max() < 2.0 * kmax
    # tail: P(deg >= k) falls like k^-(2.1 - 1), a factor 10^1.1 ~ 12.6 per decade
    ratio = (deg >= 32).sum() / (deg >= 320).sum()
    assert 8.0 < ratio < 30.0
    # edges canonical, unique
    assert (a < b).all()
    key = a.astype(np.int64) * n + b
    assert (np.diff(key) > 0).all()


def test_weights_ranges():
    w = I.log_uniform_weights(9, 100_000, -3.0, 3.0)
    assert w.min() >= 1e-3 and w.max() < 1e3
    # log10 w is uniform on [-3, 3)
    assert abs(np.log10(w).mean()) < 0.03
    v = I.unit_interval_weights(9, 100_000)
    assert v.min() > 0.0 and v.max() <= 1.0 and abs(v.mean() - 0.5) < 5e-3


def test_largest_component_tie_rule():
    # two components of equal size: the one holding vertex 0 is kept
    n2, a2, b2, keep = I.largest_component(4, np.array([0, 2]), np.array([1, 3]))
    assert n2 == 2 and sorted(np.concatenate([a2, b2]).tolist()) == [0, 1]


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_mix(seed):
    items = I.config4(seed=seed, count=9, n_lo=200, n_hi=3000)
    assert len(items) == 9
    for (g, rhs, kind) in items:
        n = g[0]
        assert kind in ("grid", "rgg", "ba")
        assert 100 <= n <= 3100
        check_csr(*g)
        assert g[3].min() >= 1e-2 and g[3].max() < 1e2
        assert abs(rhs.sum()) < 1e-9 and rhs.shape == (n,)
