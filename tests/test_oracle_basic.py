"""Pins of the CPU oracle's basic operations against closed forms and brute force.

Generators, Laplacian (Sec. 2.2), SpMV/residual, colouring, Gauss-Seidel (the
smoother named in Sec. 4).  None of these tests use the HIP library.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from paper_1806_07028_amd import inputs as I


def dense_laplacian(g):
    n, rp, ci, w = g
    W = sp.csr_matrix((w, ci, rp), shape=(n, n)).toarray()
    return np.diag(W.sum(1)) - W


# ---------------------------------------------------------------------------
# SplitMix64: published first outputs of the generator seeded with 0
# ---------------------------------------------------------------------------
def test_splitmix64_published_values(oracle):
    w = I.stream_words(0, 3)
    assert [int(x) for x in w] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # oracle's start vector uses the same stream: xi = 2 * (top53 * 2^-53) - 1
    xi = oracle.xi(3, 0, 0)
    ref = 2.0 * ((w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0
    assert np.array_equal(xi, ref)
    # build r uses counter (r << 32) + i + 1
    xi2 = oracle.xi(2, 77, 3)
    w2 = I.stream_words(77, 2, start=3 << 32)
    assert np.array_equal(xi2, 2.0 * ((w2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53) - 1.0)
    assert int(oracle.colour_priority(5, 2, 10)) == int(I.stream_words(5, 1, start=(2 << 32) + 10)[0])
    w = int(I.stream_words(5, 1, start=(2 << 32) + 10)[0])
    assert oracle.colour_key(5, 2, 10, 7) == (7 << 40) | (w >> 24)
    assert oracle.colour_key(5, 2, 10, 1 << 30) == (((1 << 24) - 1) << 40) | (w >> 24)


def test_generators_shapes():
    n, rp, ci, w = I.grid2d(64, 64)
    assert n == 4096 and len(ci) == 2 * 8064
    n, rp, ci, w = I.grid3d(8, 7, 6)
    assert len(ci) == 2 * (7 * 7 * 6 + 8 * 6 * 6 + 8 * 7 * 5)
    # symmetric, sorted, no diagonal
    A = sp.csr_matrix((w, ci, rp), shape=(n, n))
    assert (A != A.T).nnz == 0
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0) and i not in row
    g = I.rgg(3000, 5)
    assert g[0] > 2500
    nrm = I.zero_mean_normal_rhs(3, 1000)
    assert abs(nrm.sum()) < 1e-10


# ---------------------------------------------------------------------------
# Laplacian spectra (closed forms)
# ---------------------------------------------------------------------------
def _check_eig(oracle, g, lam, v):
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    q = oracle.spmv(n, rp, ci, a, d, v)
    scale = max(abs(lam), 1.0) * np.abs(v).max()
    assert np.abs(q - lam * v).max() <= 1e-13 * 8 * scale


@pytest.mark.parametrize("n", [2, 5, 64, 257])
def test_path_spectrum(oracle, n):
    g = I.path(n)
    j = np.arange(n)
    for k in [0, 1, n // 2, n - 1]:
        lam = 2 - 2 * np.cos(k * np.pi / n)
        v = np.cos(k * np.pi * (j + 0.5) / n)
        _check_eig(oracle, g, lam, v)


@pytest.mark.parametrize("n,k", [(12, 2), (100, 2), (64, 4), (1024, 4)])
def test_ring_spectrum(oracle, n, k):
    g = I.ring(n, k)
    j = np.arange(n)
    for m in [0, 1, 3, n // 3]:
        lam = sum(2 - 2 * np.cos(2 * np.pi * m * s / n) for s in range(1, k // 2 + 1))
        v = np.cos(2 * np.pi * m * j / n)
        _check_eig(oracle, g, lam, v)


def test_grid_spectrum(oracle):
    nx, ny = 9, 6
    g = I.grid2d(nx, ny)
    x = np.arange(nx)
    y = np.arange(ny)
    for p, q in [(0, 0), (1, 0), (2, 3), (8, 5)]:
        lam = (2 - 2 * np.cos(p * np.pi / nx)) + (2 - 2 * np.cos(q * np.pi / ny))
        v = np.outer(np.cos(q * np.pi * (y + 0.5) / ny), np.cos(p * np.pi * (x + 0.5) / nx)).ravel()
        _check_eig(oracle, g, lam, v)


def test_laplacian_rowsum_and_residual(oracle):
    g = I.grid3d(5, 4, 3)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    ones = np.ones(n)
    assert np.all(oracle.spmv(n, rp, ci, a, d, ones) == 0.0)  # integer weights: exact
    assert np.array_equal(dinv, 1.0 / d)
    gw = I.grid2d(7, 5, weight_seed=3)
    n, rp, ci, w = gw
    a, d, dinv = oracle.laplacian(gw)
    L = dense_laplacian(gw)
    x = I.normal(1, n)
    b = I.normal(2, n)
    r = oracle.residual(n, rp, ci, a, d, b, x)
    assert np.allclose(r, b - L @ x, rtol=0, atol=1e-12 * np.abs(L).max() * np.abs(x).max() * 10)


# ---------------------------------------------------------------------------
# Colouring: proper, <= Delta + 1, equals the sequential greedy in priority
# order, and equals Jones-Plassmann rounds (the GPU algorithm)
# ---------------------------------------------------------------------------
def _priorities(seed, level, n, deg):
    """Largest degree first (capped at 2^24 - 1, top 24 bits), then the top 40
    bits of word (level << 32) + v + 1 of the SplitMix64 stream."""
    w = I.stream_words(seed, n, start=level << 32)
    d = np.minimum(np.asarray(deg, dtype=np.uint64), np.uint64((1 << 24) - 1))
    return (d << np.uint64(40)) | (w >> np.uint64(24))


def _greedy_colour(n, rp, ci, pr):
    order = sorted(range(n), key=lambda v: (int(pr[v]), v), reverse=True)
    col = -np.ones(n, dtype=int)
    for v in order:
        used = {col[u] for u in ci[rp[v]:rp[v + 1]] if col[u] >= 0}
        c = 0
        while c in used:
            c += 1
        col[v] = c
    return col


def _jones_plassmann(n, rp, ci, pr):
    col = -np.ones(n, dtype=int)
    key = [(int(pr[v]), v) for v in range(n)]
    rounds = 0
    while (col < 0).any():
        rounds += 1
        ready = []
        for v in range(n):
            if col[v] >= 0:
                continue
            nbrs = ci[rp[v]:rp[v + 1]]
            if all(col[u] >= 0 for u in nbrs if key[u] > key[v]):
                used = {col[u] for u in nbrs if key[u] > key[v]}
                c = 0
                while c in used:
                    c += 1
                ready.append((v, c))
        for v, c in ready:
            col[v] = c
    return col, rounds


@pytest.mark.parametrize("maker", [lambda: I.grid2d(13, 11), lambda: I.rgg(600, 4), lambda: I.ring(200, 4),
                                   lambda: I.csr_from_edges(*I.ba_edges(400, 9), np.ones(len(I.ba_edges(400, 9)[1])))])
def test_colouring(oracle, maker):
    n, rp, ci, w = maker()
    for level in (0, 3):
        col, nc = oracle.colour_greedy(n, rp, ci, 0xC010, level)
        rows = np.repeat(np.arange(n), np.diff(rp))
        assert np.all(col[rows] != col[ci])
        assert nc == col.max() + 1 <= np.diff(rp).max() + 1
        pr = _priorities(0xC010, level, n, np.diff(rp))
        assert np.array_equal(col, _greedy_colour(n, rp, ci, pr))
        jp, _ = _jones_plassmann(n, rp, ci, pr)
        assert np.array_equal(col, jp)


def _bipartite_spectral(n, rp, ci):
    """A connected graph is bipartite exactly when the largest eigenvalue of its
    normalised Laplacian I - D^-1/2 W D^-1/2 equals 2 (the adjacency spectrum
    is then symmetric); connectivity from the multiplicity of eigenvalue 0."""
    W = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    W[rows, ci] = 1.0
    d = W.sum(axis=1)
    if np.any(d == 0):
        return n == 1, n == 1
    s = 1.0 / np.sqrt(d)
    ev = np.linalg.eigvalsh(np.eye(n) - s[:, None] * W * s[None, :])
    connected = int(np.sum(np.abs(ev) < 1e-9)) == 1
    return connected, connected and abs(ev[-1] - 2.0) < 1e-9


def _random_graph(seed, n, m, bipartite):
    u = I.uniform(seed, 2 * m)
    a = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
    b = np.minimum((u[1::2] * n).astype(np.int64), n - 1)
    if bipartite:  # edges only between even and odd ids
        b = np.where((a - b) % 2 == 0, np.where(b + 1 < n, b + 1, b - 1), b)
    keep = a != b
    a2, b2 = I.canonical_edges(a[keep], b[keep])
    return I.csr_from_edges(n, a2, b2, np.ones(len(a2)))


def test_colouring_red_black(oracle):
    """Connected bipartite graphs: two colours, the parity of the breadth-first
    distance from vertex 0 (closed forms on grids, paths and even rings);
    everything else: the greedy first-fit colouring."""
    n, rp, ci, w = I.grid2d(13, 11)
    col, nc = oracle.colour(n, rp, ci, 0xC010, 4)
    v = np.arange(n)
    assert nc == 2 and np.array_equal(col, (v % 13 + v // 13) % 2)
    n, rp, ci, w = I.grid3d(8, 7, 6)
    col, nc = oracle.colour(n, rp, ci, 0xC010, 0)
    v = np.arange(n)
    assert nc == 2 and np.array_equal(col, (v % 8 + (v // 8) % 7 + v // 56) % 2)
    n, rp, ci, w = I.path(9)
    col, nc = oracle.colour(n, rp, ci, 1, 0)
    assert nc == 2 and np.array_equal(col, np.arange(9) % 2)
    n, rp, ci, w = I.ring(10, 2)  # even cycle
    col, nc = oracle.colour(n, rp, ci, 1, 0)
    assert nc == 2 and np.array_equal(col, np.arange(10) % 2)
    n, rp, ci, w = I.path(1)
    col, nc = oracle.colour(n, rp, ci, 1, 0)
    assert nc == 1 and list(col) == [0]
    # odd cycle, triangles, two components: the greedy colouring
    for g in (I.ring(11, 2), I.ring(40, 4), I.rgg(300, 2)):
        n, rp, ci, w = g
        col, nc = oracle.colour(n, rp, ci, 0xC010, 2)
        gcol, gnc = oracle.colour_greedy(n, rp, ci, 0xC010, 2)
        assert nc == gnc and np.array_equal(col, gcol)
    n1, a1, b1 = I.grid2d_edges(4, 4)
    a = np.concatenate([a1, a1 + 16]); b = np.concatenate([b1, b1 + 16])
    n, rp, ci, w = I.csr_from_edges(32, a, b, np.ones(len(a)))
    col, nc = oracle.colour(n, rp, ci, 5, 1)
    gcol, gnc = oracle.colour_greedy(n, rp, ci, 5, 1)
    assert np.array_equal(col, gcol) and nc == gnc
    # random graphs against the spectral test
    seen = set()
    for seed in range(40):
        n = 8 + seed % 23
        g = _random_graph(100 + seed, n, int(n * (1.0 + (seed % 5) * 0.4)), bipartite=seed % 2 == 0)
        n, rp, ci, w = g
        connected, bip = _bipartite_spectral(n, rp, ci)
        col, nc = oracle.colour(n, rp, ci, 9, seed)
        rows = np.repeat(np.arange(n), np.diff(rp))
        assert np.all(col[rows] != col[ci])
        if bip:
            assert nc == 2 and col[0] == 0
        else:
            gcol, gnc = oracle.colour_greedy(n, rp, ci, 9, seed)
            assert nc == gnc and np.array_equal(col, gcol)
        seen.add((connected, bip))
    assert {(True, True), (True, False), (False, False)} <= seen


# ---------------------------------------------------------------------------
# Gauss-Seidel: one coloured sweep is the dense triangular solve in colour order
# ---------------------------------------------------------------------------
def test_gs_equals_dense_triangular(oracle):
    g = I.grid2d(9, 8, weight_seed=5)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    col, nc = oracle.colour(n, rp, ci, 7, 0)
    L = dense_laplacian(g)
    b = I.normal(11, n)
    x0 = I.normal(12, n)
    # forward: rows of lower colour updated first
    lower = col[None, :] < col[:, None]
    upper = col[None, :] > col[:, None]
    M = np.diag(np.diag(L)) + np.where(lower, L, 0)
    N = np.where(upper, L, 0)
    ref = sla.solve_triangular(M[np.ix_(np.argsort(col, kind="stable"), np.argsort(col, kind="stable"))],
                               (b - N @ x0)[np.argsort(col, kind="stable")], lower=True)
    xf = np.empty(n)
    xf[np.argsort(col, kind="stable")] = ref
    got = oracle.gs(n, rp, ci, a, dinv, col, nc, b, x0, forward=True)
    assert np.allclose(got, xf, rtol=1e-13, atol=1e-13 * np.abs(xf).max())
    # backward: rows of higher colour first
    Mb = np.diag(np.diag(L)) + np.where(upper, L, 0)
    Nb = np.where(lower, L, 0)
    xb = np.linalg.solve(Mb, b - Nb @ x0)
    got = oracle.gs(n, rp, ci, a, dinv, col, nc, b, x0, forward=False)
    assert np.allclose(got, xb, rtol=1e-12, atol=1e-12 * np.abs(xb).max())


def test_symmetric_gs_is_a_symmetric(oracle):
    g = I.grid2d(7, 6, weight_seed=2)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    col, nc = oracle.colour(n, rp, ci, 3, 0)
    L = dense_laplacian(g)
    zero = np.zeros(n)

    def E(x):
        x = oracle.gs(n, rp, ci, a, dinv, col, nc, zero, x, True)
        return oracle.gs(n, rp, ci, a, dinv, col, nc, zero, x, False)

    x = I.normal(1, n)
    y = I.normal(2, n)
    lhs = E(x) @ L @ y
    rhs = x @ L @ E(y)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))
    # constants are fixed points of the homogeneous sweep
    c = np.full(n, 0.75)
    assert np.allclose(E(c), c, rtol=0, atol=1e-15)


def test_smooth_error_is_smoother(oracle):
    g = I.grid2d(32, 32)
    n, rp, ci, w = g
    L = dense_laplacian(g)
    xi = oracle.xi(n, 9, 0)
    e3 = oracle.smooth_error(g, 0xC010, 9, 3)
    e0 = oracle.smooth_error(g, 0xC010, 9, 0)
    assert np.array_equal(e0, xi)

    def rq(v):
        v = v - v.mean()
        return v @ L @ v / (v @ v)

    assert rq(e3) < 0.25 * rq(xi)
    # reproducible bit for bit
    assert np.array_equal(e3, oracle.smooth_error(g, 0xC010, 9, 3))


def test_gs32_close_to_gs64(oracle):
    g = I.grid2d(16, 16, weight_seed=4)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    col, nc = oracle.colour(n, rp, ci, 3, 0)
    b = I.normal(1, n)
    x64 = oracle.gs(n, rp, ci, a, dinv, col, nc, b, np.zeros(n), True)
    x32 = oracle.gs32(n, rp, ci, a.astype(np.float32), dinv.astype(np.float32), col, nc, b.astype(np.float32),
                      np.zeros(n, np.float32), True)
    assert np.abs(x32 - x64).max() <= 1e-5 * np.abs(x64).max()


def test_batch_workload_recipe():
    """The uneven batch: sizes within the log-uniform range (up to the
    rounding of the grid sides and the largest RGG component), all three kinds,
    connected graphs, zero-mean right-hand sides."""
    batch = I.config4(seed=2, count=30, n_lo=200, n_hi=4000)
    kinds = {k for g, b, k in batch}
    assert kinds == {"grid", "rgg", "ba"}
    for g, b, k in batch:
        n, rp, ci, w = g
        assert 100 <= n <= 4200 and len(b) == n and abs(b.sum()) < 1e-9
        assert np.all(w >= 1e-2) and np.all(w <= 1e2)
        n_lcc, _, _, keep = I.largest_component(n, *I.upper_edges(rp, ci))
        assert n_lcc == n and keep.all()
