"""Pins of the oracle's setup phase (Alg. 1, Alg. 3, Alg. 4) against closed
forms, exhaustive search, invariants stated in the paper and hand-derived
examples.  CPU only.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1806_07028_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_laplacian(g):
    n, rp, ci, w = g
    W = sp.csr_matrix((w, ci, rp), shape=(n, n)).toarray()
    return np.diag(W.sum(1)) - W


def cover_edges(nb):
    out = set()
    for v, (a, b) in enumerate(np.asarray(nb).reshape(-1, 2)):
        for u in (a, b):
            if u >= 0:
                out.add((min(u, v), max(u, v)))
    return out


def check_linear_forest(n, edges):
    deg = np.zeros(n, int)
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in edges:
        deg[u] += 1
        deg[v] += 1
        ru, rv = find(u), find(v)
        assert ru != rv, "cycle in cover"
        parent[ru] = rv
    assert deg.max(initial=0) <= 2


# ---------------------------------------------------------------------------
# A^2 pattern (Alg. 4, Step 2)
# ---------------------------------------------------------------------------
def e2_count_2d(nx, ny):
    return ((nx - 1) * ny + nx * (ny - 1)) + ((nx - 2) * ny + nx * (ny - 2)) + 2 * (nx - 1) * (ny - 1)


def e2_count_3d(nx, ny, nz):
    grid = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    straight = (nx - 2) * ny * nz + nx * (ny - 2) * nz + nx * ny * (nz - 2)
    diag = 2 * ((nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1))
    return grid + straight + diag


def test_a2_closed_forms(oracle):
    assert e2_count_2d(64, 64) == 23938
    assert e2_count_3d(128, 128, 128) == 24822528
    for nx, ny in [(3, 3), (64, 64), (17, 5)]:
        n, rp, ci, w = I.grid2d(nx, ny)
        rp2, ci2 = oracle.a2_pattern(n, rp, ci)
        assert len(ci2) == 2 * e2_count_2d(nx, ny)
    for dims in [(4, 5, 6), (9, 9, 9)]:
        n, rp, ci, w = I.grid3d(*dims)
        rp2, ci2 = oracle.a2_pattern(n, rp, ci)
        assert len(ci2) == 2 * e2_count_3d(*dims)


@pytest.mark.parametrize("seed,cap", [(1, 0), (2, 0), (3, 3), (4, 5)])
def test_a2_brute_force(oracle, seed, cap):
    n, rp, ci, w = I.csr_from_edges(*I.ba_edges(60, seed, 2), np.ones(len(I.ba_edges(60, seed, 2)[1])))
    A = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n)).toarray() > 0
    deg = A.sum(1)
    piv = A[:, deg <= cap] if cap else A
    R = A | ((piv.astype(int) @ piv.T.astype(int)) > 0)
    np.fill_diagonal(R, False)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci, cap)
    got = np.zeros((n, n), bool)
    for i in range(n):
        row = ci2[rp2[i]:rp2[i + 1]]
        assert np.all(np.diff(row) > 0)
        got[i, row] = True
    assert np.array_equal(got, R)


# ---------------------------------------------------------------------------
# Path cover (Alg. 1)
# ---------------------------------------------------------------------------
def test_worked_example(oracle):
    ex = json.load(open(os.path.join(GOLDEN, "grid3x3_worked_example.json")))
    g = I.grid2d(3, 3)
    n, rp, ci, w = g
    e = np.array(ex["e"], float)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci)
    assert len(ci2) == 2 * ex["a2_edges"]
    su, sv = oracle.sorted_edges(n, rp2, ci2, e)
    assert [list(p) for p in zip(su[:8].tolist(), sv[:8].tolist())] == ex["sorted_edges_head"]
    nb = oracle.path_cover(n, su, sv)
    assert cover_edges(nb) == {tuple(p) for p in ex["cover_edges"]}
    pid, pos, plen, npaths = oracle.orient(nb)
    assert npaths == 1
    assert [int(v) for v in np.argsort(pos)] == ex["cover_path"]
    H = oracle.Hierarchy(g, e, coarse_max=1)
    assert H.get_int(0, "agg").tolist() == ex["agg"]
    inf = H.info(0)
    assert inf["case2"] == 1 and inf["n_unagg"] == 1
    # coarse path of level 1, in position order
    pos1 = H.get_int(1, "pos")
    assert [int(v) for v in np.argsort(pos1)] == ex["coarse_path"]
    # e is 0 on {2,4,6} after centring: aggregate {2,4} takes the boolean fallback
    assert inf["p1_fallback"] == 1
    pv = H.get_dbl(0, "pval")
    assert pv[2] == 1.0 and pv[4] == 1.0


def test_path_cover_hand_cases(oracle):
    # triangle, weights 3 > 2 > 1: the lightest edge would close a cycle
    nb = oracle.path_cover(3, np.array([0, 1, 0]), np.array([1, 2, 2]))
    assert cover_edges(nb) == {(0, 1), (1, 2)}
    # star with centre 0: only the two heaviest edges
    nb = oracle.path_cover(5, np.array([0, 0, 0, 0]), np.array([3, 1, 4, 2]))
    assert cover_edges(nb) == {(0, 3), (0, 1)}
    # a path graph in any weight order is covered entirely
    order = [3, 0, 5, 1, 4, 2]
    nb = oracle.path_cover(7, np.array(order), np.array(order) + 1)
    assert cover_edges(nb) == {(i, i + 1) for i in range(6)}
    # merging two paths through their ends
    nb = oracle.path_cover(4, np.array([0, 2, 1]), np.array([1, 3, 2]))
    assert cover_edges(nb) == {(0, 1), (2, 3), (1, 2)}
    # ...but not the ends of one path (cycle)
    nb = oracle.path_cover(4, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 3]))
    assert cover_edges(nb) == {(0, 1), (1, 2), (2, 3)}


def best_path_cover_weight(n, edges, wts):
    best = 0.0
    m = len(edges)
    for mask in range(1 << m):
        deg = [0] * n
        parent = list(range(n))
        ok = True
        tot = 0.0

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x

        for t in range(m):
            if mask >> t & 1:
                u, v = edges[t]
                deg[u] += 1
                deg[v] += 1
                if deg[u] > 2 or deg[v] > 2:
                    ok = False
                    break
                ru, rv = find(u), find(v)
                if ru == rv:
                    ok = False
                    break
                parent[ru] = rv
                tot += wts[t]
        if ok:
            best = max(best, tot)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_path_cover_half_approximation(oracle, seed):
    """Greedy cover weight >= 1/2 of the maximum path cover weight (Sec. 2.2)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 10))
    pairs = list(itertools.combinations(range(n), 2))
    m = int(rng.integers(n, min(14, len(pairs)) + 1))
    pick = rng.choice(len(pairs), m, replace=False)
    edges = [pairs[t] for t in sorted(pick)]
    wts = rng.uniform(0.1, 10.0, m)
    order = np.argsort(-wts, kind="stable")
    su = np.array([edges[t][0] for t in order])
    sv = np.array([edges[t][1] for t in order])
    nb = oracle.path_cover(n, su, sv)
    got = cover_edges(nb)
    check_linear_forest(n, got)
    wmap = {edges[t]: wts[t] for t in range(m)}
    gw = sum(wmap[e] for e in got)
    assert gw >= 0.5 * best_path_cover_weight(n, edges, wts) - 1e-12


@pytest.mark.parametrize("maker", [lambda: I.grid2d(20, 17), lambda: I.rgg(800, 3), lambda: I.grid3d(7, 6, 5)])
def test_path_cover_invariants(oracle, maker):
    g = maker()
    n, rp, ci, w = g
    e = oracle.smooth_error(g, 1, 2, 3)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci)
    su, sv = oracle.sorted_edges(n, rp2, ci2, e)
    nb = oracle.path_cover(n, su, sv)
    got = cover_edges(nb)
    check_linear_forest(n, got)
    allowed = set(zip(su.tolist(), sv.tolist()))
    assert got <= allowed
    # maximal: every rejected edge has a saturated end or joins one path
    deg = np.zeros(n, int)
    for u, v in got:
        deg[u] += 1
        deg[v] += 1
    pid, pos, plen, _ = oracle.orient(nb)
    for u, v in zip(su.tolist(), sv.tolist()):
        if (u, v) in got:
            continue
        assert deg[u] == 2 or deg[v] == 2 or (pid[u] >= 0 and pid[u] == pid[v])
    # sorted order: keys ascending, ties by lexicographic index
    keys = np.abs(e[su] - e[sv])
    assert np.all(np.diff(keys) >= 0)
    idx = np.array(su, np.int64) * n + sv
    tie = np.diff(keys) == 0
    assert np.all(np.diff(idx)[tie] > 0)


# ---------------------------------------------------------------------------
# Aggregation (Alg. 3)
# ---------------------------------------------------------------------------
def level_graph(n, edges, wts):
    a = np.array([min(u, v) for u, v in edges])
    b = np.array([max(u, v) for u, v in edges])
    o = np.lexsort((b, a))
    return I.csr_from_edges(n, a[o], b[o], np.asarray(wts, float)[o])


def nb_from_paths(n, paths):
    nb = -np.ones((n, 2), np.int32)
    cnt = np.zeros(n, int)
    for p in paths:
        for u, v in zip(p[:-1], p[1:]):
            nb[u, cnt[u]] = v
            cnt[u] += 1
            nb[v, cnt[v]] = u
            cnt[v] += 1
    return nb


def test_aggregation_cases(oracle):
    # path 0-1-2-3-4 (odd: 4 left over); 5, 6 isolated; weights pick partners
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 3), (5, 6), (4, 5), (6, 2)]
    edges = sorted({(min(u, v), max(u, v)) for u, v in edges})
    w = {(0, 1): 1, (1, 2): 1, (2, 3): 1, (3, 4): 1, (5, 6): 5, (4, 5): 2, (2, 6): 1}
    n, rp, ci, gw = level_graph(7, edges, [w[e] for e in edges])
    nb = nb_from_paths(7, [[0, 1, 2, 3, 4]])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb)
    # pairs {0,1},{2,3}; u=4 best is 5 (unaggregated): Case 1 {4,5}; u=6 best is 5 -> Case 2 {4,5,6}
    assert st["case1"] == 1 and st["case2"] == 1
    assert agg.tolist() == [0, 0, 1, 1, 2, 2, 2]

    # Case 3 (steal): triple {2,3,4} with 2~4 adjacent; u=5's best neighbour is 3
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (2, 4), (3, 5)]
    wts = [1, 1, 1, 1, 1, 9]
    n, rp, ci, gw = level_graph(6, edges, wts)
    # cover: paths [0,1] and [2,3,4]; vertex 4 is the odd tail, its best neighbour 2 or 3 ...
    nb = nb_from_paths(6, [[0, 1], [2, 3, 4]])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb)
    # 4: neighbours 3 (w 1), 2 (w 1): tie -> smaller id 2 -> Case 2 {2,3,4}; 5: best 3 in a triple, 2~4 adjacent
    assert st["case2"] == 1 and st["case3"] == 1
    assert agg.tolist() == [0, 0, 1, 2, 1, 2]

    # middle: triple 2-3-4 as a chain (2 !~ 4); u=5's best neighbour is the
    # middle 3: taking 3 out would leave {2, 4} disconnected, so 5 joins
    # (no isolated vertex, Sec. 3.3)
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (3, 5)]
    wts = [1, 1, 1, 1, 9]
    n, rp, ci, gw = level_graph(6, edges, wts)
    nb = nb_from_paths(6, [[0, 1], [2, 3, 4]])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb)
    assert st["case2"] == 1 and st["middle"] == 1 and st["singleton"] == 0
    assert agg.tolist() == [0, 0, 1, 1, 1, 1]

    # star: 5 and then 6 join at the centre 3; 7's best neighbour is the leaf
    # 5, which leaves the star (the rest stays connected through 3): {5, 7}
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (3, 5), (3, 6), (5, 7)]
    wts = [1, 1, 1, 1, 9, 9, 1]
    n, rp, ci, gw = level_graph(8, edges, wts)
    nb = nb_from_paths(8, [[0, 1], [2, 3, 4]])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb)
    assert st["case2"] == 1 and st["middle"] == 2 and st["case3"] == 1
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 1, 2] and nc == 3

    # the centre stays: 8's best neighbour is the centre 3 of the star {2,3,4,5,6}
    # (after 7 took 5 out it is {2,3,4,6}): 8 joins it
    edges = [(0, 1), (1, 2), (2, 3), (3, 4), (3, 5), (3, 6), (5, 7), (3, 8)]
    wts = [1, 1, 1, 1, 9, 9, 1, 9]
    n, rp, ci, gw = level_graph(9, edges, wts)
    nb = nb_from_paths(9, [[0, 1], [2, 3, 4]])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb)
    assert st["middle"] == 3 and st["case3"] == 1
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 1, 2, 1]

    # a vertex without neighbours is a singleton
    n, rp, ci, gw = level_graph(3, [(0, 1)], [1.0])
    agg, nc, st = oracle.aggregate(n, rp, ci, gw, nb_from_paths(3, [[0, 1]]))
    assert agg.tolist() == [0, 0, 1] and st["singleton"] == 1


def test_path_graph_pairs_and_triple(oracle):
    """A path graph with a linear smooth error is covered by one path: pairs plus
    a final triple when the length is odd (Sec. 3.3: sizes 2 or 3 along a path)."""
    for n in (10, 11):
        g = I.path(n)
        e = np.arange(n, dtype=float)
        H = oracle.Hierarchy(g, e, coarse_max=1)
        agg = H.get_int(0, "agg")
        sizes = np.bincount(agg)
        if n % 2 == 0:
            assert np.all(sizes == 2)
        else:
            assert sorted(sizes.tolist()) == [2] * (n // 2 - 1) + [3]


def agg_checks(H, level):
    inf = H.info(level)
    agg = H.get_int(level, "agg")
    nc = inf["nc"]
    sizes = np.bincount(agg, minlength=nc)
    assert sizes.min() >= 1
    assert (sizes == 1).sum() == inf["singleton"]
    # every member past the third joined at the middle or centre
    assert np.maximum(sizes - 3, 0).sum() <= inf["middle"]
    # connected in the level graph
    grp, gci = H.get_int(level, "G_rp"), H.get_int(level, "G_ci")
    adj = lambda a, b: b in set(gci[grp[a]:grp[a + 1]].tolist())
    members = [[] for _ in range(nc)]
    for v, a in enumerate(agg):
        members[a].append(v)
    for m in members:
        if len(m) == 2:
            assert adj(m[0], m[1])
        if len(m) == 3:
            links = adj(m[0], m[1]) + adj(m[0], m[2]) + adj(m[1], m[2])
            assert links >= 2
        if len(m) > 3:  # a star: one member adjacent to all the others
            assert any(all(adj(c, x) for x in m if x != c) for c in m)
    # ids ordered by smallest member
    mins = [min(m) for m in members]
    assert mins == sorted(mins)


@pytest.mark.parametrize("maker", [lambda: I.grid2d(40, 33), lambda: I.rgg(3000, 7),
                                   lambda: I.grid3d(12, 11, 10, weight_seed=2),
                                   lambda: I.config3(n0=5000)[0]])
def test_hierarchy_invariants(oracle, maker):
    g = maker()
    n = g[0]
    H = oracle.Hierarchy(g, None, coarse_max=8)
    L = dense_laplacian(g)
    assert H.nlevels >= 3
    for l in range(H.nlevels - 1):
        agg_checks(H, l)
    # P_1 * 1 = e (the prolongation reproduces the smooth error, Sec. 3.3)
    agg = H.get_int(0, "agg")
    pv = H.get_dbl(0, "pval")
    nc = H.info(0)["nc"]
    P = sp.csr_matrix((pv, agg, np.arange(n + 1)), shape=(n, nc))
    e_used = P @ np.ones(nc)
    assert np.array_equal(e_used, pv)
    # the intuition test (Sec. 3.1): restrict-then-prolong reproduces e
    PtP = (P.T @ P).diagonal()
    proj = P @ ((P.T @ e_used) / PtP)
    assert np.linalg.norm(proj - e_used) <= 1e-10 * np.linalg.norm(e_used)
    # Galerkin: A_2 y = P^T A P y and A_2 1 = P^T A e
    rp1, ci1, av1, d1 = H.level_matrix(1)
    A2 = sp.csr_matrix((av1, ci1, rp1), shape=(nc, nc)) + sp.diags(d1)
    y = I.normal(5, nc)
    ref = P.T @ (L @ (P @ y))
    assert np.linalg.norm(A2 @ y - ref) <= 1e-13 * np.linalg.norm(ref) * 10
    assert np.allclose(A2 @ np.ones(nc), P.T @ (L @ e_used), atol=1e-12 * np.abs(d1).max())
    # symmetric up to the rounding of the two sum orders of c_IJ and c_JI
    assert abs(A2 - A2.T).max() <= 1e-15 * abs(A2).max()


def test_galerkin_closed_form(oracle):
    """Horizontal pairs on a unit nx x ny grid coarsen (boolean P) to the
    anisotropic grid Laplacian with weights 1 (horizontal) and 2 (vertical)."""
    nx, ny = 8, 5
    g = I.grid2d(nx, ny)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    agg = np.array([(v // nx) * (nx // 2) + (v % nx) // 2 for v in range(n)], np.int32)
    nc = n // 2
    rpc, cic, vc, dc = oracle.galerkin(n, rp, ci, a, d, nc, agg, np.ones(n))
    n2, a2, b2 = I.grid2d_edges(nx // 2, ny)
    wts = np.where(b2 - a2 == 1, 1.0, 2.0)
    ref = dense_laplacian(I.csr_from_edges(n2, a2, b2, wts))
    got = sp.csr_matrix((vc, cic, rpc), shape=(nc, nc)).toarray() + np.diag(dc)
    assert np.array_equal(got, ref)
    # unit path in pairs -> unit path of half the size
    g = I.path(12)
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    rpc, cic, vc, dc = oracle.galerkin(n, rp, ci, a, d, 6, (np.arange(12) // 2).astype(np.int32), np.ones(12))
    got = sp.csr_matrix((vc, cic, rpc), shape=(6, 6)).toarray() + np.diag(dc)
    assert np.array_equal(got, dense_laplacian(I.path(6)))


def test_const_mode_levels_are_laplacians(oracle):
    g = I.grid2d(30, 30, weight_seed=8)
    H = oracle.Hierarchy(g, None, p1_mode=1, coarse_max=8)
    for l in range(1, H.nlevels):
        rp, ci, av, d = H.level_matrix(l)
        n = len(d)
        rows = np.repeat(np.arange(n), np.diff(rp))
        rs = d + np.bincount(rows, weights=av, minlength=n)
        assert np.abs(rs).max() <= 1e-12 * d.max()
        assert np.all(av <= 0)
    assert H.info(H.nlevels - 1)["grounded"] == 1


def test_shortening_invariants(oracle):
    g = I.grid2d(30, 27)
    H = oracle.Hierarchy(g, None, coarse_max=4)
    for l in range(1, H.nlevels):
        nb = H.get_int(l, "nb").reshape(-1, 2)
        n = len(nb)
        edges = cover_edges(nb)
        check_linear_forest(n, edges)
        grp, gci = H.get_int(l, "G_rp"), H.get_int(l, "G_ci")
        for u, v in edges:
            assert v in set(gci[grp[u]:grp[u + 1]].tolist())


def test_shorten_first_occurrence(oracle):
    # two paths [0,1,2,3] and [4,5,6]; aggregate {3,4} appears at the end of
    # path 0 and the start of path 4: it stays in path 0 only.
    nb = nb_from_paths(7, [[0, 1, 2, 3], [4, 5, 6]])
    agg = np.array([0, 0, 1, 2, 2, 3, 3], np.int32)
    nbc = oracle.shorten(nb, 4, agg)
    assert cover_edges(nbc) == {(0, 1), (1, 2)}
    # a repeat inside one path cuts it: [0,1,2,3,4] with agg 0 0 1 0? (not
    # consecutive) -> 0, 1 then 0 again is dropped
    nb = nb_from_paths(5, [[0, 1, 2, 3, 4]])
    agg = np.array([0, 0, 1, 0, 2], np.int32)
    nbc = oracle.shorten(nb, 3, agg)
    assert cover_edges(nbc) == {(0, 1)}


# ---------------------------------------------------------------------------
# Smooth error before a build (Sec. 3.2), level loop and operator complexity
# (Alg. 4 Steps 4-9)
# ---------------------------------------------------------------------------
def xi_ref(seed, r, n):
    """U[-1, 1) start vector of build r: word (r << 32) + i + 1 of the stream."""
    k = (np.uint64(r) << np.uint64(32)) + np.arange(1, n + 1, dtype=np.uint64)
    return 2.0 * I.uniform_at(seed, k) - 1.0


def relax_ref(g, colour, e, sweeps):
    """Symmetric Gauss-Seidel on A e = 0 in colour order, written independently:
    the rows of one colour share no edge, so a colour's update is one sparse
    product with the values the earlier colours have just written."""
    n, rp, ci, w = g
    W = sp.csr_matrix((w, ci, rp), shape=(n, n))
    d = np.asarray(W.sum(1)).ravel()
    ncol = int(colour.max()) + 1
    rows = [np.flatnonzero(colour == c) for c in range(ncol)]
    e = e.copy()
    for _ in range(sweeps):
        for c in list(range(ncol)) + list(range(ncol - 1, -1, -1)):
            r = rows[c]
            e[r] = (W[r] @ e) / d[r]  # (0 - sum_j a_ij e_j) / a_ii with a_ij = -w_ij
    return e


@pytest.mark.parametrize("maker", [lambda: I.grid2d(21, 17, weight_seed=4),
                                   lambda: I.rgg(900, 12),
                                   lambda: I.config3(n0=3000)[0]])
def test_first_build_error_is_relaxed_xi(oracle, maker):
    g = maker()
    n, rp, ci, w = g
    H = oracle.Hierarchy(g, None, coarse_max=8, rebuild_vcycles=0)
    colour = H.get_int(0, "colour")
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert (colour[rows] != colour[ci]).all(), "colour classes must be independent sets"
    p = H.p
    x0 = xi_ref(p.seed, 0, n)
    assert np.array_equal(oracle.xi(n, p.seed, 0), x0)
    ref = relax_ref(g, colour, x0, p.relax_sweeps)
    got = H.get_dbl(0, "e")
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # the relaxation lowers the energy e^T A e (it smooths)
    L = dense_laplacian(g)
    assert got @ L @ got < 0.5 * (x0 @ L @ x0)
    # a re-setup's vector: fresh xi of build r, the hierarchy's V-cycles on
    # A e = 0, then the same sweeps
    for r in (1, 3):
        xr = xi_ref(p.seed, r, n)
        assert not np.array_equal(xr, x0)
        got_r = H.relax_error(r)
        ref_r = relax_ref(g, colour, xr, p.relax_sweeps)
        assert np.linalg.norm(got_r - ref_r) <= 1e-13 * np.linalg.norm(ref_r)
    H2 = oracle.Hierarchy(g, None, coarse_max=8, rebuild_vcycles=2)
    xr = xi_ref(p.seed, 2, n)
    v = H2.vcycle(np.zeros(n), xr)
    v = H2.vcycle(np.zeros(n), v)
    ref_r = relax_ref(g, colour, v, p.relax_sweeps)
    got_r = H2.relax_error(2)
    assert np.linalg.norm(got_r - ref_r) <= 1e-12 * np.linalg.norm(ref_r)


@pytest.mark.parametrize("maker,cmax", [(lambda: I.grid2d(40, 37, weight_seed=6), 64),
                                        (lambda: I.grid3d(11, 10, 9, weight_seed=3), 8),
                                        (lambda: I.config3(n0=4000)[0], 64)])
def test_level_loop_and_operator_complexity(oracle, maker, cmax):
    g = maker()
    H = oracle.Hierarchy(g, None, coarse_max=cmax)
    L = H.nlevels
    inf = [H.info(l) for l in range(L)]
    assert inf[0]["n"] == g[0] and inf[0]["nnz"] == len(g[2])
    for l in range(L - 1):
        assert inf[l]["n"] > cmax  # coarsening continues above the limit
        assert inf[l + 1]["n"] == inf[l]["nc"]
        # connected levels: no singleton, every aggregate holds two or more
        assert inf[l]["singleton"] == 0 and 2 * inf[l]["nc"] <= inf[l]["n"]
    assert inf[-1]["n"] <= cmax or inf[-1]["coarse_fallback"]
    # operator complexity: stored entries of all levels (diagonal included)
    # over those of the finest operator
    tot = sum(i["nnz"] + i["n"] for i in inf)
    assert H.op_complexity == pytest.approx(tot / (inf[0]["nnz"] + inf[0]["n"]), rel=1e-15)
    assert H.op_complexity > 1.0
