"""Power-law workload: Chung-Lu graphs (degree exponent 2.1, mean degree 16,
largest component kept, weights uniform in (0, 1], zero-mean normal
right-hand side), A^2 pattern with the hub cap 64, FCG(1) with FP32 cycles
to 1e-8 relative residual.

At 500,000 drawn vertices every stage of the first hierarchy runs in the
oracle on the library's own input of that stage, level by level, and must
give the library's output bit for bit: the Laplacian, the first smooth
error, the A^2 pattern, the sorted edges and path cover (Alg. 1), the
aggregates (Alg. 3), the Galerkin operators of A and of the weight graph,
the path shortening and every level's colouring.

At the full size (4,000,000 drawn; 3,926,673 vertices and 32,002,743 edges
kept) the oracle's A^2 stages take minutes, so there: the Laplacian, smooth
error, colourings, Galerkin operators of A and path shortening bit for bit
against the oracle; sampled rows of the A^2 pattern, its keys and weights
against their definitions; the path cover, aggregates and prolongation by
the invariants that hold at any size (a cover of vertex-disjoint simple
paths inside the weight graph, one aggregate per vertex, every aggregate
connected in its level's weight graph); and the solve by its FP64 residual,
recomputed on the host."""
import time

import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I
from test_gpu_parity import host, same

pytestmark = pytest.mark.gpu

COLOUR_SEED = 0xC010
HUB_CAP = 64


def _log(msg):
    print(f"powerlaw: {msg}", flush=True)


def _build(gpu, n0):
    t = time.time()
    g, b = I.config3(n0=n0)
    n, rp, ci, w = g
    _log(f"n0={n0}: graph n={n} edges={len(ci) // 2} in {time.time() - t:.1f}s")
    t = time.time()
    s = gpu.Solver(rp, ci, w, b, outer="fcg", cycle_prec="f32", theta=0.5, a2_hub_cap=HUB_CAP, keep_setup=1)
    _log(f"setup {time.time() - t:.1f}s, {s.num_levels(0)} levels: "
         f"{[s.level_info(l, 0)['n'] for l in range(s.num_levels(0))]}")
    return g, b, s


@pytest.fixture(scope="module")
def c3_500k(gpu):
    return _build(gpu, 500_000)


@pytest.fixture(scope="module")
def c3(gpu):
    return _build(gpu, 4_000_000)


def _finest_common(g, s, oracle):
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    same(s.level_get(0, "A_v", 0), a)
    same(s.level_get(0, "d", 0), d)
    same(s.level_get(0, "dinv", 0), dinv)
    e = host(s.initial_error())
    same(e, oracle.smooth_error(g, COLOUR_SEED, s.p.seed, s.p.relax_sweeps))
    return e


def _levels_exact(s, oracle, with_graph):
    """Every level: colouring; below the coarsest, the Galerkin operator of A
    and the shortened paths; with_graph: also the aggregates of levels > 0 and
    the Galerkin operator of the weight graph."""
    L = s.num_levels(0)
    for l in range(L):
        inf = s.level_info(l, 0)
        m = inf["n"]
        arp, aci = s.level_get(l, "A_rp", 0), s.level_get(l, "A_ci", 0)
        rcol, rnc = oracle.colour(m, arp, aci, COLOUR_SEED, l)
        same(s.level_get(l, "colour", 0), rcol)
        assert inf["ncolours"] == rnc
        if l + 1 == L:
            break
        nc = inf["nc"]
        nb = s.level_get(l, "nb", 0).reshape(-1, 2)
        agg = s.level_get(l, "agg", 0)
        if with_graph:
            grp, gci, gv = s.level_get(l, "G_rp", 0), s.level_get(l, "G_ci", 0), s.level_get(l, "G_v", 0)
            if l > 0:
                ragg, rnc_, st = oracle.aggregate(m, grp, gci, gv, nb)
                same(agg, ragg)
                assert rnc_ == nc and all(inf[k] == v for k, v in st.items())
            if l + 2 < L:  # the coarsest level keeps no weight graph
                grpc, gcic, gvc, _ = oracle.galerkin(m, grp, gci, gv, np.zeros(m), nc, agg, np.ones(m))
                same(s.level_get(l + 1, "G_rp", 0), grpc)
                same(s.level_get(l + 1, "G_ci", 0), gcic)
                same(s.level_get(l + 1, "G_v", 0), gvc)
            del grp, gci, gv
        pval = s.level_get(l, "pval", 0) if l == 0 else np.ones(m)
        rpc, cic, vc, dc = oracle.galerkin(m, arp, aci, s.level_get(l, "A_v", 0), s.level_get(l, "d", 0), nc, agg,
                                           pval)
        same(s.level_get(l + 1, "A_rp", 0), rpc)
        same(s.level_get(l + 1, "A_ci", 0), cic)
        same(s.level_get(l + 1, "A_v", 0), vc)
        same(s.level_get(l + 1, "d", 0), dc)
        nbc = oracle.shorten(nb, nc, agg)
        same(np.sort(s.level_get(l + 1, "nb", 0).reshape(-1, 2), axis=1), np.sort(nbc, axis=1))
    return L


# ---------------------------------------------------------------------------
# 500k: every stage against the oracle
# ---------------------------------------------------------------------------
def test_powerlaw_500k_finest_stages(c3_500k, oracle):
    """Level 0: Laplacian, first smooth error, capped A^2 pattern, sorted
    edges and path cover, aggregates."""
    g, b, s = c3_500k
    n, rp, ci, w = g
    e = _finest_common(g, s, oracle)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci, HUB_CAP)
    grp, gci = s.level_get(0, "G_rp", 0), s.level_get(0, "G_ci", 0)
    same(grp, rp2)
    same(gci, ci2)
    del rp2, ci2
    su, sv = oracle.sorted_edges(n, grp, gci, e)
    nb = oracle.path_cover(n, su, sv)
    del su, sv
    same(np.sort(s.level_get(0, "nb", 0).reshape(-1, 2), axis=1), np.sort(nb, axis=1))
    gv, gkey = s.level_get(0, "G_v", 0), s.level_get(0, "gkey", 0)
    agg, nc, st = oracle.aggregate(n, grp, gci, gv, nb, gkey)
    same(s.level_get(0, "agg", 0), agg)
    info = s.level_info(0, 0)
    assert info["nc"] == nc and all(info[k] == v for k, v in st.items())
    _log(f"500k level 0: A^2 {len(gci) // 2} edges, {nc} aggregates, {st['middle']} joined at a middle or centre")


def test_powerlaw_500k_levels(c3_500k, oracle):
    g, b, s = c3_500k
    L = _levels_exact(s, oracle, with_graph=True)
    assert s.level_info(L - 1, 0)["n"] <= 4096


# ---------------------------------------------------------------------------
# full size: exact where the oracle is quick, definitions and invariants else
# ---------------------------------------------------------------------------
def _edge_keys(rp, ci):
    rows = np.repeat(np.arange(len(rp) - 1, dtype=np.int64), np.diff(rp))
    return (rows << 32) | ci.astype(np.int64)


def _has_edges(keys, a, b):
    q = (np.asarray(a, np.int64) << 32) | np.asarray(b, np.int64)
    i = np.minimum(np.searchsorted(keys, q), len(keys) - 1)
    return keys[i] == q


def test_powerlaw_exact_stages(c3, oracle):
    """Laplacian, first smooth error; every level's colouring, Galerkin
    operator of A and shortened paths, bit for bit."""
    g, b, s = c3
    _finest_common(g, s, oracle)
    L = _levels_exact(s, oracle, with_graph=False)
    assert s.level_info(L - 1, 0)["n"] <= 4096


def test_powerlaw_a2_sampled_rows(c3):
    """Rows of the level-0 weight graph against the definitions: the
    off-diagonal pattern of A^2 with two-step pairs only through vertices of
    degree <= 64, keys |e_i - e_j| and weights 1 / max(key, 2^-52 max|e|)
    (Alg. 4, Step 2), on 512 random rows and the 16 of largest degree."""
    (n, rp, ci, w), b, s = c3
    e = host(s.initial_error())
    grp = s.level_get(0, "G_rp", 0)
    gci, gkey, gv = s.level_get(0, "G_ci", 0), s.level_get(0, "gkey", 0), s.level_get(0, "G_v", 0)
    deg = np.diff(rp)
    tau = 2.0 ** -52 * np.abs(e).max()
    rows = np.concatenate([np.minimum((I.uniform(7, 512) * n).astype(np.int64), n - 1), np.argsort(deg)[-16:]])
    for i in rows.tolist():
        nbr = ci[rp[i]:rp[i + 1]]
        piv = nbr[deg[nbr] <= HUB_CAP]
        row = np.unique(np.concatenate([nbr] + [ci[rp[k]:rp[k + 1]] for k in piv]))
        row = row[row != i]
        lo, hi = grp[i], grp[i + 1]
        assert np.array_equal(gci[lo:hi], row), i
        key = np.abs(e[i] - e[row])
        assert np.array_equal(gkey[lo:hi], key), i
        assert np.array_equal(gv[lo:hi], 1.0 / np.maximum(key, tau)), i


def test_powerlaw_cover_and_aggregates(c3, oracle):
    """Level 0: the cover is symmetric, inside the weight graph, and made of
    simple paths (every covered vertex lies on a path from an endpoint, with
    the oracle's orientation); every level: one aggregate per vertex, ids
    0..nc-1 numbered by smallest member, every aggregate connected in the
    level's weight graph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    (n, rp, ci, w), b, s = c3
    L = s.num_levels(0)
    for l in range(L - 1):
        inf = s.level_info(l, 0)
        m, nc = inf["n"], inf["nc"]
        grp, gci = s.level_get(l, "G_rp", 0), s.level_get(l, "G_ci", 0)
        agg = s.level_get(l, "agg", 0)
        assert agg.min() == 0 and agg.max() == nc - 1
        sizes = np.bincount(agg, minlength=nc)
        assert sizes.min() >= 1
        first = np.full(nc, m, dtype=np.int64)
        np.minimum.at(first, agg, np.arange(m))
        assert np.all(np.diff(first) > 0)
        rows = np.repeat(np.arange(m, dtype=np.int32), np.diff(grp))
        keep = agg[rows] == agg[gci]
        intra = sp.csr_matrix((np.ones(int(keep.sum()), np.int8), (rows[keep], gci[keep])), shape=(m, m))
        del rows, keep
        ncomp, _ = connected_components(intra, directed=False)
        assert ncomp == nc, (l, ncomp, nc)
        if l == 0:
            nb = s.level_get(0, "nb", 0).reshape(-1, 2)
            v = np.repeat(np.arange(m), 2)
            u = nb.reshape(-1)
            on = u >= 0
            v, u = v[on], u[on]
            keys = _edge_keys(grp, gci)
            assert np.all(_has_edges(keys, v, u))
            back = nb[u]
            assert np.all((back[:, 0] == v) | (back[:, 1] == v))
            del keys
            pid, pos, plen, npaths = oracle.orient(nb)
            covered = (nb >= 0).any(axis=1)
            assert np.all(pid[covered] >= 0)
            same(s.level_get(0, "path_id", 0), pid)
            same(s.level_get(0, "pos", 0), pos)
            assert inf["npaths"] == npaths
        _log(f"level {l}: n={m} nc={nc} largest aggregate {sizes.max()} joined {inf['middle']}")


def test_powerlaw_solve(c3):
    """FCG(1) with FP32 cycles reaches 1e-8: the FP64 residual recomputed on
    the host from the returned x."""
    import scipy.sparse as sp

    (n, rp, ci, w), b, s = c3
    t = time.time()
    x, st = s.solve()
    x = host(x)
    _log(f"solve {time.time() - t:.1f}s, {st['iterations']} iterations, {st['rebuilds']} rebuilds")
    W = sp.csr_matrix((w, ci, rp), shape=(n, n))
    r = b - (np.asarray(W.sum(axis=1)).ravel() * x - W @ x)
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(b)
