"""GPU parity: every stage of the HIP library against the CPU oracle on the same
seeded inputs.

Bars (written per assertion):
 * integer / index outputs (colours, A^2 pattern, edge order, path cover,
   orientation, aggregates, coarse covers): bit-exact;
 * FP64 kernels whose summation order is defined (Laplacian, Gauss-Seidel,
   residual, Galerkin, prolongation values, cycles, coarsest solve): bit-exact;
 * quantities that pass through global reductions (Alg. 2 PCG steps, norms,
   means, the adaptive loop): relative 1e-12 per vector, iteration counts equal.
"""
import ctypes

import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def host(t):
    return t.detach().cpu().numpy()


def same(a, b):
    """Bit-for-bit equality (floats compared as their bit patterns)."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.dtype.kind == "f":
        assert a.dtype == b.dtype, (a.dtype, b.dtype)
        u = np.uint64 if a.itemsize == 8 else np.uint32
        ne = a.view(u) != b.view(u)
    else:
        ne = a != b
    if ne.any():
        i = np.flatnonzero(ne)[:5]
        raise AssertionError(f"{int(ne.sum())} of {a.size} differ, e.g. idx {i}: {a.ravel()[i]} vs {b.ravel()[i]}")


def close_elementwise(got, ref, rel):
    """Every entry within rel * max|ref| of the reference: the bound of a
    rounding-order change in a sum of products (a dense operator against the
    recursion), checked entry by entry rather than through a norm."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert got.shape == ref.shape
    scale = np.max(np.abs(ref))
    bad = np.abs(got - ref) > rel * scale
    if bad.any():
        i = np.flatnonzero(bad)[:5]
        raise AssertionError(f"{int(bad.sum())} of {got.size} entries beyond {rel} * {scale:.3e}: idx {i}, "
                             f"{got[i]} vs {ref[i]}")


GRAPHS = {
    "grid64": lambda: I.grid2d(64, 64),
    "grid3d_w": lambda: I.grid3d(17, 13, 11, weight_seed=3),
    "rgg": lambda: I.rgg(5000, 11),
    "ring": lambda: I.ring(3001, 4),
    "ba": lambda: I.csr_from_edges(*I.ba_edges(2000, 5), I.log_uniform_weights(6, len(I.ba_edges(2000, 5)[1]),
                                                                               -2, 2)),
    "hub": lambda: hub_graph(),
}


def hub_graph():
    """Ring lattice plus one hub joined to every 5th vertex: its A^2 row and the
    coarse rows around it take the long-row paths."""
    n0, a, b = I.ring_edges(3000, 4)
    hub = np.full(600, 3000)
    a2, b2 = I.canonical_edges(np.concatenate([a, hub]), np.concatenate([b, np.arange(0, 3000, 5)]))
    return I.csr_from_edges(3001, a2, b2, I.log_uniform_weights(4, len(a2), -1, 1))


@pytest.fixture(scope="module", params=list(GRAPHS))
def graph(request):
    return request.param, GRAPHS[request.param]()


def test_laplacian_colour_gs_residual(gpu, oracle, graph):
    name, g = graph
    n, rp, ci, w = g
    S = gpu.stages
    a, d, dinv = S.laplacian(rp, ci, w)
    ra, rd, rdinv = oracle.laplacian(g)
    same(host(a), ra)
    same(host(d), rd)
    same(host(dinv), rdinv)
    for level in (0, 5):
        col, nc = S.colour(rp, ci, 0xC010, level)
        rcol, rnc = oracle.colour(n, rp, ci, 0xC010, level)
        assert nc == rnc
        same(host(col), rcol)
    col, nc = oracle.colour(n, rp, ci, 0xC010, 0)
    b = I.normal(1, n)
    x0 = I.normal(2, n)
    for fwd in (True, False):
        got = S.gs(rp, ci, ra, rdinv, col, nc, b, x0, forward=fwd, count=2)
        ref = oracle.gs(n, rp, ci, ra, rdinv, col, nc, b, x0, forward=fwd, count=2)
        same(host(got), ref)
    same(host(S.residual(rp, ci, ra, rd, b, x0)), oracle.residual(n, rp, ci, ra, rd, b, x0))


def test_a2_sort_cover_orient(gpu, oracle, graph):
    name, g = graph
    n, rp, ci, w = g
    S = gpu.stages
    rp2, ci2 = S.a2_pattern(rp, ci)
    orp2, oci2 = oracle.a2_pattern(n, rp, ci)
    same(host(rp2), orp2)
    same(host(ci2), oci2)
    e = oracle.smooth_error(g, 0xC010, 7, 3)
    su, sv = S.sort_edges(orp2, oci2, e)
    osu, osv = oracle.sorted_edges(n, orp2, oci2, e)
    same(host(su), osu)
    same(host(sv), osv)
    nb = S.path_cover(n, osu, osv)
    onb = oracle.path_cover(n, osu, osv)
    same(np.sort(host(nb), axis=1), np.sort(onb, axis=1))
    pid, pos, plen = S.orient(onb)
    opid, opos, oplen, _ = oracle.orient(onb)
    same(host(pid), opid)
    same(host(pos), opos)
    same(host(plen), oplen)


def test_a2_hub_cap(gpu, oracle):
    g = GRAPHS["ba"]()
    n, rp, ci, w = g
    rp2, ci2 = gpu.stages.a2_pattern(rp, ci, hub_cap=20)
    orp2, oci2 = oracle.a2_pattern(n, rp, ci, 20)
    same(host(rp2), orp2)
    same(host(ci2), oci2)


def test_path_cover_adversarial_orders(gpu, oracle):
    """Random edge orders on dense random graphs: many conflicts per round."""
    rng = np.random.default_rng(0)
    for t in range(6):
        n = int(rng.integers(50, 3000))
        m = int(rng.integers(n, 8 * n))
        a, b = I.canonical_edges(rng.integers(0, n, m), rng.integers(0, n, m))
        order = rng.permutation(len(a))
        su, sv = a[order].astype(np.int32), b[order].astype(np.int32)
        nb = gpu.stages.path_cover(n, su, sv)
        onb = oracle.path_cover(n, su, sv)
        same(np.sort(host(nb), axis=1), np.sort(onb, axis=1))


def test_aggregate_galerkin_shorten(gpu, oracle, graph):
    name, g = graph
    n = g[0]
    H = oracle.Hierarchy(g, None, coarse_max=16)
    S = gpu.stages
    for level in range(min(H.nlevels - 1, 4)):
        grp, gci, gv = H.get_int(level, "G_rp"), H.get_int(level, "G_ci"), H.get_dbl(level, "G_v")
        gkey = H.get_dbl(level, "gkey") if level == 0 else None
        nb = H.get_int(level, "nb")
        agg, nc, st = S.aggregate(grp, gci, gv, nb, gkey)
        ragg, rnc, rst = oracle.aggregate(len(grp) - 1, grp, gci, gv, nb, gkey)
        assert nc == rnc and st == rst
        same(host(agg), ragg)
        same(ragg, H.get_int(level, "agg"))
        rp, ci, av, d = H.level_matrix(level)
        pv = H.get_dbl(level, "pval")
        rpc, cic, vc, dc = S.galerkin(rp, ci, av, d, nc, ragg, pv)
        orpc, ocic, ovc, odc = oracle.galerkin(len(rp) - 1, rp, ci, av, d, nc, ragg, pv)
        same(host(rpc), orpc)
        same(host(cic), ocic)
        same(host(vc), ovc)
        same(host(dc), odc)
        nbc = S.shorten(nb, nc, ragg)
        same(host(nbc), oracle.shorten(nb, nc, ragg))


def solver_for(gpu, g, b=None, **kw):
    """Solver with per-level arrays kept; W- and V-cycles recurse (w_dense = 0,
    v_dense_max_n = 0) unless asked otherwise, so every cycle is the oracle's
    bit for bit."""
    n, rp, ci, w = g
    if b is None:
        b = I.zero_mean_normal_rhs(99, n)
    kw.setdefault("w_dense", 0)
    kw.setdefault("v_dense_max_n", 0)
    return gpu.Solver(rp, ci, w, b, keep_setup=1, **kw)


def compare_hierarchy(s, H, h=-1):
    assert s.num_levels(h) == H.nlevels
    for l in range(H.nlevels):
        gi, oi = s.level_info(l, h), H.info(l)
        for k in ("n", "nnz", "ncolours", "nc", "nnz_G", "npaths", "n_unagg", "case1", "case2", "case3", "middle",
                  "singleton", "p1_fallback", "grounded", "coarse_fallback", "n_path_vertices"):
            if l == H.nlevels - 1 and k in ("nnz_G",):
                continue
            assert gi[k] == oi[k], (l, k, gi[k], oi[k])
        for name in ("colour", "A_rp", "A_ci", "A_v", "d", "dinv"):
            same(s.level_get(l, name, h), H.get_int(l, name) if name[0] in "cA" and name != "A_v" else
                 H.get_dbl(l, name))
        if l + 1 < H.nlevels:
            for name in ("agg", "path_id", "pos", "G_rp", "G_ci"):
                same(s.level_get(l, name, h), H.get_int(l, name))
            same(s.level_get(l, "G_v", h), H.get_dbl(l, "G_v"))
            same(np.sort(s.level_get(l, "nb", h).reshape(-1, 2), axis=1),
                 np.sort(H.get_int(l, "nb").reshape(-1, 2), axis=1))
            opv = H.get_dbl(l, "pval")
            if l == 0 and not np.all(opv == 1.0):  # smooth prolongation values on level 1
                same(s.level_get(l, "pval", h), opv)
            else:  # boolean levels: the library stores no values
                assert np.all(opv == 1.0)
    same(s.level_get(0, "gkey", h), H.get_dbl(0, "gkey"))


@pytest.mark.parametrize("p1", ["smooth", "const"])
def test_first_hierarchy_bit_exact(gpu, oracle, graph, p1):
    name, g = graph
    s = solver_for(gpu, g, p1_mode=p1)
    H = oracle.Hierarchy(g, None, p1_mode=0 if p1 == "smooth" else 1)
    same(host(s.initial_error()), H.get_dbl(0, "e"))
    compare_hierarchy(s, H)


def test_rebuild_from_given_error(gpu, oracle):
    g = GRAPHS["grid3d_w"]()
    n = g[0]
    e = I.normal(5, n)
    s = solver_for(gpu, g)
    s.rebuild(torch.as_tensor(e, device="cuda"))
    # the library relaxes e (3 symmetric sweeps on A e = 0) before building
    H = oracle.Hierarchy(g, e_relaxed(oracle, g, e))
    compare_hierarchy(s, H, h=1)


@pytest.mark.parametrize("gname", ["grid64", "grid3d_w", "rgg"])
def test_cycles_bit_exact(gpu, oracle, gname):
    g = GRAPHS[gname]()
    n = g[0]
    s = solver_for(gpu, g)
    H = oracle.Hierarchy(g, None)
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    for gamma in (1, 2):
        same(host(s.cycle(b, x0, gamma)), H.cycle(b, x0, gamma))
    b32 = b.astype(np.float32)
    same(host(s.cycle32(b32)), H.vcycle32(b32))
    x32 = x0.astype(np.float32)
    same(host(s.cycle32(b32, x32, 2)), H.cycle32(b32, x32, 2))
    # coarsest grounded case (boolean prolongations)
    sc = solver_for(gpu, g, p1_mode="const")
    Hc = oracle.Hierarchy(g, None, p1_mode=1)
    same(host(sc.cycle(b, None, 1)), Hc.vcycle(b))


@pytest.mark.parametrize("gname", ["hub", "powerlaw"])
def test_long_rows_cycles(gpu, oracle, gname):
    """Rows of 256 entries or more (hubs) take one workgroup each in the
    cycles, with a fixed summation tree: the same hierarchy (the relaxation
    before a build keeps the single chain), cycles within rounding of the
    oracle (FP64 1e-12, FP32 1e-5 relative); with long_row_min = 0 the cycles
    are the oracle's bit for bit."""
    g = GRAPHS["hub"]() if gname == "hub" else I.config3(n0=30000)[0]
    n = g[0]
    H = oracle.Hierarchy(g, None)
    s0 = solver_for(gpu, g, long_row_min=0)
    s = solver_for(gpu, g)
    compare_hierarchy(s, H)
    long_levels = 0
    for l in range(s.num_levels()):
        m = s.level_info(l)["n"]
        if m > 2048 and np.diff(s.level_get(l, "A_rp")).max() >= 256:
            long_levels += 1
    assert long_levels >= 1
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    b32, x32 = b.astype(np.float32), x0.astype(np.float32)
    for gamma in (1, 2):
        ref = H.cycle(b, x0, gamma)
        same(host(s0.cycle(b, x0, gamma)), ref)
        got = host(s.cycle(b, x0, gamma))
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), gamma
        ref32 = H.cycle32(b32, x32, gamma).astype(np.float64)
        same(host(s0.cycle32(b32, x32, gamma)).astype(np.float64), ref32)
        got32 = host(s.cycle32(b32, x32, gamma)).astype(np.float64)
        assert np.linalg.norm(got32 - ref32) <= 1e-5 * np.linalg.norm(ref32), gamma
    # the solve converges the same way
    xs, st = s.solve()
    x0s, st0 = s0.solve()
    assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8
    assert abs(st["iterations"] - st0["iterations"]) <= 1


def test_approx_error(gpu, oracle):
    """Alg. 2 with one hierarchy (W-cycle preconditioner), relative 1e-12."""
    g = GRAPHS["grid3d_w"]()
    n = g[0]
    s = solver_for(gpu, g)
    H1 = oracle.Hierarchy(g, None)
    r = I.zero_mean_normal_rhs(8, n)
    e1 = host(s.approx_error(r, count=1))
    o1 = oracle.approximate_error([H1], r)
    assert np.linalg.norm(e1 - o1) <= 1e-12 * np.linalg.norm(o1)


def e_relaxed(oracle, g, e):
    n, rp, ci, w = g
    a, d, dinv = oracle.laplacian(g)
    col, nc = oracle.colour(n, rp, ci, 0xC010, 0)
    z = np.zeros(n)
    e = np.array(e, float)
    for _ in range(3):
        e = oracle.gs(n, rp, ci, a, dinv, col, nc, z, e, True)
        e = oracle.gs(n, rp, ci, a, dinv, col, nc, z, e, False)
    return e


def test_composite_approx_error(gpu, oracle):
    g = GRAPHS["grid64"]()
    n = g[0]
    s = solver_for(gpu, g)
    e2, e3 = I.normal(31, n), I.normal(32, n)
    s.rebuild(torch.as_tensor(e2, device="cuda"))
    s.rebuild(torch.as_tensor(e3, device="cuda"))
    Hs = [oracle.Hierarchy(g, None), oracle.Hierarchy(g, e_relaxed(oracle, g, e2)),
          oracle.Hierarchy(g, e_relaxed(oracle, g, e3))]
    r = I.zero_mean_normal_rhs(9, n)
    for count in (1, 2, 3):
        got = host(s.approx_error(r, count=count))
        ref = oracle.approximate_error(Hs[:count], r)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), count
    # FP32 preconditioning cycles (W for Re <= numW, composite after): the FP32
    # cycles are bit-exact, the PCG scalars go through reductions
    s32 = solver_for(gpu, g, cycle_prec="f32")
    s32.rebuild(torch.as_tensor(e2, device="cuda"))
    s32.rebuild(torch.as_tensor(e3, device="cuda"))
    for count in (1, 3):
        got = host(s32.approx_error(r, count=count))
        ref = oracle.approximate_error(Hs[:count], r, cycle_prec=1)
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref), count


@pytest.mark.parametrize("kw", [dict(), dict(p1_mode="const"), dict(outer="fcg", cycle_prec="f32", theta=0.5),
                                dict(outer="fcg", cycle_prec="f64", theta=0.5), dict(theta=1e-6)])
def test_solve_matches_oracle(gpu, oracle, kw):
    g, b = I.config1()
    okw = {k: {"const": 1, "smooth": 0, "fcg": 1, "f32": 1, "f64": 0}.get(v, v) for k, v in kw.items()}
    ref = oracle.solve(g, b, **okw)
    s = solver_for(gpu, g, b, **kw)
    x, st = s.solve()
    assert st["status"] == 0
    assert st["iterations"] == ref.stats["iterations"]
    assert st["rebuilds"] == ref.stats["rebuilds"]
    assert st["true_relres"] <= 1.0001e-8
    # Until the first re-setup every step is reproduced (reductions aside); a
    # re-setup's smooth error comes from Alg. 2's PCG, whose dot products feed
    # the key order, so later hierarchies may differ at near-ties of the keys.
    hist = st["relres_hist"]
    k1 = (int(ref.rebuild_at[0]) if len(ref.rebuild_at) else len(hist) - 1) + 1
    assert np.allclose(hist[:k1], ref.relres_hist[:k1], rtol=1e-10, atol=0)
    xs = host(x)
    assert np.linalg.norm(xs - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_solve_3d_weighted(gpu, oracle):
    """Default settings (dense W sub-cycle operator included): the same
    convergence as the oracle within one iteration and one re-setup."""
    g = I.grid3d(24, 24, 24, weight_seed=1)
    b = I.zero_mean_normal_rhs(5, g[0])
    for kw, okw in [(dict(theta=0.5, w_dense=1), dict(theta=0.5)),
                    (dict(outer="fcg", cycle_prec="f32", theta=0.5, w_dense=1),
                     dict(outer=1, cycle_prec=1, theta=0.5))]:
        ref = oracle.solve(g, b, **okw)
        s = solver_for(gpu, g, b, **kw)
        x, st = s.solve()
        assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8
        assert abs(st["iterations"] - ref.stats["iterations"]) <= 1
        assert abs(st["rebuilds"] - ref.stats["rebuilds"]) <= 1


def test_lanes_settings_identical(gpu):
    """Lanes per row only change how a row's operands reach its fma chain:
    the heuristic, the autotuned choice (row_lanes = -1) and forced 4 / 16
    lanes give the same solve bit for bit (FP32 cycles inside FCG and FP64
    V-cycles, dense W operator included)."""
    g = I.grid3d(40, 36, 32, weight_seed=4)
    b = I.zero_mean_normal_rhs(6, g[0])
    for kw in (dict(outer="fcg", cycle_prec="f32", theta=0.5, w_dense=1), dict(theta=0.5)):
        ref = None
        for lanes in (0, -1, 4, 16):
            s = solver_for(gpu, g, b, row_lanes=lanes, **kw)
            x, st = s.solve()
            assert st["status"] == 0
            got = (host(x), st["iterations"], st["rebuilds"])
            if ref is None:
                ref = got
            else:
                same(got[0], ref[0])
                assert got[1:] == ref[1:]


def test_edge_cases(gpu, oracle):
    # tiny graphs: a single level (n <= coarse_max) is a direct grounded solve
    for g in (I.path(2), I.path(3), I.grid2d(3, 3)):
        n = g[0]
        b = I.zero_mean_normal_rhs(1, n)
        s = solver_for(gpu, g, b)
        x, st = s.solve()
        assert st["iterations"] == 1 and st["true_relres"] <= 1e-12
        same(host(x), oracle.solve(g, b).x)
    # forced coarsening of the worked example
    g = I.grid2d(3, 3)
    s = solver_for(gpu, g, coarse_max=1)
    e = np.array([x + y for y in range(3) for x in range(3)], float)
    s.rebuild(torch.as_tensor(e, device="cuda"))
    H = oracle.Hierarchy(g, e_relaxed(oracle, g, e), coarse_max=1)
    compare_hierarchy(s, H, h=1)
    # zero rhs returns at once
    g = I.grid2d(10, 10)
    s = solver_for(gpu, g, np.zeros(100))
    x, st = s.solve()
    assert st["iterations"] == 0 and float(x.abs().max()) == 0.0


def test_edge_cases_default_settings(gpu, oracle):
    """The library defaults (dense V and W operators, hub rows on workgroups,
    autotuning off) on small and shallow hierarchies: one level, two levels,
    a coarsest level right below the dense start, forced deep coarsening; the
    solve reaches 1e-8 and agrees with the oracle's answer (to 1e-4: two
    solutions at 1e-8 relative residual differ by up to the condition number
    times that)."""
    import paper_1806_07028_amd as P
    cases = [(I.path(3), {}), (I.grid2d(9, 9), {}), (I.grid2d(40, 40), {}), (I.grid2d(12, 12), dict(coarse_max=2)),
             (I.grid3d(14, 14, 14, weight_seed=2), dict(v_dense_max_n=100000)),
             (GRAPHS["hub"](), {}), (I.config3(n0=8000)[0], {})]
    for g, kw in cases:
        n = g[0]
        b = I.zero_mean_normal_rhs(2, n)
        s = P.Solver(g[1], g[2], g[3], b, **kw)
        x, st = s.solve()
        assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8, (n, kw, st["true_relres"])
        for gamma in (1, 2):
            s.cycle(b, None, gamma)
            s.cycle32(b.astype(np.float32), None, gamma)
        ref = oracle.solve(g, b, **{k: v for k, v in kw.items() if k == "coarse_max"})
        xs = host(x)
        assert np.linalg.norm(xs - ref.x) <= 1e-4 * np.linalg.norm(ref.x), (n, kw)
        s.close()


def test_errors(gpu):
    import paper_1806_07028_amd as P

    n, rp, ci, w = I.grid2d(5, 5)
    b = I.zero_mean_normal_rhs(1, n)
    with pytest.raises(P.PcamgError) as ei:
        P.Solver(rp, ci, w, b + 1.0)
    assert ei.value.status == -7
    w2 = w.copy()
    w2[3] = -1.0
    with pytest.raises(P.PcamgError) as ei:
        P.Solver(rp, ci, w2, b)
    assert ei.value.status in (-5, -2)
    w3 = w.copy()
    w3[0] *= 2.0
    with pytest.raises(P.PcamgError) as ei:
        P.Solver(rp, ci, w3, b)
    assert ei.value.status == -2
    # two components
    n2, a2, b2 = I.grid2d_edges(4, 4)
    a2 = np.concatenate([a2, a2 + 16])
    b2 = np.concatenate([b2, b2 + 16])
    g = I.csr_from_edges(32, a2, b2, np.ones(len(a2)))
    with pytest.raises(P.PcamgError) as ei:
        P.Solver(g[1], g[2], g[3], I.zero_mean_normal_rhs(1, 32))
    assert ei.value.status == -6
    # max_iter reached
    g, b = I.config1()
    s = P.Solver(g[1], g[2], g[3], b, max_iter=2, theta=1e9)
    x, st = s.solve(raise_on_noconv=False)
    assert st["status"] == -10 and st["iterations"] == 2


def test_stage_null_entry_arrays(gpu):
    """Stage entry points refuse a null array indexed by stored entry when the
    pattern has entries (checked on the host before any launch), and accept
    one for a pattern without entries."""
    import torch

    from paper_1806_07028_amd import stages as S
    from paper_1806_07028_amd._lib import lib

    n, rp, ci, w = I.grid2d(5, 4)
    st = torch.cuda.current_stream().cuda_stream
    rpd = torch.as_tensor(rp, dtype=torch.int32, device="cuda")
    cid = torch.as_tensor(ci, dtype=torch.int32, device="cuda")
    wd = torch.as_tensor(w, dtype=torch.float64, device="cuda")
    out = torch.empty(len(ci) + 2 * n, dtype=torch.float64, device="cuda")
    a_p, d_p, dinv_p = out.data_ptr(), out.data_ptr() + 8 * len(ci), out.data_ptr() + 8 * (len(ci) + n)
    assert lib().pcamg_laplacian(n, rpd.data_ptr(), cid.data_ptr(), None, a_p, d_p, dinv_p, st) == -1
    assert lib().pcamg_laplacian(n, rpd.data_ptr(), cid.data_ptr(), wd.data_ptr(), None, d_p, dinv_p, st) == -1
    col = torch.zeros(n, dtype=torch.int32, device="cuda")
    nc = ctypes.c_int32()
    assert lib().pcamg_colour(n, rpd.data_ptr(), None, 7, 0, col.data_ptr(), ctypes.byref(nc), st) == -1
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    assert lib().pcamg_gs(n, rpd.data_ptr(), cid.data_ptr(), a_p, None, col.data_ptr(), 1, x.data_ptr(),
                          x.data_ptr(), 1, 1, st) == -1
    assert lib().pcamg_residual(n, rpd.data_ptr(), None, a_p, d_p, x.data_ptr(), x.data_ptr(), x.data_ptr(),
                                st) == -1
    # the library still works after the refusals
    a, d, dinv = S.laplacian(rp, ci, w)
    assert np.array_equal(host(a), -w)
    # no stored entries: null entry arrays are fine
    rp0 = torch.zeros(4, dtype=torch.int32, device="cuda")
    d0 = torch.empty(6, dtype=torch.float64, device="cuda")
    assert lib().pcamg_laplacian(3, rp0.data_ptr(), None, None, None, d0.data_ptr(), d0.data_ptr() + 24, st) == 0
    assert (host(d0[:3]) == 0.0).all()


@pytest.mark.parametrize("gname", ["grid3d_20", "grid2d_128"])
def test_dense_w_cycle(gpu, oracle, gname):
    """W-cycles with the two tail sub-cycles applied as one precomputed dense
    operator: the same linear map as the recursion, different rounding order.
    FP64 within 1e-12 relative, FP32 within 1e-5 relative of the recursive
    cycle; graph replays equal the eager dense cycle bit for bit."""
    g = I.grid3d(20, 20, 20, weight_seed=7) if gname == "grid3d_20" else I.grid2d(128, 128, weight_seed=2)
    n = g[0]
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    rec = solver_for(gpu, g)
    dense = solver_for(gpu, g, w_dense=1, dense_max_n=6144)
    dense_eager = solver_for(gpu, g, w_dense=1, use_graphs=0, dense_max_n=6144)
    H = oracle.Hierarchy(g, None)
    assert dense.num_levels() == H.nlevels >= 4
    w_ref = H.cycle(b, x0, 2)
    same(host(rec.cycle(b, x0, 2)), w_ref)
    w64 = host(dense.cycle(b, x0, 2))
    close_elementwise(w64, w_ref, 1e-12)
    assert not np.array_equal(w64, w_ref)  # the dense path is really taken
    b32 = b.astype(np.float32)
    w32_ref = H.cycle32(b32, None, 2)
    w32 = host(dense.cycle32(b32, None, 2))
    close_elementwise(w32, w32_ref, 1e-5)
    e64 = host(dense_eager.cycle(b, x0, 2))
    e32 = host(dense_eager.cycle32(b32, None, 2))
    for rep in range(3):
        same(host(dense.cycle(b, x0, 2)), e64)
        same(host(dense.cycle32(b32, None, 2)), e32)
        dense_eager.cycle(b, None, 1)
        torch.cuda.synchronize()
    # V-cycles are untouched
    same(host(dense.cycle(b, x0, 1)), H.cycle(b, x0, 1))


@pytest.mark.parametrize("gname", ["grid40", "ba"])
def test_dense_whole_cycle_small_graph(gpu, oracle, gname):
    """With top_dense_max_n, a graph of at most 2048 vertices runs each cycle
    type as one dense operator C of the whole cycle, applied from any start vector as
    x + C (b - A x) (a cycle is affine in x and fixes the exact solutions):
    V- and W-cycles from a nonzero start within 1e-12 (FP64) and 1e-5 (FP32)
    of the oracle's recursive cycles, entry by entry; the dense path is
    really taken (its rounding differs from the recursion's); graph replays
    equal the eager cycles bit for bit; the default solve reaches 1e-8."""
    import paper_1806_07028_amd as P
    g = I.grid2d(40, 40) if gname == "grid40" else GRAPHS["ba"]()
    n = g[0]
    assert n <= 2048
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    kw = dict(v_dense_max_n=4096, w_dense=1, long_row_min=0, top_dense_max_n=2048)
    dense = solver_for(gpu, g, **kw)
    dense_eager = solver_for(gpu, g, use_graphs=0, **kw)
    recursive = solver_for(gpu, g, long_row_min=0)
    H = oracle.Hierarchy(g, None)
    assert dense.num_levels() == H.nlevels >= 3
    b32, x32 = b.astype(np.float32), x0.astype(np.float32)
    for gamma in (1, 2):
        ref = H.cycle(b, x0, gamma)
        got = host(dense.cycle(b, x0, gamma))
        close_elementwise(got, ref, 1e-12)
        same(host(recursive.cycle(b, x0, gamma)), ref)  # the recursion is the oracle's bit for bit ...
        assert not np.array_equal(got, ref)  # ... the dense operator is not
        ref32 = H.cycle32(b32, x32, gamma).astype(np.float64)
        got32 = host(dense.cycle32(b32, x32, gamma)).astype(np.float64)
        close_elementwise(got32, ref32, 1e-5)
        e64 = host(dense_eager.cycle(b, x0, gamma))
        e32 = host(dense_eager.cycle32(b32, x32, gamma))
        for rep in range(2):
            same(host(dense.cycle(b, x0, gamma)), e64)
            same(host(dense.cycle32(b32, x32, gamma)), e32)
    for prec in ("f64", "f32"):
        s = P.Solver(g[1], g[2], g[3], b, outer="fcg", cycle_prec=prec, theta=0.5, top_dense_max_n=2048)
        x, st = s.solve()
        assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8, (prec, st["true_relres"])
        s.close()


@pytest.mark.parametrize("gname", ["grid3d_20", "powerlaw"])
def test_dense_v_cycle(gpu, oracle, gname):
    """V-cycles with the cycle of the first level of at most 2048 vertices
    applied as one precomputed dense operator: the same linear map as the
    recursion, different rounding order. FP64 within 1e-12 relative, FP32
    within 1e-5 relative of the oracle's recursive cycle; graph replays equal
    the eager dense cycle bit for bit; W-cycles untouched.  On the power-law
    graph the operator's near-dense levels (more than one colour per 8 rows)
    are built with blocked dense sweeps (GEMMs and 32-row triangular blocks)
    instead of colour passes."""
    g = I.grid3d(20, 20, 20, weight_seed=7) if gname == "grid3d_20" else I.config3(n0=30000)[0]
    n = g[0]
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    kw = dict(long_row_min=0)  # hub rows by the single chain, as in the oracle
    dense = solver_for(gpu, g, v_dense_max_n=2048, **kw)
    dense_eager = solver_for(gpu, g, v_dense_max_n=2048, use_graphs=0, **kw)
    H = oracle.Hierarchy(g, None)
    assert dense.num_levels() == H.nlevels >= 4
    sizes = [dense.level_info(l)["n"] for l in range(dense.num_levels())]
    assert sizes[1] > 2048  # a launched level applies the operator below it
    if gname == "powerlaw":  # the blocked dense sweeps are taken
        infos = [dense.level_info(l) for l in range(dense.num_levels())]
        assert any(i["n"] <= 2048 and 8 * i["ncolours"] > i["n"] for i in infos[:-1])
    v_ref = H.cycle(b, x0, 1)
    v64 = host(dense.cycle(b, x0, 1))
    close_elementwise(v64, v_ref, 1e-12)
    # a smooth right-hand side, whose solution comes mostly from the coarse
    # levels: the dense path is really taken (its rounding shows)
    a, d, dinv = oracle.laplacian(g)
    e = H.get_dbl(0, "e")
    bs = d * e + np.bincount(np.repeat(np.arange(n), np.diff(g[1])), weights=a * e[g[2]], minlength=n)
    bs -= bs.mean()
    vs_ref = H.cycle(bs, None, 1)
    vs = host(dense.cycle(bs, None, 1))
    close_elementwise(vs, vs_ref, 1e-12)
    assert not np.array_equal(vs, vs_ref)
    b32 = b.astype(np.float32)
    v32_ref = H.vcycle32(b32).astype(np.float64)
    v32 = host(dense.cycle32(b32)).astype(np.float64)
    close_elementwise(v32, v32_ref, 1e-5)
    e64 = host(dense_eager.cycle(b, x0, 1))
    e32 = host(dense_eager.cycle32(b32))
    for rep in range(3):
        same(host(dense.cycle(b, x0, 1)), e64)
        same(host(dense.cycle32(b32)), e32)
        dense_eager.cycle(b, None, 2)
        torch.cuda.synchronize()
    same(host(dense.cycle(b, x0, 2)), H.cycle(b, x0, 2))
    # the solve converges as with recursive V-cycles
    rec = solver_for(gpu, g, b, **kw)
    x, st = solver_for(gpu, g, b, v_dense_max_n=2048, **kw).solve()
    xr, str_ = rec.solve()
    assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8
    assert abs(st["iterations"] - str_["iterations"]) <= 1


@pytest.mark.parametrize("gname", ["grid3d_w", "hub"])
def test_graph_and_tail_equal_eager(gpu, gname):
    """Whole cycles replayed from captured graphs, with the small levels in the
    single-workgroup tail kernel, equal the eager per-step launches bit for bit
    on every replay (eager work and synchronisations between replays)."""
    g = GRAPHS[gname]() if gname != "grid3d_w" else I.grid3d(20, 20, 20, weight_seed=7)
    n = g[0]
    b = I.zero_mean_normal_rhs(3, n)
    x0 = I.normal(4, n)
    eager = solver_for(gpu, g, use_graphs=0, tail_max_n=0)
    fused = solver_for(gpu, g)
    ref1 = host(eager.cycle(b, x0, 1))
    ref2 = host(eager.cycle(b, x0, 2))
    ref32 = host(eager.cycle32(b.astype(np.float32)))
    ref32w = host(eager.cycle32(b.astype(np.float32), None, 2))
    for rep in range(4):
        same(host(fused.cycle(b, x0, 1)), ref1)
        eager.cycle(b, None, 1)
        torch.cuda.synchronize()
        same(host(fused.cycle(b, x0, 2)), ref2)
        same(host(fused.cycle32(b.astype(np.float32))), ref32)
        same(host(fused.cycle32(b.astype(np.float32), None, 2)), ref32w)


BATCH_SKIP = pytest.mark.skip(
    reason="multi-threaded batch path: one run ended in a host segmentation fault inside pcamg_batch_solve "
           "(after dense-operator builds with rocBLAS joined it); cause not shown, so the path is switched off "
           "(the library refuses workers > 1) and the case stays off the GPU until the cause is found")


def _batch_equals_individual(gpu, oracle, workers):
    batch = I.config4(seed=3, count=12, n_lo=400, n_hi=20000)
    graphs = [(g[1], g[2], g[3]) for g, b, k in batch]
    rhs = [b for g, b, k in batch]
    ref = []
    for (g, b, k) in batch:
        s = gpu.Solver(g[1], g[2], g[3], b)
        x, st = s.solve()
        ref.append((host(x), st))
        s.close()
    for rep in range(2):
        xs, sts = gpu.batch_solve(graphs, rhs, workers=workers)
        for i, ((xr, sr), x, st) in enumerate(zip(ref, xs, sts)):
            same(host(x), xr)
            for key in ("iterations", "rebuilds", "levels", "status"):
                assert st[key] == sr[key], (i, key)
            assert st["true_relres"] <= 1.0001e-8
    for (g, b, k), (xr, sr) in zip(batch, ref):
        if g[0] <= 3000:
            o = oracle.solve(g, b)
            assert o.stats["iterations"] == sr["iterations"] and o.stats["rebuilds"] == sr["rebuilds"]


@BATCH_SKIP
def test_batch_equals_individual(gpu, oracle):
    """Batched setup + solve of uneven graphs on four worker streams: every
    graph's solution and statistics equal its own single-graph solve bit for
    bit, on a first and a second batch (the second reuses cached memory across
    streams); the small graphs also match the oracle's counts."""
    _batch_equals_individual(gpu, oracle, 4)


def test_batch_one_worker_equals_individual(gpu, oracle):
    """The same with one worker (the graphs one after another on the calling
    thread, no host threads)."""
    _batch_equals_individual(gpu, oracle, 1)


def _batch_errors(gpu, workers):
    batch = I.config4(seed=5, count=5, n_lo=300, n_hi=3000)
    graphs = [(g[1], g[2], g[3]) for g, b, k in batch]
    rhs = [b for g, b, k in batch]
    n2, a2, b2 = I.grid2d_edges(4, 4)
    bad = I.csr_from_edges(32, np.concatenate([a2, a2 + 16]), np.concatenate([b2, b2 + 16]), np.ones(2 * len(a2)))
    graphs.insert(2, (bad[1], bad[2], bad[3]))
    rhs.insert(2, I.zero_mean_normal_rhs(1, 32))
    xs, sts = gpu.batch_solve(graphs, rhs, workers=workers[0], raise_on_error=False)
    assert sts[2]["status"] == -6
    for i, st in enumerate(sts):
        if i != 2:
            assert st["status"] == 0 and st["true_relres"] <= 1.0001e-8
    import paper_1806_07028_amd as P
    with pytest.raises(P.PcamgError) as ei:
        gpu.batch_solve(graphs, rhs, workers=workers[1])
    assert ei.value.status == -6
    xs, sts = gpu.batch_solve([], [], workers=workers[1])
    assert xs == [] and sts == []


@BATCH_SKIP
def test_batch_errors(gpu):
    """A disconnected graph fails on its own (its status), the others are solved."""
    _batch_errors(gpu, (3, 2))


def test_batch_errors_one_worker(gpu):
    """The same with one worker on the calling thread."""
    _batch_errors(gpu, (1, 1))


def test_batch_several_workers_refused(gpu):
    """Several host threads are switched off: the call fails before any graph
    is touched."""
    import paper_1806_07028_amd as P

    (n, rp, ci, w), b = I.config1()
    x0 = np.full(n, 7.0)
    for workers in (0, 2, 4):
        with pytest.raises(P.PcamgError) as ei:
            gpu.batch_solve([(rp, ci, w)], [b], x0=[x0], workers=workers)
        assert ei.value.status == -1
    xs, sts = gpu.batch_solve([(rp, ci, w)], [b], workers=1)
    assert sts[0]["status"] == 0 and sts[0]["true_relres"] <= 1.0001e-8


def test_colour_dense_levels(gpu, oracle):
    """Near-dense graphs (more than 48 entries per row) of up to 8192
    vertices take the one-vertex-at-a-time greedy kernel (order sorted in
    LDS), the others the data-driven Jones-Plassmann rounds (long priority
    chains: the power-law graph's first rounds colour a few dozen of its
    99,090 vertices each; hub rows of more than 256 entries get their
    higher-priority lists from a workgroup each): all equal the oracle's
    first-fit in priority order."""
    S = gpu.stages
    cases = []
    n = 300  # complete graph
    a, b = np.triu_indices(n, 1)
    cases.append(I.csr_from_edges(n, a, b, np.ones(len(a))))
    n = 2500  # random dense graph, mean degree ~150
    u = I.uniform(77, 2 * 190000)
    a = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
    b = np.minimum((u[1::2] * n).astype(np.int64), n - 1)
    m = a != b
    a2, b2 = I.canonical_edges(a[m], b[m])
    cases.append(I.csr_from_edges(n, a2, b2, np.ones(len(a2))))
    cases.append(I.rgg(2500, 5))  # sparse, same size range
    cases.append(I.config3(n0=100000)[0])
    for n, deg, seed in ((3000, 60, 78), (20000, 60, 79), (20000, 40, 80)):
        u = I.uniform(seed, 2 * n * deg // 2)
        a = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
        b = np.minimum((u[1::2] * n).astype(np.int64), n - 1)
        m = a != b
        a2, b2 = I.canonical_edges(a[m], b[m])
        cases.append(I.csr_from_edges(n, a2, b2, np.ones(len(a2))))
    for g in cases:
        n, rp, ci, w = g
        for level in (0, 3):
            col, nc = S.colour(rp, ci, 0xC010, level)
            rcol, rnc = oracle.colour(n, rp, ci, 0xC010, level)
            assert nc == rnc
            same(host(col), rcol)


def _star(n):
    a = np.zeros(n - 1, dtype=np.int64)
    b = np.arange(1, n, dtype=np.int64)
    return I.csr_from_edges(n, a, b, np.ones(n - 1))


def _two_grids():
    n1, a1, b1 = I.grid2d_edges(30, 20)
    a = np.concatenate([a1, a1 + n1])
    b = np.concatenate([b1, b1 + n1])
    return I.csr_from_edges(2 * n1, a, b, np.ones(len(a)))


@pytest.mark.parametrize("name,make", [
    ("grid3d_64", lambda: I.grid3d(64, 64, 64)),   # bipartite, 190 frontier rounds
    ("path_3000", lambda: I.path(3000)),           # bipartite, 2999 rounds
    ("star_5000", lambda: _star(5000)),            # one round claims n - 1 vertices
    ("ring_4001", lambda: I.ring(4001, 2)),         # odd cycle seen only at depth 2000
    ("two_grids", _two_grids),                     # bipartite but not connected
    ("single", lambda: I.path(1)),
])
def test_colour_red_black(gpu, oracle, name, make):
    """Red-black colouring of connected bipartite graphs (breadth-first depth
    parity) and the Jones-Plassmann fallback otherwise: bit-exact with the
    oracle."""
    n, rp, ci, w = make()
    print(f"colour_red_black {name} n={n}", flush=True)
    col, nc = gpu.stages.colour(rp, ci, 0xC010, 1)
    rcol, rnc = oracle.colour(n, rp, ci, 0xC010, 1)
    assert nc == rnc
    same(host(col), rcol)


def _cliques_plus_random(n, ncliques, size, deg, seed):
    """ncliques disjoint cliques of `size` vertices, plus random edges of mean
    degree `deg` over all n vertices and a ring (connected)."""
    a, b = [], []
    for q in range(ncliques):
        i, j = np.triu_indices(size, 1)
        a.append(q * size + i)
        b.append(q * size + j)
    m = n * deg // 2
    u = I.uniform(seed, 2 * m)
    a.append(np.minimum((u[0::2] * n).astype(np.int64), n - 1))
    b.append(np.minimum((u[1::2] * n).astype(np.int64), n - 1))
    a.append(np.arange(n))
    b.append((np.arange(n) + 1) % n)
    a, b = np.concatenate(a), np.concatenate(b)
    keep = a != b
    a2, b2 = I.canonical_edges(a[keep], b[keep])
    return I.csr_from_edges(n, a2, b2, np.ones(len(a2)))


@pytest.mark.parametrize("n,ncl,size,deg", [(20000, 1, 100, 2),    # data-driven rounds
                                            (3000, 1, 80, 2),      # rounds in one workgroup
                                            (4000, 10, 80, 50),    # near-dense: one vertex at a time, LDS
                                            (12000, 20, 80, 50),   # near-dense and larger: data-driven rounds
                                            (12000, 20, 80, 34),   # denser: data-driven rounds
                                            (140000, 20, 80, 34),  # denser and large: data-driven rounds
                                            (6000, 1, 480, 2)])    # a clique of 480: long rows, long chains
def test_colour_many_colours(gpu, oracle, n, ncl, size, deg):
    """More than 64 colours (every vertex of a clique of 80-100 takes its own):
    the first-fit search beyond the first 64 colours, on every colouring path,
    equals the oracle."""
    n_, rp, ci, w = _cliques_plus_random(n, ncl, size, deg, 90 + n)
    col, nc = gpu.stages.colour(rp, ci, 0xC010, 2)
    rcol, rnc = oracle.colour(n, rp, ci, 0xC010, 2)
    assert nc == rnc > 64
    same(host(col), rcol)


@pytest.mark.parametrize("shape,dmax", [((24, 24, 16), 6144), ((32, 32, 32), 12288)])
def test_dense_w_cycle_nested(gpu, oracle, shape, dmax):
    """A dense operator several levels above the coarsest (built level by
    level, each level's coarse correction a GEMM with the operator below; its
    first level launched step by step above the tail): still the W-cycle up to
    rounding (FP64 1e-12, FP32 1e-5 relative)."""
    g = I.grid3d(*shape, weight_seed=11)
    n = g[0]
    b = I.zero_mean_normal_rhs(3, n)
    s = solver_for(gpu, g, w_dense=1, dense_max_n=dmax)
    H = oracle.Hierarchy(g, None)
    sizes = [s.level_info(l)["n"] for l in range(s.num_levels())]
    assert any(2048 < m <= dmax for m in sizes[1:]) and any(m <= 2048 for m in sizes)
    w_ref = H.cycle(b, None, 2)
    w64 = host(s.cycle(b, None, 2))
    close_elementwise(w64, w_ref, 1e-12)
    b32 = b.astype(np.float32)
    w32_ref = H.cycle32(b32, None, 2)
    w32 = host(s.cycle32(b32, None, 2))
    close_elementwise(w32, w32_ref, 1e-5)


@pytest.mark.parametrize("n0", [60000, 150000])
def test_block_sweep_bit_identical(gpu, n0):
    """Levels with many colours of a few rows each (near-dense coarse levels of
    power-law graphs) run each sweep in one single-workgroup launch: the same
    arithmetic as one launch per colour, so every cycle and the whole solve are
    bit-identical with the block sweep switched off."""
    g = I.config3(n0=n0)[0]
    kw = dict(a2_hub_cap=64)
    n = g[0]
    b = I.zero_mean_normal_rhs(3, n)
    on = solver_for(gpu, g, b, block_sweep_min_colours=64, **kw)
    off = solver_for(gpu, g, b, block_sweep_min_colours=0, **kw)
    sizes = [(on.level_info(l)["n"], on.level_info(l)["ncolours"]) for l in range(on.num_levels())]
    print(f"power-law n0={n0}: levels (n, colours) {sizes}", flush=True)
    assert any(c >= 64 and m <= 64 * c and m > 2048 for m, c in sizes[1:-1]), sizes
    x0 = I.normal(4, n)
    b32 = b.astype(np.float32)
    for gamma in (1, 2):
        same(host(on.cycle(b, x0, gamma)), host(off.cycle(b, x0, gamma)))
        same(host(on.cycle32(b32, None, gamma)), host(off.cycle32(b32, None, gamma)))
    for outer, prec in (("fcg", "f64"), ("fcg", "f32")):
        xa, sa = solver_for(gpu, g, b, block_sweep_min_colours=64, outer=outer, cycle_prec=prec, theta=0.5,
                            **kw).solve()
        xb, sb = solver_for(gpu, g, b, block_sweep_min_colours=0, outer=outer, cycle_prec=prec, theta=0.5,
                            **kw).solve()
        assert sa["iterations"] == sb["iterations"] and sa["rebuilds"] == sb["rebuilds"]
        same(host(xa), host(xb))
