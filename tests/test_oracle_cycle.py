"""Pins of the oracle's solve phase: coarsest solve, two-level exactness,
cycle symmetry, the error approximation of Alg. 2 and the adaptive loop of
Alg. 5 against dense linear algebra.  CPU only.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1806_07028_amd import inputs as I


def dense_laplacian(g):
    n, rp, ci, w = g
    W = sp.csr_matrix((w, ci, rp), shape=(n, n)).toarray()
    return np.diag(W.sum(1)) - W


def level_dense(H, l):
    rp, ci, av, d = H.level_matrix(l)
    n = len(d)
    return sp.csr_matrix((av, ci, rp), shape=(n, n)).toarray() + np.diag(d)


def prolongation(H, l):
    agg = H.get_int(l, "agg")
    pv = H.get_dbl(l, "pval")
    n = len(agg)
    return sp.csr_matrix((pv, agg, np.arange(n + 1)), shape=(n, H.info(l)["nc"])).toarray()


def test_grounded_coarsest_is_pseudo_inverse(oracle):
    """Laplacian coarsest level (boolean P): grounded LDL^T + mean removal gives
    L^+ b; checked with the closed-form eigenbasis of the path Laplacian."""
    n = 40
    g = I.path(n)
    H = oracle.Hierarchy(g, np.arange(n, dtype=float), p1_mode=1, coarse_max=64)
    assert H.nlevels == 1 and H.info(0)["grounded"] == 1
    j = np.arange(n)
    b = I.zero_mean_normal_rhs(3, n)
    x_ref = np.zeros(n)
    for k in range(1, n):
        v = np.cos(k * np.pi * (j + 0.5) / n)
        v /= np.linalg.norm(v)
        x_ref += (v @ b) / (2 - 2 * np.cos(k * np.pi / n)) * v
    x = H.coarsest_solve(b)
    assert np.abs(x - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
    # V-cycle of a one-level hierarchy is the direct solve
    assert np.array_equal(H.vcycle(b), x)


def test_full_coarsest_is_dense_solve(oracle):
    g = I.grid2d(9, 7, weight_seed=2)
    H = oracle.Hierarchy(g, None, coarse_max=40)
    L = H.nlevels - 1
    assert H.info(L)["grounded"] == 0
    A = level_dense(H, L)
    b = I.normal(4, len(A))
    x = H.coarsest_solve(b)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_two_level_exactness(oracle):
    """e is in Range(P_1) (Sec. 3.3): with an exact (full) coarse solve the
    coarse-grid correction removes it; a grounded solve of the same operator
    does not (why the smooth-P_1 coarsest level is not grounded)."""
    g = I.grid2d(6, 5, weight_seed=7)
    n = g[0]
    H = oracle.Hierarchy(g, None, coarse_max=16)
    assert H.nlevels == 2
    A = dense_laplacian(g)
    P = prolongation(H, 0)
    e = P @ np.ones(P.shape[1])
    xc = H.coarsest_solve(P.T @ (A @ e))
    assert np.abs(xc - 1.0).max() <= 1e-10
    corr = e - P @ xc
    assert np.linalg.norm(corr) <= 1e-10 * np.linalg.norm(e)
    Hg = oracle.Hierarchy(g, None, coarse_max=16, coarse_solve=1)
    xg = Hg.coarsest_solve(P.T @ (A @ e))
    assert np.linalg.norm(e - P @ xg) > 1e-3 * np.linalg.norm(e)


def two_level_matrix(H, g):
    """E = S_bwd (I - P A_c^-1 P^T A) S_fwd as a dense matrix (b = 0)."""
    n = g[0]
    A = dense_laplacian(g)
    P = prolongation(H, 0)
    Ac = P.T @ A @ P
    col = H.get_int(0, "colour")
    lower = col[None, :] < col[:, None]
    upper = col[None, :] > col[:, None]
    D = np.diag(np.diag(A))
    Sf = np.eye(n) - np.linalg.solve(D + np.where(lower, A, 0), A)
    Sb = np.eye(n) - np.linalg.solve(D + np.where(upper, A, 0), A)
    CG = np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)
    return Sb @ CG @ Sf


def test_two_level_cycle_matches_dense(oracle):
    g = I.grid2d(5, 4, weight_seed=1)
    n = g[0]
    H = oracle.Hierarchy(g, None, coarse_max=12)
    assert H.nlevels == 2
    E = two_level_matrix(H, g)
    zero = np.zeros(n)
    for s in range(3):
        x = I.normal(10 + s, n)
        got = H.vcycle(zero, x)
        ref = E @ x
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(x)
    # the spectral radius bounds the measured per-cycle reduction
    A = dense_laplacian(g)
    ev = np.linalg.eigvals(E)
    rho = np.max(np.abs(ev[np.abs(ev) < 1 - 1e-12])) if np.any(np.abs(ev) < 1 - 1e-12) else 0.0
    x = I.normal(99, n)
    x -= x.mean()
    for _ in range(30):
        x = H.vcycle(zero, x)
        x -= x.mean()
    y = H.vcycle(zero, x)
    y -= y.mean()
    ratio = np.sqrt(y @ A @ y) / np.sqrt(x @ A @ x)
    assert ratio <= rho * 1.05 + 1e-12


@pytest.mark.parametrize("gamma", [1, 2])
def test_cycles_are_symmetric(oracle, gamma):
    g = I.grid2d(24, 19, weight_seed=3)
    n = g[0]
    H = oracle.Hierarchy(g, None, coarse_max=10)
    assert H.nlevels >= 3
    x = I.normal(1, n)
    y = I.normal(2, n)
    Bx = H.cycle(x, None, gamma)
    By = H.cycle(y, None, gamma)
    assert abs(Bx @ y - x @ By) <= 1e-12 * abs(Bx @ y)
    # the W-cycle is a better approximate inverse than the V-cycle here
    A = dense_laplacian(g)
    b = I.zero_mean_normal_rhs(3, n)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    ev = np.linalg.norm(H.cycle(b, None, 1) - xs)
    ew = np.linalg.norm(H.cycle(b, None, 2) - xs)
    assert ew < ev


def test_fp32_cycle_close(oracle):
    g = I.grid2d(32, 32, weight_seed=3)
    n = g[0]
    H = oracle.Hierarchy(g, None)
    b = I.zero_mean_normal_rhs(5, n)
    x64 = H.vcycle(b)
    x32 = H.vcycle32(b.astype(np.float32))
    assert np.linalg.norm(x32 - x64) <= 1e-5 * np.linalg.norm(x64)
    # the FP32 W-cycle is the FP64 W-cycle up to single-precision rounding
    w64 = H.cycle(b, None, 2)
    w32 = H.cycle32(b.astype(np.float32), None, 2)
    assert np.linalg.norm(w32 - w64) <= 1e-5 * np.linalg.norm(w64)
    assert np.array_equal(H.cycle32(b.astype(np.float32), None, 1), x32)


def test_approximate_error_fp32_cycles(oracle):
    """Alg. 2 with FP32 preconditioning cycles: one PCG step with the FP32
    W-cycle is the step-length-scaled widened W-cycle; with more steps the
    result agrees with the FP64-cycle one to single-precision accuracy."""
    g = I.grid2d(20, 20, weight_seed=4)
    n = g[0]
    A = dense_laplacian(g)
    r = I.zero_mean_normal_rhs(8, n)
    H1 = oracle.Hierarchy(g, None)
    w1 = H1.cycle32(r.astype(np.float32), None, 2).astype(np.float64)
    w1 -= w1.mean()
    alpha = (r @ w1) / (w1 @ A @ w1)
    e_one = oracle.approximate_error([H1], r, iterW=1, cycle_prec=1)
    assert np.allclose(e_one, alpha * w1 - (alpha * w1).mean(), rtol=0, atol=1e-12 * np.abs(e_one).max())
    H2 = oracle.Hierarchy(g, None, seed=77)
    H3 = oracle.Hierarchy(g, None, seed=78)
    es = np.linalg.lstsq(A, r, rcond=None)[0]
    errA = lambda e: np.sqrt((e - es) @ A @ (e - es)) / np.sqrt(es @ A @ es)
    for hs in ([H1], [H1, H2, H3]):
        e64 = oracle.approximate_error(hs, r)
        e32 = oracle.approximate_error(hs, r, cycle_prec=1)
        # a perturbed preconditioner: PCG amplifies the rounding over its
        # steps, but the approximation quality is the same
        assert 0 < np.linalg.norm(e32 - e64) <= 1e-3 * np.linalg.norm(e64)
        assert errA(e32) <= 1.01 * errA(e64) + 1e-6


def test_approximate_error_alg2(oracle):
    """Alg. 2: with the W-cycle (Re <= numW) and the composite preconditioner
    (Re > numW) the PCG iterates approach A e = r; the composite product is
    symmetric, so PCG with it is CG in another inner product."""
    g = I.grid2d(20, 20, weight_seed=4)
    n = g[0]
    A = dense_laplacian(g)
    r = I.zero_mean_normal_rhs(8, n)
    es = np.linalg.lstsq(A, r, rcond=None)[0]
    H1 = oracle.Hierarchy(g, None)
    H2 = oracle.Hierarchy(g, None, seed=77)
    H3 = oracle.Hierarchy(g, None, seed=78)
    errA = lambda e: np.sqrt((e - es) @ A @ (e - es)) / np.sqrt(es @ A @ es)
    e1 = oracle.approximate_error([H1], r)
    e_short = oracle.approximate_error([H1], r, iterW=2)
    assert errA(e1) < errA(e_short) < 1.0
    assert abs(e1.mean()) < 1e-14 * np.abs(e1).max()
    e3 = oracle.approximate_error([H1, H2, H3], r)  # Re = 3 > numW: composite, iterV steps
    e3_one = oracle.approximate_error([H1, H2, H3], r, iterV=1)
    assert errA(e3) < errA(e3_one) < 1.0
    # composite order B_1, B_2, B_3, B_3, B_2, B_1, each applied to the current iterate
    z = np.zeros(n)
    for H in (H1, H2, H3, H3, H2, H1):
        z = H.cycle(r, z, 1)
    z -= z.mean()
    alpha = (r @ z) / (z @ A @ z)
    ref = alpha * z - (alpha * z).mean()
    assert np.allclose(e3_one, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # the composite product is symmetric
    y = I.zero_mean_normal_rhs(9, n)
    zy = np.zeros(n)
    for H in (H1, H2, H3, H3, H2, H1):
        zy = H.cycle(y, zy, 1)
    assert abs(z @ y - (zy - zy.mean()) @ r) <= 1e-11 * abs(z @ y)
    # Re = 1 with iterW = 1 is one W-cycle, scaled by the PCG step length
    w1 = H1.cycle(r, None, 2)
    w1 -= w1.mean()
    e_one = oracle.approximate_error([H1], r, iterW=1)
    alpha = (r @ w1) / (w1 @ A @ w1)
    assert np.allclose(e_one, alpha * w1 - (alpha * w1).mean(), rtol=0, atol=1e-12 * np.abs(e_one).max())


@pytest.mark.parametrize("kw", [dict(), dict(p1_mode=1), dict(outer=1, cycle_prec=1, theta=0.5),
                                dict(outer=1, cycle_prec=0, theta=0.5)])
def test_solve_reaches_pseudo_inverse(oracle, kw):
    g = I.grid2d(24, 24, weight_seed=6)
    n = g[0]
    b = I.zero_mean_normal_rhs(2, n)
    res = oracle.solve(g, b, **kw)
    st = res.stats
    assert st["status"] == 0
    assert st["true_relres"] <= 1.01e-8
    A = dense_laplacian(g)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    xs -= xs.mean()
    x = res.x - res.x.mean()
    errA = np.sqrt((x - xs) @ A @ (x - xs)) / np.sqrt(xs @ A @ xs)
    assert errA <= 1e-6
    assert len(res.relres_hist) == st["iterations"] + 1
    assert st["iterations"] < 60


def test_solve_rebuild_thresholds(oracle):
    g, b = I.config1()
    # threshold 1e-6 re-sets up after every iteration (Alg. 5(1))
    r1 = oracle.solve(g, b, theta=1e-6)
    assert r1.stats["rebuilds"] == r1.stats["iterations"] - 1
    # an infinite threshold never re-sets up: the plain UA-AMG V-cycle
    rinf = oracle.solve(g, b, theta=np.inf, max_iter=40)
    assert rinf.stats["rebuilds"] == 0
    r2 = oracle.solve(g, b)
    assert r2.stats["iterations"] < rinf.stats["iterations"] or rinf.stats["status"] == -10
    # paper's low-frequency right-hand side
    rl = oracle.solve(g, I.low_frequency_rhs(g[0]))
    assert rl.stats["status"] == 0 and rl.stats["true_relres"] <= 1.01e-8
    # b = 0 returns immediately
    r0 = oracle.solve(g, np.zeros(g[0]))
    assert r0.stats["iterations"] == 0 and np.all(r0.x == 0)


def test_solve_relaxation_rebuild_source(oracle):
    """The homogeneous relaxation variant (fresh start vector, V-cycles and
    sweeps on A e = 0, no correction) still converges with boolean P."""
    g, b = I.config1()
    r = oracle.solve(g, b, rebuild_source=1, p1_mode=1, max_iter=600)
    assert r.stats["status"] == 0
