"""Seeded synthetic inputs: graphs, edge weights and right-hand sides.

This module only *generates data*.  It holds none of the solver's arithmetic
and imports neither the HIP library nor the CPU oracle, so both sides can be fed
byte-identical arrays from it.

Randomness comes from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used as a
counter-based generator: word k (k >= 1) of stream ``seed`` is
``mix64(seed + k * 0x9E3779B97F4A7C15)``.  Uniforms take the top 53 bits,
normals come from the Box-Muller transform.

Workload shapes follow the paper's test families (Section 4): 2D regular grids,
Watts-Strogatz ring graphs with rewiring probability 0 and mean degree 4, and
stand-ins for the real-world graphs of Tables 7-8 (random geometric graphs for
meshes/road networks, Chung-Lu and Barabasi-Albert graphs for power-law
networks).  Real graphs get the paper's preprocessing: largest connected
component, no self loops, positive weights, undirected.

All graphs are returned as symmetric CSR: ``(n, row_ptr int32[n+1],
col int32[nnz], w float64[nnz])`` with columns ascending within each row, no
diagonal, no duplicates and ``w[i->j] == w[j->i]`` bitwise.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_words(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Words start+1 .. start+count of the SplitMix64 stream seeded with ``seed``."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * np.uint64(GAMMA)
    return mix64(z)


def uniform(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of each stream word times 2^-53."""
    w = stream_words(seed, count, start)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive pairs of uniforms."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m)
    u1, u2 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    z = np.empty(2 * m)
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:count]


# ----------------------------------------------------------------------------
# CSR assembly
# ----------------------------------------------------------------------------

def canonical_edges(i: np.ndarray, j: np.ndarray):
    """Return unique undirected edges (a < b) sorted lexicographically."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    a = np.minimum(i, j)
    b = np.maximum(i, j)
    keep = a != b
    a, b = a[keep], b[keep]
    key = np.unique(a * (np.int64(1) << 32) + b)
    return (key >> 32).astype(np.int64), (key & 0xFFFFFFFF).astype(np.int64)


def csr_from_edges(n: int, a: np.ndarray, b: np.ndarray, w: np.ndarray):
    """Symmetric CSR from canonical undirected edges (a < b, unique) and weights."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    import scipy.sparse as sp

    if 2 * len(a) >= 2 ** 31:
        raise ValueError("graph too large for int32 row pointers")
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    vals = np.concatenate([w, w])
    # bucket by row, then sort each row by column (the edges are unique, so
    # nothing is summed)
    m = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    m.sort_indices()
    assert m.nnz == len(rows), "duplicate edges"
    return n, m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64)


def upper_edges(row_ptr, col):
    """Canonical undirected edge list (a < b) of a symmetric CSR, in lexicographic order."""
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    col = np.asarray(col, dtype=np.int64)
    m = rows < col
    return rows[m], col[m]


def largest_component(n, a, b):
    """Relabel the largest connected component (ties: the one holding the smallest vertex).

    Returns (n_lcc, a', b', keep_mask) with vertex order preserved.
    """
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    g = sp.coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n)).tocsr()
    ncomp, lab = connected_components(g, directed=False)
    sizes = np.bincount(lab, minlength=ncomp)
    best = int(np.argmax(sizes))  # argmax returns the first maximum
    keep = lab == best
    newid = -np.ones(n, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()))
    m = keep[a] & keep[b]
    a2, b2 = newid[a[m]], newid[b[m]]
    return int(keep.sum()), a2, b2, keep


# ----------------------------------------------------------------------------
# Graph families
# ----------------------------------------------------------------------------

def grid2d_edges(nx: int, ny: int):
    """5-point grid, vertex v = y*nx + x."""
    v = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    a = np.concatenate([v[:, :-1].ravel(), v[:-1, :].ravel()])
    b = np.concatenate([v[:, 1:].ravel(), v[1:, :].ravel()])
    a, b = canonical_edges(a, b)
    return nx * ny, a, b


def grid3d_edges(nx: int, ny: int, nz: int):
    """7-point grid, vertex v = (z*ny + y)*nx + x."""
    v = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    a = np.concatenate([v[:, :, :-1].ravel(), v[:, :-1, :].ravel(), v[:-1, :, :].ravel()])
    b = np.concatenate([v[:, :, 1:].ravel(), v[:, 1:, :].ravel(), v[1:, :, :].ravel()])
    a, b = canonical_edges(a, b)
    return nx * ny * nz, a, b


def ring_edges(n: int, k: int = 4):
    """Watts-Strogatz ring lattice with rewiring probability 0: i ~ i+1..i+k/2 (mod n)."""
    i = np.arange(n, dtype=np.int64)
    a = np.concatenate([i for _ in range(1, k // 2 + 1)])
    b = np.concatenate([(i + s) % n for s in range(1, k // 2 + 1)])
    return n, *canonical_edges(a, b)


def path_edges(n: int):
    i = np.arange(n - 1, dtype=np.int64)
    return n, i, i + 1


def rgg_edges(n: int, seed: int, mean_degree: float = 8.0, radius: float | None = None):
    """Random geometric graph in the unit square, largest component kept."""
    from scipy.spatial import cKDTree

    if radius is None:
        radius = float(np.sqrt(mean_degree / (np.pi * n)))
    u = uniform(seed, 2 * n)
    pts = np.stack([u[0::2], u[1::2]], axis=1)
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    a, b = canonical_edges(pairs[:, 0], pairs[:, 1])
    n2, a2, b2, _ = largest_component(n, a, b)
    return n2, *canonical_edges(a2, b2)


def ba_edges(n: int, seed: int, m: int = 4):
    """Barabasi-Albert graph: K_{m+1} seed, each new vertex links to m distinct
    existing vertices drawn proportionally to degree (repeated-endpoint list)."""
    u = uniform(seed, 8 * m * n + 64)
    ptr = 0
    m0 = m + 1
    src, dst = [], []
    ends = []
    for x in range(m0):
        for y in range(x + 1, m0):
            src.append(x)
            dst.append(y)
            ends += [x, y]
    ends_arr = np.empty(2 * m * n + m0 * m0, dtype=np.int64)
    ne = len(ends)
    ends_arr[:ne] = ends
    for v in range(m0, n):
        chosen = set()
        while len(chosen) < m:
            if ptr >= len(u):
                u = np.concatenate([u, uniform(seed + 1, 8 * m * n, start=ptr)])
            t = int(ends_arr[int(u[ptr] * ne)])
            ptr += 1
            chosen.add(t)
        for t in sorted(chosen):
            src.append(v)
            dst.append(t)
            ends_arr[ne] = v
            ends_arr[ne + 1] = t
            ne += 2
    return n, *canonical_edges(np.array(src), np.array(dst))


def uniform_at(seed: int, k: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from stream words k (any uint64 counters)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + np.asarray(k, dtype=np.uint64) * np.uint64(GAMMA)
    return (mix64(z) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def chung_lu_edges(n0: int, seed: int, gamma: float = 2.1, mean_degree: float = 16.0,
                   max_degree: float | None = None):
    """Chung-Lu graph with expected degrees w_i = c (i + i0)^(-1/(gamma-1)).

    Edges are independent with p_ij = min(1, w_i w_j / sum(w)); each source a
    walks its candidates b > a with the skipping method of Miller & Hagberg
    (2011): a geometric jump with the current probability p, then acceptance
    with q/p.  Draw t of source a is word (a << 24) + t + 1 of the stream, so
    all sources advance together, one step per numpy pass.  Largest component
    kept.
    """
    if max_degree is None:
        max_degree = float(np.sqrt(mean_degree * n0))
    ex = 1.0 / (gamma - 1.0)
    i = np.arange(n0, dtype=np.float64)
    # choose i0 so that w_0 / mean(w) = max_degree / mean_degree
    lo, hi = 1e-3, float(n0)
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        wv = (i + mid) ** (-ex)
        ratio = wv[0] / wv.mean()
        if ratio > max_degree / mean_degree:
            lo = mid
        else:
            hi = mid
    wv = (i + np.sqrt(lo * hi)) ** (-ex)
    wv *= mean_degree / wv.mean()
    S = wv.sum()
    a = np.arange(n0 - 1, dtype=np.int64)
    b = a + 1
    p = np.minimum(1.0, wv[a] * wv[b] / S)
    t = np.zeros(n0 - 1, dtype=np.int64)
    act = (b < n0) & (p > 0)
    a, b, p, t = a[act], b[act], p[act], t[act]
    src, dst = [], []
    while len(a):
        # geometric jump over the candidates rejected with probability p each
        jump = p < 1.0
        if jump.any():
            r = 1.0 - uniform_at(seed, (a[jump] << 24) + t[jump] + 1)  # in (0, 1]
            t[jump] += 1
            b[jump] += np.floor(np.log(r) / np.log1p(-p[jump])).astype(np.int64)
        live = b < n0
        a, b, p, t = a[live], b[live], p[live], t[live]
        if not len(a):
            break
        q = np.minimum(1.0, wv[a] * wv[b] / S)
        u = 1.0 - uniform_at(seed, (a << 24) + t + 1)
        t += 1
        acc = u < q / p
        src.append(a[acc])
        dst.append(b[acc])
        p = q
        b = b + 1
        live = (b < n0) & (p > 0)
        a, b, p, t = a[live], b[live], p[live], t[live]
    src = np.concatenate(src) if src else np.zeros(0, np.int64)
    dst = np.concatenate(dst) if dst else np.zeros(0, np.int64)
    a_, b_ = canonical_edges(src, dst)
    n2, a2, b2, _ = largest_component(n0, a_, b_)
    return n2, *canonical_edges(a2, b2)


# ----------------------------------------------------------------------------
# Weights and right-hand sides
# ----------------------------------------------------------------------------

def log_uniform_weights(seed: int, m: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """w = 10^(lo + (hi - lo) u), one per canonical undirected edge."""
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * uniform(seed, m))


def unit_interval_weights(seed: int, m: int) -> np.ndarray:
    """w uniform in (0, 1], taken as 1 - u."""
    return 1.0 - uniform(seed, m)


def zero_mean_normal_rhs(seed: int, n: int) -> np.ndarray:
    b = normal(seed, n)
    return b - b.mean()


def low_frequency_rhs(n: int) -> np.ndarray:
    """The paper's low-frequency right-hand side [1, ..., 1, 1 - n]."""
    b = np.ones(n)
    b[-1] = 1.0 - n
    return b


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def grid2d(nx: int, ny: int, weight_seed: int | None = None, lo: float = -3.0, hi: float = 3.0):
    n, a, b = grid2d_edges(nx, ny)
    w = np.ones(len(a)) if weight_seed is None else log_uniform_weights(weight_seed, len(a), lo, hi)
    return csr_from_edges(n, a, b, w)


def grid3d(nx: int, ny: int, nz: int, weight_seed: int | None = None, lo: float = -3.0, hi: float = 3.0):
    n, a, b = grid3d_edges(nx, ny, nz)
    w = np.ones(len(a)) if weight_seed is None else log_uniform_weights(weight_seed, len(a), lo, hi)
    return csr_from_edges(n, a, b, w)


def ring(n: int, k: int = 4):
    n, a, b = ring_edges(n, k)
    return csr_from_edges(n, a, b, np.ones(len(a)))


def path(n: int, weights=None):
    n, a, b = path_edges(n)
    w = np.ones(len(a)) if weights is None else np.asarray(weights, dtype=np.float64)
    return csr_from_edges(n, a, b, w)


def rgg(n: int, seed: int, mean_degree: float = 8.0, lo: float = -3.0, hi: float = 3.0, radius=None):
    n2, a, b = rgg_edges(n, seed, mean_degree, radius)
    return csr_from_edges(n2, a, b, log_uniform_weights(seed + 7919, len(a), lo, hi))


def config1(seed: int = 1):
    """64x64 5-point grid, unit weights, zero-mean N(0,1) rhs."""
    g = grid2d(64, 64)
    return g, zero_mean_normal_rhs(seed, g[0])


def config2(seed: int = 1, side: int = 128):
    """side^3 7-point grid, log-uniform weights on [1e-3, 1e3], zero-mean N(0,1) rhs."""
    g = grid3d(side, side, side, weight_seed=seed, lo=-3.0, hi=3.0)
    return g, zero_mean_normal_rhs(seed + 1000, g[0])


def config3(seed: int = 1, n0: int = 4_000_000):
    """Chung-Lu power-law graph: n0 vertices, degree exponent 2.1, mean degree
    16, largest component kept; weights uniform in (0, 1]; zero-mean N(0,1)
    rhs.  Solved with the A^2 hub cap (2-hop pairs only through pivots of
    degree <= 64)."""
    n, a, b = chung_lu_edges(n0, seed)
    g = csr_from_edges(n, a, b, unit_interval_weights(seed + 1, len(a)))
    return g, zero_mean_normal_rhs(seed + 2000, n)


def config4(seed: int = 1, count: int = 512, n_lo: float = 1e3, n_hi: float = 2e5):
    """Batch of `count` graphs of uneven size: n_g log-uniform on [n_lo, n_hi];
    type by an equal-probability draw among a 2D grid (nx = round(sqrt(n)),
    ny = round(n / nx)), a random geometric graph in the unit square with mean
    degree 8 (largest component) and a Barabasi-Albert graph (m = 4); edge
    weights 10^(-2 + 4u); zero-mean N(0,1) right-hand side per graph.
    Returns a list of (graph, rhs, kind)."""
    u = uniform(seed * 7 + 3, 2 * count)
    out = []
    for g in range(count):
        n = int(round(np.exp(np.log(n_lo) + u[2 * g] * np.log(n_hi / n_lo))))
        kind = ("grid", "rgg", "ba")[min(2, int(u[2 * g + 1] * 3))]
        s = seed * 1_000_003 + 17 * g
        if kind == "grid":
            nx = max(2, int(round(np.sqrt(n))))
            ny = max(2, int(round(n / nx)))
            nv, a, b = grid2d_edges(nx, ny)
        elif kind == "rgg":
            nv, a, b = rgg_edges(n, s)
        else:
            nv, a, b = ba_edges(n, s)
        gr = csr_from_edges(nv, a, b, log_uniform_weights(s + 1, len(a), -2.0, 2.0))
        out.append((gr, zero_mean_normal_rhs(s + 2, nv), kind))
    return out
