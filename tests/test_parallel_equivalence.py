"""The GPU builds the sequential greedy decisions of Alg. 1 (path cover) and of
Alg. 3 Steps 9-19 (isolated vertices) with deterministic reservations, and the
path orientation with pointer jumping.  These CPU simulations of exactly those
parallel schedules must reproduce the sequential oracle on random inputs,
whatever the window size.  No HIP code is involved.
"""
import numpy as np
import pytest

from paper_1806_07028_amd import inputs as I

INF = 1 << 62


def reservation_path_cover(n, su, sv, window):
    """Rounds over a window of the pending edges (rank order).  An edge that is
    not rejected reserves {u, v, far end of u, far end of v} with its rank and
    commits iff it holds all four."""
    m = len(su)
    deg = np.zeros(n, int)
    other = np.arange(n)
    nb = -np.ones((n, 2), int)
    pending = list(range(m))
    rounds = 0
    while pending:
        rounds += 1
        win = pending[:window]
        res = {}
        ends = {}
        done = set()
        for t in win:
            u, v = su[t], sv[t]
            if deg[u] >= 2 or deg[v] >= 2 or other[u] == v:
                done.add(t)
                continue
            a, b = other[u], other[v]
            ends[t] = (a, b)
            for s in (u, v, a, b):
                res[s] = min(res.get(s, INF), t)
        for t, (a, b) in ends.items():
            u, v = su[t], sv[t]
            if all(res[s] == t for s in (u, v, a, b)):
                nb[u, deg[u]] = v
                nb[v, deg[v]] = u
                deg[u] += 1
                deg[v] += 1
                other[a] = b
                other[b] = a
                done.add(t)
        pending = [t for t in pending if t not in done]
    return nb, rounds


def edge_set(nb):
    s = set()
    for v, row in enumerate(np.asarray(nb).reshape(-1, 2)):
        for u in row:
            if u >= 0:
                s.add((min(u, v), max(u, v)))
    return s


@pytest.mark.parametrize("seed", range(40))
def test_reservation_path_cover_equals_greedy(oracle, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 40))
    m = int(rng.integers(n, 4 * n))
    a = rng.integers(0, n, m)
    b = rng.integers(0, n, m)
    a, b = I.canonical_edges(a, b)
    order = rng.permutation(len(a))
    su, sv = a[order].astype(np.int32), b[order].astype(np.int32)
    ref = oracle.path_cover(n, su, sv)
    for window in (1, 3, 17, 10 ** 6):
        got, _ = reservation_path_cover(n, su, sv, window)
        assert edge_set(got) == edge_set(ref)


def test_reservation_path_cover_grid(oracle):
    g = I.grid2d(30, 30, weight_seed=3)
    n, rp, ci, w = g
    e = oracle.smooth_error(g, 1, 5, 3)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci)
    su, sv = oracle.sorted_edges(n, rp2, ci2, e)
    ref = oracle.path_cover(n, su, sv)
    got, rounds = reservation_path_cover(n, su, sv, 4096)
    assert edge_set(got) == edge_set(ref)
    assert rounds < len(su) // 4


def pointer_jump_orient(nb):
    """Half-edge list ranking: for vertex v and direction d the end reached and
    the distance; path start = smaller end; pos = distance to the start."""
    nb = np.asarray(nb).reshape(-1, 2)
    n = len(nb)
    # half-edge h = 2v + d follows nb[v][d]
    nxt = -np.ones(2 * n, int)
    end = -np.ones(2 * n, int)
    dist = np.zeros(2 * n, int)
    for v in range(n):
        for d in range(2):
            w = nb[v, d]
            if w < 0:
                continue
            # continue from w away from v
            dd = 0 if nb[w, 1] == v else 1
            if nb[w, dd] < 0 or nb[w, dd] == v:
                end[2 * v + d] = w
                dist[2 * v + d] = 1
            else:
                nxt[2 * v + d] = 2 * w + dd
                dist[2 * v + d] = 1
    while (nxt >= 0).any():
        nxt2, dist2, end2 = nxt.copy(), dist.copy(), end.copy()
        for h in range(2 * n):
            if nxt[h] >= 0:
                j = nxt[h]
                dist2[h] = dist[h] + dist[j]
                nxt2[h] = nxt[j]
                end2[h] = end[j]
        nxt, dist, end = nxt2, dist2, end2
    pid = -np.ones(n, int)
    pos = -np.ones(n, int)
    for v in range(n):
        ends = [(v, 0)] if (nb[v] < 0).any() else []
        for d in range(2):
            if nb[v, d] >= 0:
                ends.append((end[2 * v + d], dist[2 * v + d]))
        if nb[v, 0] < 0 and nb[v, 1] < 0:
            continue
        s, p = min(ends)
        pid[v] = s
        pos[v] = p
    return pid, pos


@pytest.mark.parametrize("seed", range(6))
def test_pointer_jumping_orientation(oracle, seed):
    g = I.rgg(500, seed + 1)
    n, rp, ci, w = g
    e = oracle.smooth_error(g, 1, seed, 3)
    rp2, ci2 = oracle.a2_pattern(n, rp, ci)
    su, sv = oracle.sorted_edges(n, rp2, ci2, e)
    nb = oracle.path_cover(n, su, sv)
    pid, pos, plen, _ = oracle.orient(nb)
    gp, gpos = pointer_jump_orient(nb)
    assert np.array_equal(gp, pid) and np.array_equal(gpos, pos)


def reservation_repair(n, grp, gci, gw, gkey, obj, members, window):
    """Alg. 3 Steps 9-19 by reservations with priority = vertex id.  An iterate
    u reserves its own slot, its best neighbour v and v's aggregate object."""
    best = -np.ones(n, int)
    for u in range(n):
        lo, hi = grp[u], grp[u + 1]
        if hi == lo:
            continue
        if gkey is not None:
            k = min(range(lo, hi), key=lambda t: (gkey[t], gci[t]))
        else:
            k = min(range(lo, hi), key=lambda t: (-gw[t], gci[t]))
        best[u] = gci[k]
    adj = lambda a, b: b in set(gci[grp[a]:grp[a + 1]].tolist())
    obj = list(obj)
    members = {k: list(v) for k, v in members.items()}
    centre = {}
    pending = [u for u in range(n) if obj[u] < 0]
    while pending:
        pending = [u for u in pending if obj[u] < 0]
        if not pending:
            break
        win = pending[:window]
        rv, ro = {}, {}
        plan = {}
        for u in win:
            v = best[u]
            slots_v = [u] + ([v] if v >= 0 else [])
            slots_o = [obj[v]] if v >= 0 and obj[v] >= 0 else []
            plan[u] = (slots_v, slots_o)
            for s in slots_v:
                rv[s] = min(rv.get(s, INF), u)
            for s in slots_o:
                ro[s] = min(ro.get(s, INF), u)
        for u in win:
            sv_, so_ = plan[u]
            if not (all(rv[s] == u for s in sv_) and all(ro[s] == u for s in so_)):
                continue
            v = best[u]
            if v < 0:
                members[u] = [u]
                obj[u] = u
            elif obj[v] < 0:
                members[u] = [u, v]
                obj[u] = obj[v] = u
            else:
                T = obj[v]
                if len(members[T]) <= 2:
                    members[T].append(u)
                    obj[u] = T
                else:
                    rest = [x for x in members[T] if x != v]
                    take_out = adj(rest[0], rest[1]) if len(rest) == 2 else v != centre[T]
                    if take_out:
                        members[T] = rest
                        members[u] = [u, v]
                        obj[u] = obj[v] = u
                    else:  # v is the middle or the centre: u joins at v
                        members[T].append(u)
                        obj[u] = T
                        centre[T] = v
    # canonical ids by smallest member
    live = sorted((min(m), k) for k, m in members.items() if m)
    canon = {k: i for i, (_, k) in enumerate(live)}
    return np.array([canon[obj[v]] for v in range(n)])


@pytest.mark.parametrize("seed", range(10))
def test_reservation_repair_equals_sequential(oracle, seed):
    # random geometric graphs, and power-law graphs whose hubs grow stars
    g = I.rgg(700, 50 + seed) if seed < 8 else I.config3(seed=seed, n0=3000)[0]
    n, rp, ci, w = g
    e = oracle.smooth_error(g, 1, seed, 3)
    H = oracle.Hierarchy(g, e, coarse_max=8)
    if seed >= 8:
        assert sum(H.info(l)["middle"] for l in range(H.nlevels - 1)) > 0
    for level in range(min(3, H.nlevels - 1)):
        grp, gci, gw = H.get_int(level, "G_rp"), H.get_int(level, "G_ci"), H.get_dbl(level, "G_v")
        gkey = H.get_dbl(level, "gkey") if level == 0 else None
        nb = H.get_int(level, "nb").reshape(-1, 2)
        ref, nc, _ = oracle.aggregate(len(nb), grp, gci, gw, nb, gkey)
        pid, pos, plen, _ = oracle.orient(nb)
        obj = -np.ones(len(nb), int)
        members = {}
        for v in range(len(nb)):
            if pid[v] >= 0 and pos[v] % 2 == 0 and pos[v] + 1 < plen[v]:
                w_ = [u for u in nb[v] if u >= 0 and pos[u] == pos[v] + 1][0]
                obj[v] = obj[w_] = v
                members[v] = [v, w_]
        for window in (1, 5, 10 ** 6):
            got = reservation_repair(len(nb), grp, gci, gw, gkey, obj, members, window)
            assert np.array_equal(got, ref)


def wake_rounds(n, rp, ci, key, rng, stale):
    """Data-driven Jones-Plassmann rounds as the library runs them: the first
    round tries every vertex; a vertex that takes its colour wakes its
    uncoloured neighbours for the next round, each at most once per round (a
    stamp per vertex); a blocked vertex keeps a cursor into its
    higher-priority list and resumes there.  Within a round the vertices run
    in a random order, and with probability `stale` a read of a colour
    written earlier in the same round still sees the vertex uncoloured (the
    write not yet visible to that thread)."""
    higher = lambda u, v: (key[u], u) > (key[v], v)
    hl = [[u for u in ci[rp[v]:rp[v + 1]] if higher(u, v)] for v in range(n)]
    colour = -np.ones(n, int)
    cur = [0] * n
    stamp = [0] * n
    work = list(range(n))
    rounds = 0
    while work:
        rounds += 1
        assert rounds <= n
        assert len(set(work)) == len(work)  # at most once per round
        done_now = set()
        seen = lambda u: colour[u] >= 0 and not (u in done_now and rng.random() < stale)
        nxt = []
        for v in rng.permutation(work):
            if colour[v] >= 0:
                continue
            while cur[v] < len(hl[v]) and seen(hl[v][cur[v]]):
                cur[v] += 1
            if cur[v] < len(hl[v]):
                continue  # blocked on an uncoloured higher neighbour
            used = {colour[u] for u in hl[v]}
            colour[v] = next(c for c in range(n + 1) if c not in used)
            done_now.add(v)
            for w in ci[rp[v]:rp[v + 1]]:
                if not seen(w) and stamp[w] < rounds + 1:
                    stamp[w] = rounds + 1
                    nxt.append(w)
        work = nxt
    return colour, rounds


@pytest.mark.parametrize("case", ["powerlaw", "clique", "grid"])
def test_wake_rounds_equal_greedy(oracle, case):
    """The colouring schedule of the library (data-driven rounds over the
    vertices woken by the previous round's colours, resumable cursors) gives
    the greedy first-fit in priority order, whatever the order and the
    visibility of writes within a round: checked against the oracle."""
    if case == "powerlaw":
        n, rp, ci, w = I.config3(n0=1500)[0]
    elif case == "clique":  # a clique of 60 that every other vertex waits on, plus a ring
        n = 400
        a, b = np.triu_indices(60, 1)
        a = np.concatenate([a, np.arange(n), np.arange(60, n)])
        b = np.concatenate([b, (np.arange(n) + 1) % n, np.arange(60, n) % 60])
        keep = a != b
        a2, b2 = I.canonical_edges(a[keep], b[keep])
        n, rp, ci, w = I.csr_from_edges(n, a2, b2, np.ones(len(a2)))
    else:
        n, rp, ci, w = I.grid2d(20, 20)
    deg = np.diff(rp)
    key = [oracle.colour_key(0xC010, 1, v, int(deg[v])) for v in range(n)]
    ref, _ = oracle.colour_greedy(n, rp, ci, 0xC010, 1)
    for seed, stale in ((0, 0.0), (1, 0.5), (2, 1.0)):
        got, rounds = wake_rounds(n, rp, ci, key, np.random.default_rng(seed), stale)
        assert np.array_equal(got, ref), (seed, stale)
        assert rounds > 1


def greedy_stamps(n, rp, ci, key):
    """The one-vertex-at-a-time colouring of near-dense levels as the library
    runs it: vertices in descending (key, id) order; step t stamps t at the
    colour of every coloured neighbour, and the vertex takes the lowest colour
    without the stamp (at most the largest colour so far plus one).  The
    colour written at step t - 1 is not yet visible at step t (a write after
    the last barrier of that step): it comes from the step's own record of
    the previous vertex and its colour."""
    order = sorted(range(n), key=lambda v: (key[v], v), reverse=True)
    visible = [-1] * n  # colours written up to step t - 2
    seen = [-1] * (n + 1)
    cmax, vprev, cprev, pending = -1, -1, -1, None
    for t, v in enumerate(order):
        for u in ci[rp[v]:rp[v + 1]]:
            c = cprev if u == vprev else visible[u]
            if c >= 0:
                seen[c] = t
        mex = next((c for c in range(cmax + 1) if seen[c] != t), cmax + 1)
        if pending is not None:  # the write of step t - 1 lands now
            visible[pending[0]] = pending[1]
        pending = (v, mex)
        vprev, cprev, cmax = v, mex, max(cmax, mex)
    visible[pending[0]] = pending[1]
    return np.array(visible)


@pytest.mark.parametrize("case", ["powerlaw", "clique", "dense"])
def test_greedy_stamps_equal_greedy(oracle, case):
    """Stamped first-fit with the previous vertex's colour from a register
    gives the oracle's greedy colouring."""
    if case == "powerlaw":
        n, rp, ci, w = I.config3(n0=1500)[0]
    elif case == "clique":  # a clique of 60 that every other vertex waits on, plus a ring
        n = 400
        a, b = np.triu_indices(60, 1)
        a = np.concatenate([a, np.arange(n), np.arange(60, n)])
        b = np.concatenate([b, (np.arange(n) + 1) % n, np.arange(60, n) % 60])
        keep = a != b
        a2, b2 = I.canonical_edges(a[keep], b[keep])
        n, rp, ci, w = I.csr_from_edges(n, a2, b2, np.ones(len(a2)))
    else:  # a random graph of mean degree about 60
        rng = np.random.default_rng(5)
        n = 300
        a = rng.integers(0, n, 9000)
        b = rng.integers(0, n, 9000)
        keep = a != b
        a2, b2 = I.canonical_edges(a[keep], b[keep])
        n, rp, ci, w = I.csr_from_edges(n, a2, b2, np.ones(len(a2)))
    deg = np.diff(rp)
    key = [oracle.colour_key(0xC010, 1, v, int(deg[v])) for v in range(n)]
    ref, _ = oracle.colour_greedy(n, rp, ci, 0xC010, 1)
    assert np.array_equal(greedy_stamps(n, rp, ci, key), ref)


def list_rounds(n, rp, ci, key, rng, stale):
    """Jones-Plassmann rounds over every pending vertex (the library's path
    for levels without hub rows), with a resumable cursor per vertex; in a
    random order, with reads of same-round colours missed at random."""
    higher = lambda u, v: (key[u], u) > (key[v], v)
    hl = [[u for u in ci[rp[v]:rp[v + 1]] if higher(u, v)] for v in range(n)]
    colour = -np.ones(n, int)
    cur = [0] * n
    pending = list(range(n))
    rounds = 0
    while pending:
        rounds += 1
        assert rounds <= n
        done_now = set()
        seen = lambda u: colour[u] >= 0 and not (u in done_now and rng.random() < stale)
        left = []
        for v in rng.permutation(pending):
            while cur[v] < len(hl[v]) and seen(hl[v][cur[v]]):
                cur[v] += 1
            if cur[v] < len(hl[v]):
                left.append(v)
                continue
            used = {colour[u] for u in hl[v]}
            colour[v] = next(c for c in range(n + 1) if c not in used)
            done_now.add(v)
        pending = left
    return colour


@pytest.mark.parametrize("case", ["grid", "rgg"])
def test_list_rounds_equal_greedy(oracle, case):
    """The list rounds of levels without hub rows give the greedy first-fit in
    priority order as well."""
    n, rp, ci, w = I.grid2d(20, 20) if case == "grid" else I.rgg(600, 3)
    deg = np.diff(rp)
    key = [oracle.colour_key(0xC010, 1, v, int(deg[v])) for v in range(n)]
    ref, _ = oracle.colour_greedy(n, rp, ci, 0xC010, 1)
    for seed, stale in ((0, 0.0), (1, 0.5)):
        assert np.array_equal(list_rounds(n, rp, ci, key, np.random.default_rng(seed), stale), ref)
