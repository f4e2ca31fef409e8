// PC-alphaAMG CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded FP64 implementation of the path-cover adaptive
// unsmoothed-aggregation AMG of Hu, Lin & Zikatanov, "An Adaptive Multigrid
// Method Based on Path Cover" (arXiv 1806.07028).  It exists to check the HIP
// library: only the test suite, the smoke check and the benchmark's CPU-baseline
// leg load it.  It shares no source with the HIP library.
//
// Build: g++ -O2 -ffp-contract=off -fPIC -shared (no fast-math).  Every fused
// multiply-add below is an explicit std::fma; nothing else is contracted.
//
// Where the paper is silent or ambiguous the following readings are used
// (each function names the passage it follows):
//  * Smooth error: every build relaxes its vector by S^nu, S = one symmetric
//    (forward then backward) multicoloured Gauss-Seidel sweep on A e = 0.  The
//    first build starts from xi_i = 2u_i - 1 (SplitMix64 counter stream) --
//    or, with init = MWM, is the UA-AMG hierarchy of Alg. 5/6 Step 2 (Sec.
//    2.1) built without any vector.  A re-setup of Alg. 5 starts from the
//    error approximation of Alg. 2 (default; x <- x + e afterwards), or from a
//    fresh xi exposed to m_V V-cycles of the current hierarchy on A e = 0
//    (rebuild_source 1), or -- Alg. 6, b = 0 -- from the current iterate
//    itself, normalised, with no further sweeps (rebuild_source 2).
//  * MWM aggregation (Sec. 2.1): edges heaviest first (ties by lexicographic
//    edge index) match two unaggregated ends; every vertex left over joins the
//    aggregate of its heaviest neighbour (ties to the smaller id), which is
//    always a matched vertex, so aggregates keep diameter <= 3.  Boolean
//    prolongation on every level.
//  * Reweighting (Alg. 4, Step 2): keys k_ij = |e_i - e_j| on the off-diagonal
//    pattern of A^2; heavier weight = smaller key; ties by lexicographic edge
//    index; numeric weight 1/max(k, 2^-52 max|e|).
//  * Path cover (Alg. 1): a free vertex counts as an endpoint; an edge joining
//    the two ends of one path is rejected (it would close a cycle).
//  * Matching along paths (Alg. 3, Steps 5-7): paths start at their smaller
//    endpoint id; positions (2t, 2t+1) are paired; an odd tail is left over.
//  * Isolated vertices (Alg. 3, Steps 9-19): ascending vertex id; best
//    neighbour by weight, ties to the smaller id; size-1 aggregates take Case 2;
//    Case 3 takes v out of its aggregate only if the rest stays connected: when
//    v is the middle of a 3-chain, or the centre of a star that grew that way,
//    u joins v's aggregate instead (no vertex is left isolated, Sec. 3.3, and
//    the aggregate keeps diameter <= 2, within the bound of three of the
//    matching-based aggregation of Sec. 2.1); a vertex with no neighbour is a
//    singleton.  This departs from Sec. 3.3's "all of size 2 or 3" (stars can
//    be larger); case3 = 1 keeps the printed Step 17 instead (v always leaves,
//    even when that splits a 3-chain).
//  * Prolongation (Sec. 3.3, Alg. 3 Steps 20-24): level 1 uses e normalised by a
//    power of two (max|e| in [0.5,1)) and centred by its mean measured in fixed
//    point at resolution 2^-32; an aggregate whose |e| stays below 2^-26 uses 1.
//    Levels > 1 are boolean.  Reweighted graph coarsened with the boolean matrix.
//  * Path shortening (Alg. 4, Step 7): contract, collapse repeats, keep only the
//    first occurrence of a coarse vertex (paths ordered by start id) and cut there.
//  * Coarsest level: n <= coarse_max, or stall (n_c > 0.9 n) on a level of at
//    most 4096 vertices (a larger stalled level keeps coarsening while
//    n_c < n), or max levels;
//    dense LDL^T, grounded (last vertex pinned, mean removed) iff the coarsest
//    operator is a Laplacian (every prolongation boolean, or a single level),
//    full otherwise; a non-positive pivot falls back to grounded.
//  * Gauss-Seidel ordering (the paper names only Gauss-Seidel): multicolour,
//    red-black (parity of the breadth-first distance from vertex 0) on a
//    connected bipartite level graph, else greedy first-fit in descending
//    (degree, SplitMix64 word) order, largest degree first.
//  * Outer loop (Alg. 5): V(1,1) with forward GS before and backward GS after
//    the coarse correction; x made orthogonal to 1 after each cycle; ConvR =
//    ||r_{k+1}||/||r_k||; rebuild when the mean ConvR since the last rebuild
//    exceeds theta; relative residual tolerance.  FCG(1) variant with an FP32
//    V-cycle preconditioner (not in the paper); the FP32 setting applies to
//    every cycle used as a preconditioner inside an FP64 PCG, i.e. to Alg. 2 too.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <numeric>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based stream:
// word k (k >= 1) of stream `seed` is mix64(seed + k * gamma).
// ---------------------------------------------------------------------------
const uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t stream_word(uint64_t seed, uint64_t k) { return mix64(seed + k * kGamma); }

// Random start vector of build r: xi_i = 2u - 1, u = top 53 bits * 2^-53.
double xi_value(uint64_t seed, int r, int i) {
  uint64_t w = stream_word(seed, ((uint64_t)(uint32_t)r << 32) + (uint64_t)(uint32_t)i + 1ull);
  double u = (double)(w >> 11) * 0x1.0p-53;
  return 2.0 * u - 1.0;
}

// Random word of vertex v on level l for the colouring order.
uint64_t colour_priority(uint64_t seed, int level, int v) {
  return stream_word(seed, ((uint64_t)(uint32_t)level << 32) + (uint64_t)(uint32_t)v + 1ull);
}

// Colouring order key: largest degree first (degree capped at 2^24 - 1 in the
// top 24 bits), then the top 40 bits of the random word.
uint64_t colour_key(uint64_t seed, int level, int v, int deg) {
  const uint64_t dg = (uint64_t)std::min(deg, (1 << 24) - 1);
  return (dg << 40) | (colour_priority(seed, level, v) >> 24);
}

// ---------------------------------------------------------------------------
// Data
// ---------------------------------------------------------------------------
struct Csr {
  int n = 0;
  std::vector<int> rp{0};
  std::vector<int> ci;
  std::vector<double> v;
  int nnz() const { return rp[n]; }
  int deg(int i) const { return rp[i + 1] - rp[i]; }
};

struct Params {
  double tol;
  double theta;
  int max_iter;
  int outer;           // 0 standalone V-cycle, 1 FCG
  int cycle_prec;      // 0 FP64, 1 FP32 (every preconditioning cycle: outer FCG and Alg. 2's PCG)
  int coarse_max;
  int relax_sweeps;
  int rebuild_vcycles; // V-cycles on A e = 0 before the sweeps (rebuild_source 1)
  int rebuild_source;  // 0 error approximation (Alg. 2), 1 relaxation of A e = 0
  int p1_mode;         // 0 smooth error values (paper), 1 boolean
  int coarse_solve;    // 0 auto, 1 grounded, 2 full
  int a2_hub_cap;      // 0 = exact A^2
  int max_rebuilds;
  int max_levels;
  int numW, iterW, iterV; // Alg. 2 parameters
  int rebuild_rule;       // 0 mean ConvR since the last re-setup (Alg. 5), 1 last ConvR (Alg. 6)
  uint64_t seed;
  uint64_t colour_seed;
  int case3;              // 0 connected reading of Alg. 3 Case 3, 1 as printed (v always leaves)
  int init;               // 0 first hierarchy from the relaxed start vector, 1 MWM (Alg. 5/6 Step 2)
};

struct Level {
  int n = 0;
  Csr A;                       // off-diagonal entries of A_l
  std::vector<double> d, dinv; // diagonal and its reciprocal
  std::vector<int> colour;
  int ncolours = 0;
  std::vector<std::vector<int>> by_colour;
  // setup data
  Csr G;                       // level graph: A^2 pattern with reweighted values (level 0), coarsened after
  std::vector<double> gkey;    // level 0: key |e_i - e_j| per G entry
  std::vector<int> nb;         // 2n cover neighbours, -1 = none
  std::vector<int> path_id, pos, plen;
  // transfer to level l+1 (empty on the coarsest)
  int nc = 0;
  std::vector<int> agg;
  std::vector<double> pval;
  std::vector<int> moff, mem;
  // statistics of the aggregation step
  int n_paths = 0, n_path_vertices = 0, n_unagg = 0;
  int case1 = 0, case2 = 0, case3 = 0, middle = 0, singleton = 0, p1_fallback = 0;
};

struct Coarsest {
  int n = 0, m = 0;
  bool grounded = false;
  bool fallback = false;
  std::vector<double> L;  // m x m, row-major, unit lower triangle below the diagonal
  std::vector<double> D;
};

struct Hierarchy {
  std::vector<Level> lv;
  Coarsest cs;
  int nnz_fine = 0;
  double op_complexity = 0.0;
  // FP32 copies for the mixed-precision cycle
  std::vector<std::vector<float>> a32, d32, dinv32, p32;
};

// ---------------------------------------------------------------------------
// Graph Laplacian A = D - W (Sec. 2.2): off-diagonals -w_ij, d_i = sum_j w_ij in
// CSR order, dinv_i = 1/d_i.
// ---------------------------------------------------------------------------
void laplacian(const Csr& W, Csr& A, std::vector<double>& d, std::vector<double>& dinv) {
  A = W;
  for (double& x : A.v) x = -x;
  d.assign(W.n, 0.0);
  dinv.assign(W.n, 0.0);
  for (int i = 0; i < W.n; ++i) {
    double s = 0.0;
    for (int k = W.rp[i]; k < W.rp[i + 1]; ++k) s = s + W.v[k];
    d[i] = s;
    dinv[i] = 1.0 / s;
  }
}

// ---------------------------------------------------------------------------
// Multicolouring for the Gauss-Seidel smoother (the paper only says
// "Gauss-Seidel").  Greedy first-fit in descending (key, id) order, key =
// largest degree first then a random word: each vertex takes the smallest
// colour unused by its already coloured neighbours.
// ---------------------------------------------------------------------------
int colour_greedy(const Csr& G, uint64_t seed, int level, std::vector<int>& colour) {
  const int n = G.n;
  std::vector<uint64_t> pr(n);
  for (int v = 0; v < n; ++v) pr[v] = colour_key(seed, level, v, G.deg(v));
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (pr[a] != pr[b]) return pr[a] > pr[b];
    return a > b;
  });
  colour.assign(n, -1);
  int ncol = 0;
  std::vector<char> used;
  for (int v : order) {
    used.assign(G.deg(v) + 1, 0);
    for (int k = G.rp[v]; k < G.rp[v + 1]; ++k) {
      int c = colour[G.ci[k]];
      if (c >= 0 && c <= G.deg(v)) used[c] = 1;
    }
    int c = 0;
    while (used[c]) ++c;
    colour[v] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// Connected bipartite level graphs (2D/3D grids, paths, trees) get the
// red-black ordering instead: colour = parity of the breadth-first distance
// from vertex 0.  A connected graph is bipartite exactly when no edge joins two
// vertices of equal parity; a proper two-colouring with vertex 0 coloured 0 is
// then unique.  Returns false (colouring untouched) for graphs that are not
// connected or not bipartite.
bool colour_bipartite(const Csr& G, std::vector<int>& colour) {
  const int n = G.n;
  if (n == 0) return false;
  std::vector<int> depth(n, -1), queue;
  queue.reserve(n);
  depth[0] = 0;
  queue.push_back(0);
  for (size_t h = 0; h < queue.size(); ++h) {
    const int v = queue[h];
    for (int k = G.rp[v]; k < G.rp[v + 1]; ++k) {
      const int u = G.ci[k];
      if (depth[u] < 0) {
        depth[u] = depth[v] + 1;
        queue.push_back(u);
      }
    }
  }
  if ((int)queue.size() != n) return false;
  for (int v = 0; v < n; ++v)
    for (int k = G.rp[v]; k < G.rp[v + 1]; ++k)
      if ((depth[v] & 1) == (depth[G.ci[k]] & 1)) return false;
  colour.assign(n, 0);
  for (int v = 0; v < n; ++v) colour[v] = depth[v] & 1;
  return true;
}

// The smoother's colouring of a level graph: red-black when the graph is
// connected and bipartite, greedy first-fit in priority order otherwise.
int colour_level(const Csr& G, uint64_t seed, int level, std::vector<int>& colour) {
  if (colour_bipartite(G, colour)) return G.n > 1 ? 2 : 1;
  return colour_greedy(G, seed, level, colour);
}

void group_by_colour(Level& L) {
  L.by_colour.assign(L.ncolours, {});
  for (int i = 0; i < L.n; ++i) L.by_colour[L.colour[i]].push_back(i);
}

// ---------------------------------------------------------------------------
// One multicoloured Gauss-Seidel pass over all colours, forward (0..C-1) or
// backward (C-1..0).  Row i: s = sum_j a_ij x_j as an fma chain in CSR order,
// x_i = (b_i - s) * dinv_i.  Rows of one colour are independent.
// ---------------------------------------------------------------------------
template <typename T>
void gs_sweep_t(const Level& L, const std::vector<T>& a, const std::vector<T>& dinv, const T* b, T* x,
                bool forward) {
  for (int t = 0; t < L.ncolours; ++t) {
    int c = forward ? t : L.ncolours - 1 - t;
    for (int i : L.by_colour[c]) {
      T s = 0;
      for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) s = std::fma(a[k], x[L.A.ci[k]], s);
      x[i] = (b[i] - s) * dinv[i];
    }
  }
}

// Residual r = b - A x with s = d_i x_i, then the off-diagonal fma chain.
template <typename T>
void residual_t(const Level& L, const std::vector<T>& a, const std::vector<T>& d, const T* b, const T* x, T* r) {
  for (int i = 0; i < L.n; ++i) {
    T s = d[i] * x[i];
    for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) s = std::fma(a[k], x[L.A.ci[k]], s);
    r[i] = b[i] - s;
  }
}

// Product q = A p with the same sum order as the residual: s = d_i p_i, then the
// off-diagonal fma chain in CSR order.
template <typename T>
void spmv_t(const Level& L, const std::vector<T>& a, const std::vector<T>& d, const T* p, T* q) {
  for (int i = 0; i < L.n; ++i) {
    T s = d[i] * p[i];
    for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) s = std::fma(a[k], p[L.A.ci[k]], s);
    q[i] = s;
  }
}

// ---------------------------------------------------------------------------
// Off-diagonal sparsity pattern of A^2 (Alg. 4, Step 2): pairs at graph
// distance 1 or 2.  With hub_cap > 0 a two-step pair counts only through
// middle vertices of degree <= hub_cap.
// ---------------------------------------------------------------------------
Csr a2_pattern(const Csr& G, int hub_cap) {
  Csr out;
  out.n = G.n;
  out.rp.assign(G.n + 1, 0);
  std::vector<int> mark(G.n, -1), row;
  for (int i = 0; i < G.n; ++i) {
    row.clear();
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      int p = G.ci[k];
      if (mark[p] != i) { mark[p] = i; row.push_back(p); }
      if (hub_cap == 0 || G.deg(p) <= hub_cap) {
        for (int q = G.rp[p]; q < G.rp[p + 1]; ++q) {
          int j = G.ci[q];
          if (j != i && mark[j] != i) { mark[j] = i; row.push_back(j); }
        }
      }
    }
    std::sort(row.begin(), row.end());
    out.ci.insert(out.ci.end(), row.begin(), row.end());
    out.rp[i + 1] = (int)out.ci.size();
  }
  out.v.assign(out.ci.size(), 0.0);
  return out;
}

// Keys and reweighted values on the A^2 pattern (Alg. 4, Step 2).
bool reweight(Csr& G, std::vector<double>& gkey, const std::vector<double>& e) {
  double mx = 0.0;
  for (double x : e) {
    if (!std::isfinite(x)) { g_err = "smooth error is not finite"; return false; }
    mx = std::max(mx, std::fabs(x));
  }
  if (mx == 0.0) { g_err = "smooth error is identically zero"; return false; }
  const double tau = 0x1.0p-52 * mx;
  gkey.assign(G.ci.size(), 0.0);
  for (int i = 0; i < G.n; ++i)
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      double key = std::fabs(e[i] - e[G.ci[k]]);
      gkey[k] = key;
      G.v[k] = 1.0 / std::max(key, tau);
    }
  return true;
}

// Undirected edges (i < j) of a symmetric pattern in lexicographic (edge index)
// order, then sorted by descending weight = ascending key, ties by edge index
// (Alg. 1, Step 3).
void sorted_edges(const Csr& G, const std::vector<double>& gkey, std::vector<int>& su, std::vector<int>& sv) {
  std::vector<int> eu, ev;
  std::vector<double> ek;
  for (int i = 0; i < G.n; ++i)
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k)
      if (G.ci[k] > i) { eu.push_back(i); ev.push_back(G.ci[k]); ek.push_back(gkey[k]); }
  std::vector<int> idx(eu.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ek[a] < ek[b]; });
  su.resize(idx.size());
  sv.resize(idx.size());
  for (size_t t = 0; t < idx.size(); ++t) { su[t] = eu[idx[t]]; sv[t] = ev[idx[t]]; }
}

// ---------------------------------------------------------------------------
// Greedy 1/2-approximate path cover (Alg. 1).  Edges are visited in the given
// order; an edge is taken when both ends are endpoints (cover degree < 2) and
// they are not the two ends of one path.  other[v] is the far end of v's path
// (v itself when v is not yet on a path).
// ---------------------------------------------------------------------------
void path_cover(int n, const std::vector<int>& su, const std::vector<int>& sv, std::vector<int>& nb) {
  std::vector<int> deg(n, 0), other(n);
  std::iota(other.begin(), other.end(), 0);
  nb.assign(2 * (size_t)n, -1);
  for (size_t t = 0; t < su.size(); ++t) {
    int u = su[t], v = sv[t];
    if (deg[u] >= 2 || deg[v] >= 2) continue;
    if (other[u] == v) continue;
    int a = other[u], b = other[v];
    nb[2 * (size_t)u + deg[u]] = v;
    nb[2 * (size_t)v + deg[v]] = u;
    deg[u]++;
    deg[v]++;
    other[a] = b;
    other[b] = a;
  }
}

int cover_degree(const std::vector<int>& nb, int v) { return (nb[2 * (size_t)v] >= 0) + (nb[2 * (size_t)v + 1] >= 0); }

// Paths of the cover: start at the endpoint with the smaller id; pos counts from 0.
void orient_paths(int n, const std::vector<int>& nb, std::vector<int>& path_id, std::vector<int>& pos,
                  std::vector<int>& plen, int& npaths) {
  path_id.assign(n, -1);
  pos.assign(n, -1);
  plen.assign(n, 0);
  npaths = 0;
  for (int s = 0; s < n; ++s) {
    if (cover_degree(nb, s) != 1 || path_id[s] >= 0) continue;
    // find the far end
    int prev = -1, cur = s, len = 1;
    while (true) {
      int nx = -1;
      for (int t = 0; t < 2; ++t) {
        int w = nb[2 * (size_t)cur + t];
        if (w >= 0 && w != prev) nx = w;
      }
      if (nx < 0) break;
      prev = cur;
      cur = nx;
      ++len;
    }
    int start = std::min(s, cur);
    prev = -1;
    cur = start;
    for (int p = 0; p < len; ++p) {
      path_id[cur] = start;
      pos[cur] = p;
      plen[cur] = len;
      int nx = -1;
      for (int t = 0; t < 2; ++t) {
        int w = nb[2 * (size_t)cur + t];
        if (w >= 0 && w != prev) nx = w;
      }
      prev = cur;
      cur = nx;
    }
    ++npaths;
  }
}

bool adjacent(const Csr& G, int a, int b) {
  return std::binary_search(G.ci.begin() + G.rp[a], G.ci.begin() + G.rp[a + 1], b);
}

// Best neighbour of u in the level graph (Alg. 3, Step 10): the heaviest edge.
// On the finest level the keys decide (smaller key = heavier); on coarser
// levels the coarsened weights.  Ties go to the smaller neighbour id.
int best_neighbour(const Csr& G, const std::vector<double>* gkey, int u) {
  int best = -1;
  double bv = 0.0;
  for (int k = G.rp[u]; k < G.rp[u + 1]; ++k) {
    if (gkey) {
      double key = (*gkey)[k];
      if (best < 0 || key < bv) { best = G.ci[k]; bv = key; }
    } else {
      double w = G.v[k];
      if (best < 0 || w > bv) { best = G.ci[k]; bv = w; }
    }
  }
  return best;
}

// ---------------------------------------------------------------------------
// Aggregation along the path cover (Alg. 3): pair consecutive path vertices,
// then treat every vertex left over in ascending id order (Cases 1-3).
// Aggregates are numbered by their smallest member.
// ---------------------------------------------------------------------------
void aggregate(Level& L, int case3 = 0) {
  const int n = L.n;
  std::vector<int> obj(n, -1);
  std::vector<std::vector<int>> members;
  std::vector<int> centre;  // per aggregate: the vertex it grew at past three members, else -1
  // Steps 5-7: pair along paths
  L.n_path_vertices = 0;
  for (int v = 0; v < n; ++v) {
    if (L.path_id[v] < 0) continue;
    L.n_path_vertices++;
    if (L.pos[v] % 2 == 0 && L.pos[v] + 1 < L.plen[v]) {
      int w = -1;
      for (int t = 0; t < 2; ++t) {
        int c = L.nb[2 * (size_t)v + t];
        if (c >= 0 && L.pos[c] == L.pos[v] + 1) w = c;
      }
      obj[v] = obj[w] = (int)members.size();
      members.push_back({v, w});
      centre.push_back(-1);
    }
  }
  // Steps 9-19: vertices not yet aggregated, ascending id
  L.n_unagg = 0;
  L.case1 = L.case2 = L.case3 = L.middle = L.singleton = 0;
  const std::vector<int> before = obj;
  for (int u = 0; u < n; ++u) if (before[u] < 0) L.n_unagg++;
  for (int u = 0; u < n; ++u) {
    if (obj[u] >= 0) continue;
    int v = best_neighbour(L.G, L.gkey.empty() ? nullptr : &L.gkey, u);
    if (v < 0) {  // no neighbour at all
      obj[u] = (int)members.size();
      members.push_back({u});
      centre.push_back(-1);
      L.singleton++;
      continue;
    }
    if (obj[v] < 0) {  // Case 1
      obj[u] = obj[v] = (int)members.size();
      members.push_back({u, v});
      centre.push_back(-1);
      L.case1++;
      continue;
    }
    int T = obj[v];
    if (members[T].size() <= 2) {  // Case 2 (size 1 treated alike)
      members[T].push_back(u);
      obj[u] = T;
      L.case2++;
      continue;
    }
    // Case 3: take v out of its aggregate, unless that would disconnect it:
    // a 3-chain whose middle is v, or a star (grown past three members, every
    // member adjacent to its centre) whose centre is v.  Then u joins it at v.
    bool take_out;
    if (case3 == 1) {  // as printed: v always leaves
      take_out = true;
    } else if (members[T].size() == 3) {
      std::vector<int> rest;
      for (int m : members[T]) if (m != v) rest.push_back(m);
      take_out = adjacent(L.G, rest[0], rest[1]);
    } else {
      take_out = v != centre[T];
    }
    if (take_out) {
      std::vector<int> rest;
      for (int m : members[T]) if (m != v) rest.push_back(m);
      members[T] = rest;
      obj[u] = obj[v] = (int)members.size();
      members.push_back({u, v});
      centre.push_back(-1);
      L.case3++;
    } else {
      members[T].push_back(u);
      obj[u] = T;
      centre[T] = v;
      L.middle++;
    }
  }
  // canonical numbering: by smallest member
  std::vector<std::pair<int, int>> mins;  // (min member, object)
  for (int o = 0; o < (int)members.size(); ++o) {
    if (members[o].empty()) continue;
    mins.push_back({*std::min_element(members[o].begin(), members[o].end()), o});
  }
  std::sort(mins.begin(), mins.end());
  std::vector<int> canon(members.size(), -1);
  for (int I = 0; I < (int)mins.size(); ++I) canon[mins[I].second] = I;
  L.nc = (int)mins.size();
  L.agg.assign(n, -1);
  for (int v = 0; v < n; ++v) L.agg[v] = canon[obj[v]];
  L.moff.assign(L.nc + 1, 0);
  for (int v = 0; v < n; ++v) L.moff[L.agg[v] + 1]++;
  for (int I = 0; I < L.nc; ++I) L.moff[I + 1] += L.moff[I];
  L.mem.assign(n, 0);
  std::vector<int> fill(L.moff.begin(), L.moff.end() - 1);
  for (int v = 0; v < n; ++v) L.mem[fill[L.agg[v]]++] = v;  // ascending v within each aggregate
}

// ---------------------------------------------------------------------------
// MWM aggregation (Sec. 2.1) of a level on its own weighted adjacency
// w_ij = -a_ij: edges (i < j) visited from heaviest to lightest (ties by
// lexicographic edge index) match their two ends when both are unaggregated.
// The greedy matching is maximal, so every vertex left over has only matched
// neighbours; it joins the aggregate of its heaviest neighbour (ties to the
// smaller id).  A joined vertex is adjacent to one end of a matched pair, so
// every aggregate has diameter <= 3.  A vertex with no neighbour is a
// singleton.  Aggregates are numbered by their smallest member.
// ---------------------------------------------------------------------------
void mwm_aggregate(Level& L) {
  const int n = L.n;
  std::vector<int> eu, ev;
  std::vector<double> ew;
  for (int i = 0; i < n; ++i)
    for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k)
      if (L.A.ci[k] > i) { eu.push_back(i); ev.push_back(L.A.ci[k]); ew.push_back(-L.A.v[k]); }
  std::vector<int> idx(eu.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ew[a] > ew[b]; });
  std::vector<int> obj(n, -1);
  for (int t : idx) {
    const int u = eu[t], v = ev[t];
    if (obj[u] < 0 && obj[v] < 0) obj[u] = obj[v] = u;  // object named by its first end
  }
  L.n_unagg = 0;
  L.case1 = L.case2 = L.case3 = L.middle = L.singleton = 0;
  std::vector<int> joined(n, -1);
  for (int u = 0; u < n; ++u) {
    if (obj[u] >= 0) continue;
    L.n_unagg++;
    int best = -1;
    double bw = 0.0;
    for (int k = L.A.rp[u]; k < L.A.rp[u + 1]; ++k) {
      const double w = -L.A.v[k];
      if (best < 0 || w > bw) { best = L.A.ci[k]; bw = w; }
    }
    joined[u] = best;
  }
  for (int u = 0; u < n; ++u) {  // matched ends only: the left-over vertices' choices are independent
    if (obj[u] >= 0) continue;
    if (joined[u] < 0) { L.singleton++; continue; }
    L.case2++;
  }
  for (int u = 0; u < n; ++u)
    if (obj[u] < 0) obj[u] = joined[u] >= 0 ? obj[joined[u]] : u;
  // canonical numbering by smallest member (vertices in ascending id)
  std::vector<int> canon(n, -1);
  L.nc = 0;
  for (int v = 0; v < n; ++v)
    if (canon[obj[v]] < 0) canon[obj[v]] = L.nc++;
  L.agg.assign(n, -1);
  for (int v = 0; v < n; ++v) L.agg[v] = canon[obj[v]];
  L.moff.assign(L.nc + 1, 0);
  for (int v = 0; v < n; ++v) L.moff[L.agg[v] + 1]++;
  for (int I = 0; I < L.nc; ++I) L.moff[I + 1] += L.moff[I];
  L.mem.assign(n, 0);
  std::vector<int> fill(L.moff.begin(), L.moff.end() - 1);
  for (int v = 0; v < n; ++v) L.mem[fill[L.agg[v]]++] = v;
}

// Prolongation values on the finest level (Sec. 3.3): (P_1)_{k,i} = e_k for
// k in aggregate i, with e normalised and made orthogonal to 1 (Alg. 2, Steps
// 11-12).  Normalisation is a power-of-two scaling to max|e| in [0.5, 1); the
// mean is measured in fixed point (resolution 2^-32), so it is exact and
// independent of summation order.  An aggregate whose |e| < 2^-26 everywhere
// would give a zero column and takes the value 1 instead.
void smooth_prolongation(Level& L, const std::vector<double>& e_raw) {
  const int n = L.n;
  double mx = 0.0;
  for (double x : e_raw) mx = std::max(mx, std::fabs(x));
  int ex = 0;
  std::frexp(mx, &ex);
  std::vector<double> e(n);
  for (int i = 0; i < n; ++i) e[i] = std::ldexp(e_raw[i], -ex);
  int64_t S = 0;
  for (int i = 0; i < n; ++i) S += (int64_t)std::rint(std::ldexp(e[i], 32));
  const double c = std::ldexp((double)S / (double)n, -32);
  for (int i = 0; i < n; ++i) e[i] = e[i] - c;
  L.pval.assign(n, 0.0);
  L.p1_fallback = 0;
  for (int I = 0; I < L.nc; ++I) {
    double m = 0.0;
    for (int t = L.moff[I]; t < L.moff[I + 1]; ++t) m = std::max(m, std::fabs(e[L.mem[t]]));
    bool small = m < 0x1.0p-26;
    if (small) L.p1_fallback++;
    for (int t = L.moff[I]; t < L.moff[I + 1]; ++t) L.pval[L.mem[t]] = small ? 1.0 : e[L.mem[t]];
  }
}

// ---------------------------------------------------------------------------
// Galerkin coarse operator A_{l+1} = P^T A_l P (Alg. 4, Step 8).  Entry (I,J)
// sums (p_k a_kl) p_l over members k of I in ascending order and, within row
// k, the diagonal term first and then the row in CSR order.
// ---------------------------------------------------------------------------
void galerkin(const Level& L, Level& C) {
  const int nc = L.nc;
  C.n = nc;
  C.A = Csr();
  C.A.n = nc;
  C.A.rp.assign(nc + 1, 0);
  C.d.assign(nc, 0.0);
  C.dinv.assign(nc, 0.0);
  std::vector<int> where(nc, -1), cols;
  std::vector<double> acc;
  auto add = [&](int J, double t, double p) {
    if (where[J] < 0) { where[J] = (int)cols.size(); cols.push_back(J); acc.push_back(0.0); }
    acc[where[J]] = std::fma(t, p, acc[where[J]]);
  };
  for (int I = 0; I < nc; ++I) {
    cols.clear();
    acc.clear();
    for (int m = L.moff[I]; m < L.moff[I + 1]; ++m) {
      int k = L.mem[m];
      add(I, L.pval[k] * L.d[k], L.pval[k]);
      for (int e = L.A.rp[k]; e < L.A.rp[k + 1]; ++e) {
        int l = L.A.ci[e];
        add(L.agg[l], L.pval[k] * L.A.v[e], L.pval[l]);
      }
    }
    std::vector<std::pair<int, double>> row;
    for (size_t t = 0; t < cols.size(); ++t) {
      if (cols[t] == I) C.d[I] = acc[t];
      else row.push_back({cols[t], acc[t]});
      where[cols[t]] = -1;
    }
    std::sort(row.begin(), row.end());
    for (auto& pr : row) { C.A.ci.push_back(pr.first); C.A.v.push_back(pr.second); }
    C.A.rp[I + 1] = (int)C.A.ci.size();
    C.dinv[I] = 1.0 / C.d[I];
  }
}

// Reweighted graph on the coarse level (Alg. 4, Step 6) with the boolean
// aggregation matrix: W~_c(I,J) = sum of w~_kl over k in I (ascending), l in J,
// row k in CSR order; I != J.
void coarsen_graph(const Level& L, Level& C) {
  const int nc = L.nc;
  C.G = Csr();
  C.G.n = nc;
  C.G.rp.assign(nc + 1, 0);
  std::vector<int> where(nc, -1), cols;
  std::vector<double> acc;
  for (int I = 0; I < nc; ++I) {
    cols.clear();
    acc.clear();
    for (int m = L.moff[I]; m < L.moff[I + 1]; ++m) {
      int k = L.mem[m];
      for (int e = L.G.rp[k]; e < L.G.rp[k + 1]; ++e) {
        int J = L.agg[L.G.ci[e]];
        if (J == I) continue;
        if (where[J] < 0) { where[J] = (int)cols.size(); cols.push_back(J); acc.push_back(0.0); }
        acc[where[J]] = acc[where[J]] + L.G.v[e];
      }
    }
    std::vector<std::pair<int, double>> row;
    for (size_t t = 0; t < cols.size(); ++t) { row.push_back({cols[t], acc[t]}); where[cols[t]] = -1; }
    std::sort(row.begin(), row.end());
    for (auto& pr : row) { C.G.ci.push_back(pr.first); C.G.v.push_back(pr.second); }
    C.G.rp[I + 1] = (int)C.G.ci.size();
  }
}

// Path shortening (Alg. 4, Step 7): walk every path (ordered by start vertex)
// from its start, map vertices to aggregates and collapse repeats.  A coarse
// vertex belongs to the coarse cover only at its first occurrence; any later
// occurrence is dropped and cuts the coarse path there.
void shorten_paths(const Level& L, std::vector<int>& nbc) {
  const int nc = L.nc;
  std::vector<int64_t> first(nc, std::numeric_limits<int64_t>::max());
  for (int v = 0; v < L.n; ++v)
    if (L.path_id[v] >= 0) {
      int64_t key = ((int64_t)L.path_id[v] << 32) | (int64_t)L.pos[v];
      first[L.agg[v]] = std::min(first[L.agg[v]], key);
    }
  nbc.assign(2 * (size_t)nc, -1);
  std::vector<int> cdeg(nc, 0);
  auto link = [&](int I, int J) {
    nbc[2 * (size_t)I + cdeg[I]++] = J;
    nbc[2 * (size_t)J + cdeg[J]++] = I;
  };
  for (int s = 0; s < L.n; ++s) {
    if (L.path_id[s] != s) continue;  // s is a path start
    int prev = -1, cur = s;
    int prev_run_agg = -1;
    bool prev_run_owned = false;
    for (int p = 0; cur >= 0; ++p) {
      int I = L.agg[cur];
      if (I != prev_run_agg) {  // a new run starts at position p
        bool owned = first[I] == (((int64_t)s << 32) | (int64_t)p);
        if (owned && prev_run_owned) link(prev_run_agg, I);
        prev_run_agg = I;
        prev_run_owned = owned;
      }
      int nx = -1;
      for (int t = 0; t < 2; ++t) {
        int w = L.nb[2 * (size_t)cur + t];
        if (w >= 0 && w != prev) nx = w;
      }
      prev = cur;
      cur = nx;
    }
  }
}

// ---------------------------------------------------------------------------
// Coarsest level: dense LDL^T (no square roots).  Column j:
//   v_k = L_jk D_k (k < j);  D_j = A_jj - sum_k L_jk v_k;  L_ij = (A_ij - sum_k L_ik v_k) / D_j,
// sums as fma chains with k ascending.
// ---------------------------------------------------------------------------
bool ldlt(const std::vector<double>& A, int n, int m, std::vector<double>& L, std::vector<double>& D) {
  L.assign((size_t)m * m, 0.0);
  D.assign(m, 0.0);
  std::vector<double> v(m);
  for (int j = 0; j < m; ++j) {
    for (int k = 0; k < j; ++k) v[k] = L[(size_t)j * m + k] * D[k];
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s = std::fma(-L[(size_t)j * m + k], v[k], s);
    if (!(s > 0.0)) return false;
    D[j] = s;
    L[(size_t)j * m + j] = 1.0;
    for (int i = j + 1; i < m; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t = std::fma(-L[(size_t)i * m + k], v[k], t);
      L[(size_t)i * m + j] = t / s;
    }
  }
  return true;
}

bool factor_coarsest(const Level& L, bool grounded, int mode, Coarsest& cs) {
  const int n = L.n;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    A[(size_t)i * n + i] = L.d[i];
    for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) A[(size_t)i * n + L.A.ci[k]] = L.A.v[k];
  }
  cs.n = n;
  cs.fallback = false;
  bool g = mode == 1 ? true : mode == 2 ? false : grounded;
  if (!g) {
    cs.grounded = false;
    cs.m = n;
    if (ldlt(A, n, n, cs.L, cs.D)) return true;
    cs.fallback = true;
  }
  cs.grounded = true;
  cs.m = n - 1;
  if (cs.m == 0) { cs.L.clear(); cs.D.clear(); return true; }
  if (!ldlt(A, n, n - 1, cs.L, cs.D)) { g_err = "coarsest level: non-positive pivot in grounded LDL^T"; return false; }
  return true;
}

// Solve with the factor: forward (k ascending), diagonal, backward (k descending).
// Grounded: the last unknown is 0, then the mean (sequential sum / n) is removed.
void coarsest_solve(const Coarsest& cs, const double* b, double* x) {
  const int m = cs.m;
  std::vector<double> y(m);
  for (int i = 0; i < m; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s = std::fma(-cs.L[(size_t)i * m + k], y[k], s);
    y[i] = s;
  }
  for (int i = 0; i < m; ++i) y[i] = y[i] / cs.D[i];
  for (int i = m - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = m - 1; k > i; --k) s = std::fma(-cs.L[(size_t)k * m + i], x[k], s);
    x[i] = s;
  }
  if (cs.grounded) {
    x[cs.n - 1] = 0.0;
    double s = 0.0;
    for (int i = 0; i < cs.n; ++i) s = s + x[i];
    double mu = s / (double)cs.n;
    for (int i = 0; i < cs.n; ++i) x[i] = x[i] - mu;
  }
}

// ---------------------------------------------------------------------------
// Multigrid cycle (Alg. 5 "V_cycle"; Alg. 2 "W_cycle"): forward GS,
// residual, restriction b_c = P^T r (fma chain over members ascending),
// gamma recursive calls from x_c = 0 (gamma = 1 V-cycle, 2 W-cycle; one call
// when the next level is the coarsest), prolongation x += P x_c, backward GS.
// The coarsest level is solved directly.
// ---------------------------------------------------------------------------
void cycle64(const Hierarchy& H, int l, const double* b, double* x, int gamma) {
  const Level& L = H.lv[l];
  if (l + 1 == (int)H.lv.size()) { coarsest_solve(H.cs, b, x); return; }
  std::vector<double> r(L.n), bc(L.nc, 0.0), xc(L.nc, 0.0);
  gs_sweep_t<double>(L, L.A.v, L.dinv, b, x, true);
  residual_t<double>(L, L.A.v, L.d, b, x, r.data());
  for (int I = 0; I < L.nc; ++I) {
    double s = 0.0;
    for (int t = L.moff[I]; t < L.moff[I + 1]; ++t) s = std::fma(L.pval[L.mem[t]], r[L.mem[t]], s);
    bc[I] = s;
  }
  const int calls = (gamma > 1 && l + 2 < (int)H.lv.size()) ? gamma : 1;
  for (int c = 0; c < calls; ++c) cycle64(H, l + 1, bc.data(), xc.data(), gamma);
  for (int k = 0; k < L.n; ++k) x[k] = std::fma(L.pval[k], xc[L.agg[k]], x[k]);
  gs_sweep_t<double>(L, L.A.v, L.dinv, b, x, false);
}

void vcycle64(const Hierarchy& H, int l, const double* b, double* x) { cycle64(H, l, b, x, 1); }

// The same cycle in FP32 on FP32 copies of A_l, d_l, dinv_l and P (gamma = 1
// V, 2 W); the coarsest solve stays FP64 (inputs widened, result rounded to
// nearest).
void cycle32(const Hierarchy& H, int l, const float* b, float* x, int gamma) {
  const Level& L = H.lv[l];
  if (l + 1 == (int)H.lv.size()) {
    std::vector<double> b64(L.n), x64(L.n, 0.0);
    for (int i = 0; i < L.n; ++i) b64[i] = (double)b[i];
    coarsest_solve(H.cs, b64.data(), x64.data());
    for (int i = 0; i < L.n; ++i) x[i] = (float)x64[i];
    return;
  }
  std::vector<float> r(L.n), bc(L.nc, 0.0f), xc(L.nc, 0.0f);
  gs_sweep_t<float>(L, H.a32[l], H.dinv32[l], b, x, true);
  residual_t<float>(L, H.a32[l], H.d32[l], b, x, r.data());
  for (int I = 0; I < L.nc; ++I) {
    float s = 0.0f;
    for (int t = L.moff[I]; t < L.moff[I + 1]; ++t) s = std::fma(H.p32[l][L.mem[t]], r[L.mem[t]], s);
    bc[I] = s;
  }
  const int calls = (gamma > 1 && l + 2 < (int)H.lv.size()) ? gamma : 1;
  for (int c = 0; c < calls; ++c) cycle32(H, l + 1, bc.data(), xc.data(), gamma);
  for (int k = 0; k < L.n; ++k) x[k] = std::fma(H.p32[l][k], xc[L.agg[k]], x[k]);
  gs_sweep_t<float>(L, H.a32[l], H.dinv32[l], b, x, false);
}

void vcycle32(const Hierarchy& H, int l, const float* b, float* x) { cycle32(H, l, b, x, 1); }

// ---------------------------------------------------------------------------
// Hierarchy construction (Alg. 4) from the finest level (A, d, dinv, colours)
// and a smooth error e_raw.
// ---------------------------------------------------------------------------
bool finish_hierarchy(Hierarchy& H, const Params& P, bool laplacian_op);

bool build_hierarchy(const Level& fine, const std::vector<double>& e_raw, const Params& P, Hierarchy& H) {
  H.lv.clear();
  H.lv.push_back(Level());
  Level& L0 = H.lv[0];
  L0.n = fine.n;
  L0.A = fine.A;
  L0.d = fine.d;
  L0.dinv = fine.dinv;
  L0.colour = fine.colour;
  L0.ncolours = fine.ncolours;
  group_by_colour(L0);
  // Step 2: reweight on the A^2 pattern; Step 3: path cover on the finest level only
  L0.G = a2_pattern(L0.A, P.a2_hub_cap);
  if (!reweight(L0.G, L0.gkey, e_raw)) return false;
  {
    std::vector<int> su, sv;
    sorted_edges(L0.G, L0.gkey, su, sv);
    path_cover(L0.n, su, sv, L0.nb);
  }
  for (int l = 0;; ++l) {
    Level& L = H.lv[l];
    if (L.n <= P.coarse_max || l + 1 >= P.max_levels) break;
    orient_paths(L.n, L.nb, L.path_id, L.pos, L.plen, L.n_paths);
    aggregate(L, P.case3);
    // stall (n_c > 0.9 n): this level becomes the coarsest, if the dense
    // coarsest solve can take it; a larger level keeps coarsening while it
    // still shrinks
    if (L.nc > 0.9 * L.n && (L.n <= 4096 || L.nc >= L.n)) {
      L.nc = 0;
      L.agg.clear();
      L.moff.clear();
      L.mem.clear();
      break;
    }
    if (l == 0 && P.p1_mode == 0) smooth_prolongation(L, e_raw);
    else L.pval.assign(L.n, 1.0);
    Level C;
    galerkin(L, C);
    coarsen_graph(L, C);
    shorten_paths(L, C.nb);
    C.ncolours = colour_level(C.A, P.colour_seed, l + 1, C.colour);
    group_by_colour(C);
    H.lv.push_back(std::move(C));
  }
  // the coarsest operator is a (singular) Laplacian when no prolongation carries
  // smooth-error values: boolean mode, or no coarsening at all
  return finish_hierarchy(H, P, P.p1_mode == 1 || H.lv.size() == 1);
}

// UA-AMG hierarchy by MWM aggregation on every level (the MWM_setup of
// Alg. 5/6 Step 2, Sec. 2.1): boolean prolongations, Galerkin products, the
// same stopping rule and coarsest solve as Alg. 4's loop.
bool build_hierarchy_mwm(const Level& fine, const Params& P, Hierarchy& H) {
  H.lv.clear();
  H.lv.push_back(Level());
  Level& L0 = H.lv[0];
  L0.n = fine.n;
  L0.A = fine.A;
  L0.d = fine.d;
  L0.dinv = fine.dinv;
  L0.colour = fine.colour;
  L0.ncolours = fine.ncolours;
  group_by_colour(L0);
  for (int l = 0;; ++l) {
    Level& L = H.lv[l];
    if (L.n <= P.coarse_max || l + 1 >= P.max_levels) break;
    mwm_aggregate(L);
    if (L.nc > 0.9 * L.n && (L.n <= 4096 || L.nc >= L.n)) {
      L.nc = 0;
      L.agg.clear();
      L.moff.clear();
      L.mem.clear();
      break;
    }
    L.pval.assign(L.n, 1.0);
    Level C;
    galerkin(L, C);
    C.ncolours = colour_level(C.A, P.colour_seed, l + 1, C.colour);
    group_by_colour(C);
    H.lv.push_back(std::move(C));
  }
  return finish_hierarchy(H, P, true);
}

// Coarsest factor, operator complexity and FP32 copies of a built hierarchy.
bool finish_hierarchy(Hierarchy& H, const Params& P, bool laplacian_op) {
  Level& Lc = H.lv.back();
  if (Lc.n > 4096) { g_err = "coarsest level larger than 4096 vertices"; return false; }
  if (!factor_coarsest(Lc, laplacian_op, P.coarse_solve, H.cs)) return false;
  // operator complexity: nonzeros of all levels (diagonal included) / finest
  double tot = 0.0;
  for (auto& L : H.lv) tot += (double)L.A.nnz() + L.n;
  H.nnz_fine = H.lv[0].A.nnz() + H.lv[0].n;
  H.op_complexity = tot / (double)H.nnz_fine;
  // FP32 copies
  const size_t nl = H.lv.size();
  H.a32.assign(nl, {});
  H.d32.assign(nl, {});
  H.dinv32.assign(nl, {});
  H.p32.assign(nl, {});
  for (size_t l = 0; l < nl; ++l) {
    const Level& L = H.lv[l];
    for (double x : L.A.v) H.a32[l].push_back((float)x);
    for (double x : L.d) H.d32[l].push_back((float)x);
    for (double x : L.dinv) H.dinv32[l].push_back((float)x);
    for (double x : L.pval) H.p32[l].push_back((float)x);
  }
  return true;
}

// Drop the setup-only data (level graphs, keys, paths) once a hierarchy is built.
void strip_setup_data(Hierarchy& H) {
  for (auto& L : H.lv) {
    L.G = Csr();
    std::vector<double>().swap(L.gkey);
    std::vector<int>().swap(L.nb);
    std::vector<int>().swap(L.path_id);
    std::vector<int>().swap(L.pos);
    std::vector<int>().swap(L.plen);
  }
}

double norm2(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s = s + x * x;
  return std::sqrt(s);
}
double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s = s + a[i] * b[i];
  return s;
}
void remove_mean(std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s = s + x;
  double mu = s / (double)v.size();
  for (double& x : v) x = x - mu;
}

// `sweeps` symmetric GS sweeps on A e = 0 (relaxation before every build).
void relax_homogeneous(const Level& fine, int sweeps, std::vector<double>& e) {
  std::vector<double> zero(fine.n, 0.0);
  for (int s = 0; s < sweeps; ++s) {
    gs_sweep_t<double>(fine, fine.A.v, fine.dinv, zero.data(), e.data(), true);
    gs_sweep_t<double>(fine, fine.A.v, fine.dinv, zero.data(), e.data(), false);
  }
}

// Random start vector of build r.
void start_vector(const Params& P, int n, int r, std::vector<double>& e) {
  e.resize(n);
  for (int i = 0; i < n; ++i) e[i] = xi_value(P.seed, r, i);
}

// ---------------------------------------------------------------------------
// Approximate smooth error (Alg. 2): a few PCG steps on A e = r from e = 0.
// While Re <= numW the preconditioner is the W-cycle of the latest hierarchy
// (iterW steps); afterwards the symmetric composite of the V-cycles of all
// hierarchies built so far, B_1 .. B_Re then B_Re .. B_1 (iterV steps).
// Preconditioned vectors and the result are made orthogonal to 1.
// ---------------------------------------------------------------------------
void approximate_error(const Level& fine, const std::vector<Hierarchy>& hist, int Re, const Params& P,
                       const std::vector<double>& r, std::vector<double>& e) {
  const int n = fine.n;
  const bool wcyc = Re <= P.numW;
  const int steps = wcyc ? P.iterW : P.iterV;
  // cycle_prec = FP32: the preconditioning cycles run in FP32 on FP32 copies,
  // their input rounded and their result widened once
  auto prec = [&](const std::vector<double>& v, std::vector<double>& z) {
    z.assign(n, 0.0);
    if (P.cycle_prec == 1) {
      std::vector<float> v32(n), z32(n, 0.0f);
      for (int i = 0; i < n; ++i) v32[i] = (float)v[i];
      if (wcyc) {
        cycle32(hist.back(), 0, v32.data(), z32.data(), 2);
      } else {
        for (int j = 0; j < Re; ++j) cycle32(hist[j], 0, v32.data(), z32.data(), 1);
        for (int j = Re - 1; j >= 0; --j) cycle32(hist[j], 0, v32.data(), z32.data(), 1);
      }
      for (int i = 0; i < n; ++i) z[i] = (double)z32[i];
    } else if (wcyc) {
      cycle64(hist.back(), 0, v.data(), z.data(), 2);
    } else {
      for (int j = 0; j < Re; ++j) cycle64(hist[j], 0, v.data(), z.data(), 1);
      for (int j = Re - 1; j >= 0; --j) cycle64(hist[j], 0, v.data(), z.data(), 1);
    }
    remove_mean(z);
  };
  e.assign(n, 0.0);
  std::vector<double> rr = r, z, p, q(n);
  prec(rr, z);
  p = z;
  double rz = dot(rr, z);
  for (int t = 0; t < steps; ++t) {
    spmv_t<double>(fine, fine.A.v, fine.d, p.data(), q.data());
    double pq = dot(p, q);
    if (!(pq > 0.0)) break;
    double alpha = rz / pq;
    for (int i = 0; i < n; ++i) e[i] = std::fma(alpha, p[i], e[i]);
    if (t + 1 == steps) break;
    for (int i = 0; i < n; ++i) rr[i] = std::fma(-alpha, q[i], rr[i]);
    prec(rr, z);
    double rz2 = dot(rr, z);
    double beta = rz2 / rz;
    for (int i = 0; i < n; ++i) p[i] = std::fma(beta, p[i], z[i]);
    rz = rz2;
  }
  remove_mean(e);
}

struct SolveOut {
  int iterations = 0, rebuilds = 0, status = 0, levels = 0;
  double relres = 0, true_relres = 0, rho_geo = 0, convr_last10 = 0, oc_mean = 0;
  double t_setup = 0, t_solve = 0;
  std::vector<double> relres_hist;
  std::vector<int> rebuild_at;
  int first_levels = 0;
  double first_oc = 0;
};

// Adaptive loop (Alg. 5) with the readings listed at the top of this file.
int solve(const Csr& W, const std::vector<double>& b, const Params& P, const double* x0, std::vector<double>& x,
          SolveOut& out) {
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  const int n = W.n;
  Level fine;
  fine.n = n;
  laplacian(W, fine.A, fine.d, fine.dinv);
  fine.ncolours = colour_level(fine.A, P.colour_seed, 0, fine.colour);
  group_by_colour(fine);
  std::vector<Hierarchy> hist(1);
  if (P.init == 1) {  // MWM_setup (Alg. 5/6 Step 2)
    if (!build_hierarchy_mwm(fine, P, hist[0])) return -1;
  } else {
    std::vector<double> e;
    start_vector(P, n, 0, e);
    relax_homogeneous(fine, P.relax_sweeps, e);
    if (!build_hierarchy(fine, e, P, hist[0])) return -1;
  }
  strip_setup_data(hist[0]);
  out.first_levels = (int)hist[0].lv.size();
  out.first_oc = hist[0].op_complexity;
  double oc_sum = hist[0].op_complexity;
  auto t1 = clk::now();
  out.t_setup = std::chrono::duration<double>(t1 - t0).count();

  x.assign(n, 0.0);
  if (x0) x.assign(x0, x0 + n);
  std::vector<double> r(n);
  residual_t<double>(fine, fine.A.v, fine.d, b.data(), x.data(), r.data());
  const double nr0 = norm2(r);
  out.relres_hist.clear();
  out.relres_hist.push_back(1.0);
  if (nr0 == 0.0) { out.relres = 0; out.levels = (int)hist[0].lv.size(); return 0; }
  double nr_prev = nr0, nr = nr0;
  std::vector<double> conv, conv_all;
  int k = 0;
  // Re-setup (Alg. 5, Steps 13-16).  Returns the correction added to x.
  auto rebuild = [&](const std::vector<double>& res, std::vector<double>& corr) -> bool {
    const int Re = (int)hist.size();
    std::vector<double> eb;
    if (P.rebuild_source == 0) {
      approximate_error(fine, hist, Re, P, res, corr);
      eb = corr;
    } else if (P.rebuild_source == 2) {  // Alg. 6: e = x_{k+1} / ||x_{k+1}||, no further sweeps
      const double nx = norm2(x);
      eb.resize(n);
      for (int i = 0; i < n; ++i) eb[i] = x[i] / nx;
      corr.assign(n, 0.0);
    } else {  // relaxation of A e = 0 from a fresh start vector, exposed to the current cycle
      start_vector(P, n, Re, eb);
      std::vector<double> zero(n, 0.0);
      for (int c = 0; c < P.rebuild_vcycles; ++c) vcycle64(hist.back(), 0, zero.data(), eb.data());
      corr.assign(n, 0.0);
    }
    if (P.rebuild_source != 2) relax_homogeneous(fine, P.relax_sweeps, eb);
    Hierarchy H2;
    if (!build_hierarchy(fine, eb, P, H2)) return false;
    strip_setup_data(H2);
    hist.push_back(std::move(H2));
    out.rebuilds++;
    oc_sum += hist.back().op_complexity;
    out.rebuild_at.push_back(k);
    conv.clear();
    return true;
  };
  const bool mean_rule = P.rebuild_rule == 0;
  auto triggered = [&]() {
    if (out.rebuilds >= P.max_rebuilds) return false;
    if (!mean_rule) return conv.back() > P.theta;
    double mean = 0.0;
    for (double q : conv) mean = mean + q;
    mean = mean / (double)conv.size();
    return mean > P.theta;
  };
  if (P.outer == 0) {
    std::vector<double> corr;
    while (k < P.max_iter) {
      vcycle64(hist.back(), 0, b.data(), x.data());
      remove_mean(x);
      residual_t<double>(fine, fine.A.v, fine.d, b.data(), x.data(), r.data());
      nr = norm2(r);
      ++k;
      double c = nr / nr_prev;
      conv.push_back(c);
      conv_all.push_back(c);
      nr_prev = nr;
      out.relres_hist.push_back(nr / nr0);
      if (!std::isfinite(nr)) { out.status = -12; break; }
      if (nr / nr0 <= P.tol) break;
      if (triggered()) {
        if (!rebuild(r, corr)) return -1;
        if (P.rebuild_source == 0) {
          for (int i = 0; i < n; ++i) x[i] = x[i] + corr[i];
          residual_t<double>(fine, fine.A.v, fine.d, b.data(), x.data(), r.data());
          nr_prev = norm2(r);
        }
      }
    }
  } else {
    auto precond = [&](const std::vector<double>& rr, std::vector<double>& z) {
      z.assign(n, 0.0);
      if (P.cycle_prec == 1) {
        std::vector<float> r32(n), z32(n, 0.0f);
        for (int i = 0; i < n; ++i) r32[i] = (float)rr[i];
        vcycle32(hist.back(), 0, r32.data(), z32.data());
        for (int i = 0; i < n; ++i) z[i] = (double)z32[i];
      } else {
        vcycle64(hist.back(), 0, rr.data(), z.data());
      }
      remove_mean(z);
    };
    std::vector<double> z, p, q(n), rn(n), zn, corr;
    precond(r, z);
    p = z;
    double rz = dot(r, z);
    while (k < P.max_iter) {
      spmv_t<double>(fine, fine.A.v, fine.d, p.data(), q.data());
      double pq = dot(p, q);
      if (!(pq > 0.0)) { out.status = -11; break; }
      double alpha = rz / pq;
      for (int i = 0; i < n; ++i) x[i] = std::fma(alpha, p[i], x[i]);
      for (int i = 0; i < n; ++i) rn[i] = std::fma(-alpha, q[i], r[i]);
      nr = norm2(rn);
      ++k;
      double c = nr / nr_prev;
      conv.push_back(c);
      conv_all.push_back(c);
      nr_prev = nr;
      out.relres_hist.push_back(nr / nr0);
      if (!std::isfinite(nr)) { out.status = -12; break; }
      if (nr / nr0 <= P.tol) { r = rn; break; }
      bool restart = false;
      if (triggered()) {
        if (!rebuild(rn, corr)) return -1;
        if (P.rebuild_source == 0) {
          for (int i = 0; i < n; ++i) x[i] = x[i] + corr[i];
          residual_t<double>(fine, fine.A.v, fine.d, b.data(), x.data(), rn.data());
          nr_prev = norm2(rn);
        }
        restart = true;
      }
      precond(rn, zn);
      if (restart) {
        p = zn;
      } else {
        double num = 0.0;
        for (int i = 0; i < n; ++i) num = num + zn[i] * (rn[i] - r[i]);
        double beta = num / rz;
        for (int i = 0; i < n; ++i) p[i] = std::fma(beta, p[i], zn[i]);
      }
      rz = dot(rn, zn);
      r = rn;
      z = zn;
    }
    remove_mean(x);
  }
  out.iterations = k;
  out.relres = nr / nr0;
  residual_t<double>(fine, fine.A.v, fine.d, b.data(), x.data(), r.data());
  out.true_relres = norm2(r) / nr0;
  out.rho_geo = k > 0 ? std::pow(out.relres, 1.0 / k) : 0.0;
  {
    int m = std::min<int>(10, (int)conv_all.size());
    double s = 0.0;
    for (int t = (int)conv_all.size() - m; t < (int)conv_all.size(); ++t) s = s + conv_all[t];
    out.convr_last10 = m ? s / m : 0.0;
  }
  out.oc_mean = oc_sum / (double)(out.rebuilds + 1);
  out.levels = (int)hist.back().lv.size();
  if (out.status == 0 && out.relres > P.tol) out.status = -10;
  out.t_solve = std::chrono::duration<double>(clk::now() - t1).count();
  return 0;
}

Csr make_csr(int n, const int* rp, const int* ci, const double* w) {
  Csr G;
  G.n = n;
  G.rp.assign(rp, rp + n + 1);
  G.ci.assign(ci, ci + rp[n]);
  if (w) G.v.assign(w, w + rp[n]);
  else G.v.assign(rp[n], 1.0);
  return G;
}

struct HierHandle {
  Level fine;
  Hierarchy H;
  std::vector<double> e;
};

}  // namespace

// ===========================================================================
// C interface (ctypes)
// ===========================================================================
extern "C" {

const char* or_last_error() { return g_err.c_str(); }

void or_xi(int n, unsigned long long seed, int r, double* out) {
  for (int i = 0; i < n; ++i) out[i] = xi_value(seed, r, i);
}

unsigned long long or_colour_priority(unsigned long long seed, int level, int v) { return colour_priority(seed, level, v); }
unsigned long long or_colour_key(unsigned long long seed, int level, int v, int deg) { return colour_key(seed, level, v, deg); }

void or_laplacian(int n, const int* rp, const int* ci, const double* w, double* aval, double* d, double* dinv) {
  Csr W = make_csr(n, rp, ci, w), A;
  std::vector<double> dd, di;
  laplacian(W, A, dd, di);
  std::copy(A.v.begin(), A.v.end(), aval);
  std::copy(dd.begin(), dd.end(), d);
  std::copy(di.begin(), di.end(), dinv);
}

int or_colour(int n, const int* rp, const int* ci, unsigned long long seed, int level, int* colour) {
  Csr G = make_csr(n, rp, ci, nullptr);
  std::vector<int> c;
  int nc = colour_level(G, seed, level, c);
  std::copy(c.begin(), c.end(), colour);
  return nc;
}

int or_colour_greedy(int n, const int* rp, const int* ci, unsigned long long seed, int level, int* colour) {
  Csr G = make_csr(n, rp, ci, nullptr);
  std::vector<int> c;
  int nc = colour_greedy(G, seed, level, c);
  std::copy(c.begin(), c.end(), colour);
  return nc;
}

// In-place GS sweeps on (A, dinv) with the given colouring.
void or_gs(int n, const int* rp, const int* ci, const double* aval, const double* dinv, const int* colour, int ncol,
           const double* b, double* x, int forward, int count) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, aval);
  L.dinv.assign(dinv, dinv + n);
  L.colour.assign(colour, colour + n);
  L.ncolours = ncol;
  group_by_colour(L);
  for (int c = 0; c < count; ++c) gs_sweep_t<double>(L, L.A.v, L.dinv, b, x, forward != 0);
}

void or_gs32(int n, const int* rp, const int* ci, const float* aval, const float* dinv, const int* colour, int ncol,
             const float* b, float* x, int forward) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, nullptr);
  L.colour.assign(colour, colour + n);
  L.ncolours = ncol;
  group_by_colour(L);
  std::vector<float> a(aval, aval + rp[n]), di(dinv, dinv + n);
  gs_sweep_t<float>(L, a, di, b, x, forward != 0);
}

void or_residual(int n, const int* rp, const int* ci, const double* aval, const double* d, const double* b,
                 const double* x, double* r) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, aval);
  std::vector<double> dd(d, d + n);
  residual_t<double>(L, L.A.v, dd, b, x, r);
}

// First-build smooth error: Laplacian, colouring of level 0, start vector of
// build 0, `sweeps` symmetric sweeps on A e = 0.
void or_smooth_error(int n, const int* rp, const int* ci, const double* w, unsigned long long colour_seed,
                     unsigned long long seed, int sweeps, double* e_out) {
  Level fine;
  fine.n = n;
  laplacian(make_csr(n, rp, ci, w), fine.A, fine.d, fine.dinv);
  fine.ncolours = colour_level(fine.A, colour_seed, 0, fine.colour);
  group_by_colour(fine);
  Params P{};
  P.seed = seed;
  std::vector<double> e;
  start_vector(P, n, 0, e);
  relax_homogeneous(fine, sweeps, e);
  std::copy(e.begin(), e.end(), e_out);
}

long long or_a2_count(int n, const int* rp, const int* ci, int cap, int* rp2) {
  Csr G2 = a2_pattern(make_csr(n, rp, ci, nullptr), cap);
  std::copy(G2.rp.begin(), G2.rp.end(), rp2);
  return G2.nnz();
}

void or_a2_fill(int n, const int* rp, const int* ci, int cap, int* ci2) {
  Csr G2 = a2_pattern(make_csr(n, rp, ci, nullptr), cap);
  std::copy(G2.ci.begin(), G2.ci.end(), ci2);
}

// Sorted undirected edges of a symmetric pattern by (key asc, edge index asc).
void or_sorted_edges(int n, const int* rp2, const int* ci2, const double* e, int* su, int* sv) {
  Csr G = make_csr(n, rp2, ci2, nullptr);
  std::vector<double> key;
  std::vector<double> ev(e, e + n);
  reweight(G, key, ev);
  std::vector<int> a, b;
  sorted_edges(G, key, a, b);
  std::copy(a.begin(), a.end(), su);
  std::copy(b.begin(), b.end(), sv);
}

void or_path_cover(int n, int m, const int* su, const int* sv, int* nb) {
  std::vector<int> a(su, su + m), b(sv, sv + m), out;
  path_cover(n, a, b, out);
  std::copy(out.begin(), out.end(), nb);
}

// Orientation of a cover: path_id (start vertex), pos, path length per vertex.
int or_orient(int n, const int* nb, int* path_id, int* pos, int* plen) {
  std::vector<int> vnb(nb, nb + 2 * (size_t)n), pid, ps, pl;
  int np = 0;
  orient_paths(n, vnb, pid, ps, pl, np);
  std::copy(pid.begin(), pid.end(), path_id);
  std::copy(ps.begin(), ps.end(), pos);
  std::copy(pl.begin(), pl.end(), plen);
  return np;
}

// Aggregation of one level given its level graph (G, values w), optional keys
// (finest level) and cover.  stats: n_unagg, case1, case2, case3, middle, singleton.
int or_aggregate(int n, const int* grp, const int* gci, const double* gw, const double* gkey, const int* nb,
                 int case3, int* agg, int* stats) {
  Level L;
  L.n = n;
  L.G = make_csr(n, grp, gci, gw);
  if (gkey) L.gkey.assign(gkey, gkey + grp[n]);
  L.nb.assign(nb, nb + 2 * (size_t)n);
  orient_paths(n, L.nb, L.path_id, L.pos, L.plen, L.n_paths);
  aggregate(L, case3);
  std::copy(L.agg.begin(), L.agg.end(), agg);
  if (stats) {
    stats[0] = L.n_unagg; stats[1] = L.case1; stats[2] = L.case2;
    stats[3] = L.case3; stats[4] = L.middle; stats[5] = L.singleton;
  }
  return L.nc;
}

// MWM aggregation of one level given its off-diagonal entries a_ij (weights
// -a_ij).  stats: n_unagg (left after the matching), joined, singleton.
int or_mwm_aggregate(int n, const int* rp, const int* ci, const double* aval, int* agg, int* stats) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, aval);
  mwm_aggregate(L);
  std::copy(L.agg.begin(), L.agg.end(), agg);
  if (stats) { stats[0] = L.n_unagg; stats[1] = L.case2; stats[2] = L.singleton; }
  return L.nc;
}

// Hierarchy object -----------------------------------------------------------
struct or_params_c {
  double tol;
  double theta;
  int max_iter;
  int outer;
  int cycle_prec;
  int coarse_max;
  int relax_sweeps;
  int rebuild_vcycles;
  int rebuild_source;
  int p1_mode;
  int coarse_solve;
  int a2_hub_cap;
  int max_rebuilds;
  int max_levels;
  int numW, iterW, iterV;
  int rebuild_rule;
  unsigned long long seed;
  unsigned long long colour_seed;
  int case3;
  int init;
};

static Params to_params(const or_params_c* p) {
  Params P;
  P.case3 = p->case3; P.init = p->init;
  P.tol = p->tol; P.theta = p->theta; P.max_iter = p->max_iter; P.outer = p->outer;
  P.cycle_prec = p->cycle_prec; P.coarse_max = p->coarse_max; P.relax_sweeps = p->relax_sweeps;
  P.rebuild_vcycles = p->rebuild_vcycles; P.rebuild_source = p->rebuild_source; P.p1_mode = p->p1_mode;
  P.coarse_solve = p->coarse_solve; P.a2_hub_cap = p->a2_hub_cap; P.max_rebuilds = p->max_rebuilds;
  P.max_levels = p->max_levels; P.seed = p->seed; P.colour_seed = p->colour_seed;
  P.numW = p->numW; P.iterW = p->iterW; P.iterV = p->iterV; P.rebuild_rule = p->rebuild_rule;
  return P;
}

// Build a hierarchy from graph weights and a given smooth error (e == NULL:
// the first-build smooth error from the parameters' seed).
void* or_hier_build(int n, const int* rp, const int* ci, const double* w, const double* e, const or_params_c* pc) {
  Params P = to_params(pc);
  auto* h = new HierHandle();
  h->fine.n = n;
  laplacian(make_csr(n, rp, ci, w), h->fine.A, h->fine.d, h->fine.dinv);
  h->fine.ncolours = colour_level(h->fine.A, P.colour_seed, 0, h->fine.colour);
  group_by_colour(h->fine);
  if (P.init == 1 && !e) {  // MWM hierarchy: no smooth error
    if (!build_hierarchy_mwm(h->fine, P, h->H)) { delete h; return nullptr; }
    return h;
  }
  if (e) {
    h->e.assign(e, e + n);
  } else {
    start_vector(P, n, 0, h->e);
    relax_homogeneous(h->fine, P.relax_sweeps, h->e);
  }
  if (!build_hierarchy(h->fine, h->e, P, h->H)) { delete h; return nullptr; }
  return h;
}

void or_hier_free(void* hp) { delete static_cast<HierHandle*>(hp); }

int or_hier_levels(void* hp) { return (int)static_cast<HierHandle*>(hp)->H.lv.size(); }

// info: n, nnz(A), ncolours, nc, nnz(G), npaths, n_unagg, case1, case2, case3,
// middle, singleton, p1_fallback, coarsest grounded, coarsest fallback, n_path_vertices
void or_hier_info(void* hp, int l, long long* info) {
  auto* h = static_cast<HierHandle*>(hp);
  const Level& L = h->H.lv[l];
  long long v[16] = {L.n, L.A.nnz(), L.ncolours, L.nc, L.G.nnz(), L.n_paths, L.n_unagg, L.case1, L.case2,
                     L.case3, L.middle, L.singleton, L.p1_fallback, h->H.cs.grounded, h->H.cs.fallback,
                     L.n_path_vertices};
  std::memcpy(info, v, sizeof(v));
}

double or_hier_oc(void* hp) { return static_cast<HierHandle*>(hp)->H.op_complexity; }

int or_hier_get_int(void* hp, int l, const char* name, int* out) {
  auto* h = static_cast<HierHandle*>(hp);
  const Level& L = h->H.lv[l];
  const std::vector<int>* src = nullptr;
  std::string s(name);
  if (s == "colour") src = &L.colour;
  else if (s == "agg") src = &L.agg;
  else if (s == "path_id") src = &L.path_id;
  else if (s == "pos") src = &L.pos;
  else if (s == "nb") src = &L.nb;
  else if (s == "A_rp") src = &L.A.rp;
  else if (s == "A_ci") src = &L.A.ci;
  else if (s == "G_rp") src = &L.G.rp;
  else if (s == "G_ci") src = &L.G.ci;
  else if (s == "moff") src = &L.moff;
  else if (s == "mem") src = &L.mem;
  if (!src) return -1;
  std::copy(src->begin(), src->end(), out);
  return (int)src->size();
}

int or_hier_get_dbl(void* hp, int l, const char* name, double* out) {
  auto* h = static_cast<HierHandle*>(hp);
  const Level& L = h->H.lv[l];
  const std::vector<double>* src = nullptr;
  std::string s(name);
  if (s == "A_v") src = &L.A.v;
  else if (s == "d") src = &L.d;
  else if (s == "dinv") src = &L.dinv;
  else if (s == "pval") src = &L.pval;
  else if (s == "G_v") src = &L.G.v;
  else if (s == "gkey") src = &L.gkey;
  else if (s == "e") src = &h->e;
  if (!src) return -1;
  std::copy(src->begin(), src->end(), out);
  return (int)src->size();
}

void or_hier_vcycle(void* hp, const double* b, double* x) {
  auto* h = static_cast<HierHandle*>(hp);
  vcycle64(h->H, 0, b, x);
}

void or_hier_vcycle32(void* hp, const float* b, float* x) {
  auto* h = static_cast<HierHandle*>(hp);
  vcycle32(h->H, 0, b, x);
}

void or_hier_coarsest_solve(void* hp, const double* b, double* x) {
  auto* h = static_cast<HierHandle*>(hp);
  coarsest_solve(h->H.cs, b, x);
}

// One FP32 cycle (gamma = 1 V, 2 W) of this hierarchy at level 0.
void or_hier_cycle32(void* hp, const float* b, float* x, int gamma) {
  auto* h = static_cast<HierHandle*>(hp);
  cycle32(h->H, 0, b, x, gamma);
}

// One cycle (gamma = 1 V, 2 W) of this hierarchy at level 0.
void or_hier_cycle(void* hp, const double* b, double* x, int gamma) {
  auto* h = static_cast<HierHandle*>(hp);
  cycle64(h->H, 0, b, x, gamma);
}

// Error approximation (Alg. 2) with the hierarchies hs[0..count-1] as P_hist
// (Re = count).
void or_approx_error(void** hs, int count, const or_params_c* pc, const double* r, double* e_out) {
  Params P = to_params(pc);
  std::vector<Hierarchy> hist;
  for (int j = 0; j < count; ++j) hist.push_back(static_cast<HierHandle*>(hs[j])->H);
  const Level& fine = static_cast<HierHandle*>(hs[0])->fine;
  std::vector<double> rv(r, r + fine.n), e;
  approximate_error(fine, hist, count, P, rv, e);
  std::copy(e.begin(), e.end(), e_out);
}

// Homogeneous rebuild vector: start vector of build r, `rebuild_vcycles`
// V-cycles of this hierarchy on A e = 0, then the relaxation sweeps.
void or_hier_relax_error(void* hp, const or_params_c* pc, int r, double* e_out) {
  auto* h = static_cast<HierHandle*>(hp);
  Params P = to_params(pc);
  std::vector<double> e, zero(h->fine.n, 0.0);
  start_vector(P, h->fine.n, r, e);
  for (int c = 0; c < P.rebuild_vcycles; ++c) vcycle64(h->H, 0, zero.data(), e.data());
  relax_homogeneous(h->fine, P.relax_sweeps, e);
  std::copy(e.begin(), e.end(), e_out);
}

// Full adaptive solve.  stats: iterations, rebuilds, status, levels, relres,
// true_relres, rho_geo, convr_last10, oc_mean, t_setup, t_solve, first_levels, first_oc
int or_solve(int n, const int* rp, const int* ci, const double* w, const double* b, const or_params_c* pc,
             const double* x0, double* x_out, double* stats, double* hist, int hist_cap, int* rebuild_at,
             int rb_cap) {
  Params P = to_params(pc);
  std::vector<double> bv(b, b + n), x;
  SolveOut out;
  int rc = solve(make_csr(n, rp, ci, w), bv, P, x0, x, out);
  if (rc != 0) return rc;
  std::copy(x.begin(), x.end(), x_out);
  double s[13] = {(double)out.iterations, (double)out.rebuilds, (double)out.status, (double)out.levels,
                  out.relres, out.true_relres, out.rho_geo, out.convr_last10, out.oc_mean, out.t_setup,
                  out.t_solve, (double)out.first_levels, out.first_oc};
  std::memcpy(stats, s, sizeof(s));
  for (int t = 0; t < hist_cap && t < (int)out.relres_hist.size(); ++t) hist[t] = out.relres_hist[t];
  for (int t = 0; t < rb_cap && t < (int)out.rebuild_at.size(); ++t) rebuild_at[t] = out.rebuild_at[t];
  return 0;
}

}  // extern "C"

extern "C" void or_spmv(int n, const int* rp, const int* ci, const double* aval, const double* d, const double* p,
                        double* q) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, aval);
  std::vector<double> dd(d, d + n);
  spmv_t<double>(L, L.A.v, dd, p, q);
}

// Galerkin product of one level on given inputs (off-diagonal CSR + diagonal,
// aggregates, prolongation values).  Two calls: out_ci == NULL returns the
// coarse nnz and fills out_rp; otherwise fills ci, values, diagonal.
extern "C" long long or_galerkin(int n, const int* rp, const int* ci, const double* av, const double* d, int nc,
                                 const int* agg, const double* pval, int* out_rp, int* out_ci, double* out_v,
                                 double* out_d) {
  Level L;
  L.n = n;
  L.A = make_csr(n, rp, ci, av);
  L.d.assign(d, d + n);
  L.nc = nc;
  L.agg.assign(agg, agg + n);
  L.pval.assign(pval, pval + n);
  L.moff.assign(nc + 1, 0);
  for (int v = 0; v < n; ++v) L.moff[agg[v] + 1]++;
  for (int I = 0; I < nc; ++I) L.moff[I + 1] += L.moff[I];
  L.mem.assign(n, 0);
  std::vector<int> fill(L.moff.begin(), L.moff.end() - 1);
  for (int v = 0; v < n; ++v) L.mem[fill[agg[v]]++] = v;
  Level C;
  galerkin(L, C);
  if (out_rp) std::copy(C.A.rp.begin(), C.A.rp.end(), out_rp);
  if (out_ci) {
    std::copy(C.A.ci.begin(), C.A.ci.end(), out_ci);
    std::copy(C.A.v.begin(), C.A.v.end(), out_v);
    std::copy(C.d.begin(), C.d.end(), out_d);
  }
  return C.A.nnz();
}

// Path shortening on a given cover and aggregation: coarse cover neighbours.
extern "C" void or_shorten(int n, const int* nb, int nc, const int* agg, int* nbc) {
  Level L;
  L.n = n;
  L.nb.assign(nb, nb + 2 * (size_t)n);
  orient_paths(n, L.nb, L.path_id, L.pos, L.plen, L.n_paths);
  L.nc = nc;
  L.agg.assign(agg, agg + n);
  std::vector<int> out;
  shorten_paths(L, out);
  std::copy(out.begin(), out.end(), nbc);
}
