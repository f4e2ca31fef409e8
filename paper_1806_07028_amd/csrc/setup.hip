// Hierarchy construction kernels (Alg. 1, Alg. 3, Alg. 4), natural vertex
// numbering.  The greedy, order-dependent steps (path cover, isolated-vertex
// repair) run as deterministic reservations: in each round every pending item
// of a window writes its priority into the slots it reads or writes (atomicMin)
// and applies its decision only if it holds all of them.  This reproduces the
// sequential order's result exactly.
#include <algorithm>
#include <climits>

#include "internal.hpp"

namespace pcamg {

// ---------------------------------------------------------------------------
// A^2 pattern (Alg. 4, Step 2): one wave per row.  Candidates (neighbours and
// neighbours of neighbours through pivots of degree <= cap) are gathered into
// LDS, bitonic-sorted, de-duplicated, and the row itself dropped.
// ---------------------------------------------------------------------------
constexpr int A2_CAP = 2048;

__global__ void a2_cand_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               int32_t cap, int32_t* __restrict__ cand) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t c = rp[i + 1] - rp[i];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    int32_t p = ci[k];
    int32_t dp = rp[p + 1] - rp[p];
    if (cap == 0 || dp <= cap) c += dp;
  }
  cand[i] = (int32_t)std::min<int64_t>(c, INT32_MAX);
}

__global__ void __launch_bounds__(64) a2_row_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, int32_t cap,
                                                    const int32_t* __restrict__ cand,
                                                    const int32_t* __restrict__ rp2, int32_t* __restrict__ out) {
  __shared__ int32_t B[A2_CAP];
  const int32_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= n || cand[i] > A2_CAP) return;  // long rows take the global-memory path
  int cnt = 0;
  const int32_t r0 = rp[i], r1 = rp[i + 1];
  for (int32_t base = r0; base < r1; base += 64) {
    int32_t k = base + lane;
    if (k < r1) B[cnt + (k - r0)] = ci[k];
  }
  cnt += r1 - r0;
  for (int32_t kk = r0; kk < r1; ++kk) {
    const int32_t p = ci[kk];
    const int32_t p0 = rp[p], p1 = rp[p + 1];
    if (cap != 0 && p1 - p0 > cap) continue;
    for (int32_t base = p0; base < p1; base += 64) {
      int32_t k = base + lane;
      if (k < p1) B[cnt + (k - p0)] = ci[k];
    }
    cnt += p1 - p0;
  }
  int S = 1;
  while (S < cnt) S <<= 1;
  for (int t = cnt + lane; t < S; t += 64) B[t] = INT_MAX;
  __syncthreads();
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < S; t += 64) {
        int ixj = t ^ j;
        if (ixj > t) {
          int32_t a = B[t], b = B[ixj];
          bool up = (t & k) == 0;
          if ((a > b) == up) {
            B[t] = b;
            B[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // unique, without the row itself
  int32_t written = 0;
  const int32_t dst0 = rp2 ? rp2[i] : 0;
  for (int base = 0; base < S; base += 64) {
    int t = base + lane;
    int32_t v = t < S ? B[t] : INT_MAX;
    bool keep = v != INT_MAX && v != i && (t == 0 || B[t - 1] != v);
    unsigned long long m = __ballot(keep);
    if (rp2 && keep) {
      unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
      out[dst0 + written + __popcll(m & lt)] = v;
    }
    written += __popcll(m);
  }
  if (!rp2 && lane == 0) out[i] = written;
}

// Rows with more candidates than fit in LDS: candidates of all long rows are
// gathered as (row rank << 32 | column) keys, sorted once, and each row's
// sorted slice is de-duplicated by one workgroup.
constexpr int LONG_BLOCK = 256;

__global__ void long_rows_kernel(int32_t n, const int32_t* __restrict__ cand, int32_t cap_lds,
                                 uint8_t* __restrict__ is_long) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) is_long[i] = cand[i] > cap_lds;
}

__global__ void gather_cand_kernel(int32_t nL, const int32_t* __restrict__ rows, const int32_t* __restrict__ cand,
                                   int32_t* __restrict__ lc) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nL) lc[r] = cand[rows[r]];
}

__global__ void a2_long_gather_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
                                      const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int32_t cap,
                                      uint64_t* __restrict__ keys) {
  const int32_t r = blockIdx.x;
  const int32_t i = rows[r];
  const int64_t base = off[r];
  const uint64_t hi = (uint64_t)r << 32;
  int64_t cnt = 0;
  const int32_t r0 = rp[i], r1 = rp[i + 1];
  for (int32_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) keys[base + (k - r0)] = hi | (uint32_t)ci[k];
  cnt += r1 - r0;
  for (int32_t kk = r0; kk < r1; ++kk) {
    const int32_t p = ci[kk];
    const int32_t p0 = rp[p], p1 = rp[p + 1];
    if (cap != 0 && p1 - p0 > cap) continue;
    for (int32_t k = p0 + threadIdx.x; k < p1; k += blockDim.x) keys[base + cnt + (k - p0)] = hi | (uint32_t)ci[k];
    cnt += p1 - p0;
  }
}

// block-wide exclusive scan of one int per thread (LONG_BLOCK threads)
__device__ int32_t block_scan_excl(int32_t v, int32_t* total) {
  __shared__ int32_t ws[LONG_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int w = 0; w < LONG_BLOCK / 64; ++w) {
      int32_t t = ws[w];
      ws[w] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  int32_t r = x - v + ws[wid];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(LONG_BLOCK)
    a2_long_unique_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
                          const uint64_t* __restrict__ keys, const int32_t* __restrict__ rp2, int32_t* __restrict__ cnt,
                          int32_t* __restrict__ ci2) {
  __shared__ int32_t tot;
  const int32_t r = blockIdx.x;
  const int32_t i = rows[r];
  const int64_t a = off[r], b = off[r + 1];
  int32_t written = 0;
  for (int64_t base = a; base < b; base += LONG_BLOCK) {
    const int64_t t = base + threadIdx.x;
    bool keep = false;
    int32_t col = 0;
    if (t < b) {
      col = (int32_t)(uint32_t)keys[t];
      keep = col != i && (t == a || keys[t - 1] != keys[t]);
    }
    int32_t pos = block_scan_excl(keep ? 1 : 0, &tot);
    if (ci2 && keep) ci2[rp2[i] + written + pos] = col;
    written += tot;
  }
  if (!ci2 && threadIdx.x == 0) cnt[i] = written;
}

struct LongRows {
  int32_t nL = 0;
  DVec<int32_t> rows;
  DVec<int64_t> off;
  int64_t total = 0;
};

// rows whose candidate count exceeds the LDS capacity, with int64 offsets
static LongRows find_long_rows(int32_t n, const int32_t* cand, int32_t cap_lds, hipStream_t s) {
  LongRows L;
  DVec<uint8_t> fl(n);
  DVec<int32_t> rows(n), cnt(1);
  long_rows_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, cand, cap_lds, fl.p);
  PCAMG_LAUNCHED();
  compact_i32(nullptr, fl.p, rows.p, cnt.p, n, s);
  L.nL = read_scalar(cnt.p, s);
  if (L.nL == 0) return L;
  L.rows.resize(L.nL);
  copy_d2d(L.rows.p, rows.p, L.nL, s);
  DVec<int32_t> lc(L.nL);
  gather_cand_kernel<<<grid_for(L.nL, 256), 256, 0, s>>>(L.nL, L.rows.p, cand, lc.p);
  PCAMG_LAUNCHED();
  L.off.resize(L.nL + 1);
  scan_exclusive_i64(lc.p, L.off.p, L.nL, s);
  L.total = read_scalar(L.off.p + (L.nL - 1), s) + read_scalar(lc.p + (L.nL - 1), s);
  copy_h2d(L.off.p + L.nL, &L.total, 1, s);
  PCAMG_HIP(hipStreamSynchronize(s));
  require(L.total < ((int64_t)1 << 31), PCAMG_EUNSUPPORTED,
          "long rows hold more than 2^31 candidates in total; set a2_hub_cap");
  return L;
}

static void a2_long_rows(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, const int32_t* cand,
                         const int32_t* rp2, int32_t* cnt, int32_t* ci2, hipStream_t s) {
  LongRows L = find_long_rows(n, cand, A2_CAP, s);
  if (L.nL == 0) return;
  DVec<uint64_t> keys(L.total), sorted(L.total);
  DVec<uint32_t> vals(L.total), vout(L.total);
  a2_long_gather_kernel<<<L.nL, LONG_BLOCK, 0, s>>>(L.rows.p, L.off.p, rp, ci, cap, keys.p);
  PCAMG_LAUNCHED();
  iota_i32((int32_t*)vals.p, L.total, s);
  radix_sort_u64_u32(keys.p, vals.p, sorted.p, vout.p, L.total, s);
  a2_long_unique_kernel<<<L.nL, LONG_BLOCK, 0, s>>>(L.rows.p, L.off.p, sorted.p, rp2, cnt, ci2);
  PCAMG_LAUNCHED();
}

static void a2_candidates(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, int32_t* cand, hipStream_t s) {
  a2_cand_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, cap, cand);
  PCAMG_LAUNCHED();
}

int64_t a2_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, int32_t* rp2, hipStream_t s) {
  if (n <= 0) return 0;
  DVec<int32_t> cand(n), cnt(n);
  a2_candidates(n, rp, ci, cap, cand.p, s);
  a2_row_kernel<<<n, 64, 0, s>>>(n, rp, ci, cap, cand.p, nullptr, cnt.p);
  PCAMG_LAUNCHED();
  a2_long_rows(n, rp, ci, cap, cand.p, nullptr, cnt.p, nullptr, s);
  DVec<int64_t> off64(n);
  scan_exclusive_i64(cnt.p, off64.p, n, s);
  auto last_off = read_scalar(off64.p + (n - 1), s);
  auto last_cnt = read_scalar(cnt.p + (n - 1), s);
  int64_t total = last_off + last_cnt;
  require(total < INT32_MAX, PCAMG_EUNSUPPORTED, "A^2 pattern larger than 2^31 entries; set a2_hub_cap");
  scan_exclusive_i32(cnt.p, rp2, n, rp2 + n, s);
  return total;
}

void a2_fill(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, const int32_t* rp2, int32_t* ci2,
             hipStream_t s) {
  if (n <= 0) return;
  DVec<int32_t> cand(n);
  a2_candidates(n, rp, ci, cap, cand.p, s);
  a2_row_kernel<<<n, 64, 0, s>>>(n, rp, ci, cap, cand.p, rp2, ci2);
  PCAMG_LAUNCHED();
  a2_long_rows(n, rp, ci, cap, cand.p, rp2, nullptr, ci2, s);
}

// ---------------------------------------------------------------------------
// Keys |e_i - e_j| and reweighted values 1/max(key, tau) (Alg. 4, Step 2) on
// the pattern; the undirected edges (i < j) in lexicographic order get the
// key bits for sorting (non-negative doubles sort like their bit patterns).
// ---------------------------------------------------------------------------
// The A^2 pattern has no diagonal and its rows are sorted by column, so the
// entries j > i of row i are the suffix from its first column above i.
__device__ __forceinline__ int32_t first_upper(int32_t i, int32_t lo, int32_t hi, const int32_t* __restrict__ ci2) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (ci2[mid] > i) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__global__ void upper_count_kernel(int32_t n, const int32_t* __restrict__ rp2, const int32_t* __restrict__ ci2,
                                   int32_t* __restrict__ ucnt) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t k1 = rp2[i + 1];
  ucnt[i] = k1 - first_upper(i, rp2[i], k1, ci2);
}

// One wavefront per row: keys and weights of every entry, and the upper
// entries (j > i) as undirected edges in row-major order.
__global__ void __launch_bounds__(256)
    keys_kernel(int32_t n, const int32_t* __restrict__ rp2, const int32_t* __restrict__ ci2,
                const double* __restrict__ e, const uint64_t* __restrict__ maxbits, const int32_t* __restrict__ uoff,
                double* __restrict__ gkey, double* __restrict__ gv, int32_t* __restrict__ eu,
                int32_t* __restrict__ ev, uint64_t* __restrict__ ekey) {
  const int32_t i = (int32_t)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);  // uniform per wavefront
  if (i >= n) return;
  const int lane = (int)(threadIdx.x & 63);
  const double tau = 0x1.0p-52 * __longlong_as_double((long long)*maxbits);
  const double ei = e[i];
  const int32_t k0 = rp2[i], k1 = rp2[i + 1];
  const int32_t fu = first_upper(i, k0, k1, ci2);
  const int32_t ubase = uoff[i];
  for (int32_t k = k0 + lane; k < k1; k += 64) {
    const int32_t j = ci2[k];
    const double key = fabs(ei - e[j]);
    gkey[k] = key;
    gv[k] = 1.0 / fmax(key, tau);
    if (k >= fu) {
      const int32_t u = ubase + (k - fu);
      eu[u] = i;
      ev[u] = j;
      ekey[u] = (uint64_t)__double_as_longlong(key);
    }
  }
}

int32_t a2_keys(int32_t n, const int32_t* rp2, const int32_t* ci2, const double* e, double* gkey, double* gv,
                int32_t* eu, int32_t* ev, uint64_t* ekey, hipStream_t s) {
  DVec<uint64_t> mx(1);
  max_abs_bits_f64(e, n, mx.p, s);
  uint64_t mb = read_scalar(mx.p, s);
  double m;
  std::memcpy(&m, &mb, sizeof m);
  require(m > 0.0 && std::isfinite(m), PCAMG_ENAN, "smooth error is zero or not finite");
  DVec<int32_t> ucnt(n), uoff(n), tot(1);
  upper_count_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp2, ci2, ucnt.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(ucnt.p, uoff.p, n, tot.p, s);
  keys_kernel<<<grid_for((size_t)n * 64, 256), 256, 0, s>>>(n, rp2, ci2, e, mx.p, uoff.p, gkey, gv, eu, ev, ekey);
  PCAMG_LAUNCHED();
  return read_scalar(tot.p, s);
}

__global__ void sorted_endpoints_kernel(int32_t m, const uint32_t* __restrict__ order, const int32_t* __restrict__ eu,
                                        const int32_t* __restrict__ ev, int32_t* __restrict__ su,
                                        int32_t* __restrict__ sv) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  uint32_t idx = order[t];
  su[t] = eu[idx];
  sv[t] = ev[idx];
}

void sorted_endpoints(int32_t m, const uint32_t* order, const int32_t* eu, const int32_t* ev, int32_t* su,
                      int32_t* sv, hipStream_t s) {
  if (m <= 0) return;
  sorted_endpoints_kernel<<<grid_for(m, 256), 256, 0, s>>>(m, order, eu, ev, su, sv);
  PCAMG_LAUNCHED();
}

// ---------------------------------------------------------------------------
// Greedy path cover (Alg. 1) by deterministic reservations.  State: deg[v],
// other[v] = far end of v's path (v when v is on no path).  Edge t (rank t)
// is rejected if an end is saturated or the ends are the two ends of one path
// (both monotone facts, so safe to decide early); otherwise it reserves
// {u, v, other[u], other[v]} and commits iff it holds all four.
// ---------------------------------------------------------------------------
__global__ void window_kernel(int32_t ns, int32_t next, int32_t take, int32_t* __restrict__ win) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < take) win[ns + x] = next + x;
}

__global__ void pc_reserve_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                  const int32_t* __restrict__ sv, const int32_t* __restrict__ deg,
                                  const int32_t* __restrict__ other, uint32_t* __restrict__ res,
                                  int2* __restrict__ ends, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  const int32_t t = win[x];
  const int32_t u = su[t], v = sv[t];
  if (deg[u] >= 2 || deg[v] >= 2 || other[u] == v) {
    state[x] = 0;
    return;
  }
  const int32_t a = other[u], b = other[v];
  ends[x] = make_int2(a, b);
  atomicMin(&res[u], (uint32_t)t);
  atomicMin(&res[v], (uint32_t)t);
  atomicMin(&res[a], (uint32_t)t);
  atomicMin(&res[b], (uint32_t)t);
  state[x] = 1;
}

__global__ void pc_commit_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                 const int32_t* __restrict__ sv, int32_t* __restrict__ deg,
                                 int32_t* __restrict__ other, const uint32_t* __restrict__ res,
                                 const int2* __restrict__ ends, uint8_t* __restrict__ state,
                                 int32_t* __restrict__ nb) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w || state[x] != 1) return;
  const uint32_t t = (uint32_t)win[x];
  const int32_t u = su[t], v = sv[t];
  const int2 ab = ends[x];
  if (res[u] != t || res[v] != t || res[ab.x] != t || res[ab.y] != t) return;
  const int32_t du = deg[u], dv = deg[v];
  nb[2 * (size_t)u + du] = v;
  nb[2 * (size_t)v + dv] = u;
  deg[u] = du + 1;
  deg[v] = dv + 1;
  other[ab.x] = ab.y;
  other[ab.y] = ab.x;
  state[x] = 2;
}

__global__ void pc_reset_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                const int32_t* __restrict__ sv, uint32_t* __restrict__ res,
                                const int2* __restrict__ ends, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  uint8_t st = state[x];
  if (st == 0) return;
  const int32_t t = win[x];
  const int2 ab = ends[x];
  res[su[t]] = UINT_MAX;
  res[sv[t]] = UINT_MAX;
  res[ab.x] = UINT_MAX;
  res[ab.y] = UINT_MAX;
  state[x] = st == 1 ? 1 : 0;  // keep only the still-pending edges
}

int32_t path_cover(int32_t n, int32_t m, const int32_t* su, const int32_t* sv, int32_t* nb, hipStream_t s) {
  fill_i32(nb, -1, 2 * (size_t)n, s);
  if (m <= 0 || n <= 0) return 0;
  DVec<int32_t> deg(n), other(n);
  DVec<uint32_t> res(n);
  fill_i32(deg.p, 0, n, s);
  iota_i32(other.p, n, s);
  fill_u32(res.p, UINT_MAX, n, s);
  const int32_t WIN = std::max<int32_t>(1 << 16, std::min<int32_t>(1 << 20, m / 8 + 1));
  DVec<int32_t> win(WIN), surv(WIN), cnt(1);
  DVec<int2> ends(WIN);
  DVec<uint8_t> state(WIN);
  int32_t ns = 0, next = 0, rounds = 0;
  while (ns > 0 || next < m) {
    // the survivors of the last round are already at the front of win
    const int32_t take = std::min<int32_t>(WIN - ns, m - next);
    if (take > 0) {
      window_kernel<<<grid_for(take, 256), 256, 0, s>>>(ns, next, take, win.p);
      PCAMG_LAUNCHED();
    }
    const int32_t w = ns + take;
    next += take;
    const unsigned g = grid_for(w, 256);
    pc_reserve_kernel<<<g, 256, 0, s>>>(w, win.p, su, sv, deg.p, other.p, res.p, ends.p, state.p);
    PCAMG_LAUNCHED();
    pc_commit_kernel<<<g, 256, 0, s>>>(w, win.p, su, sv, deg.p, other.p, res.p, ends.p, state.p, nb);
    PCAMG_LAUNCHED();
    pc_reset_kernel<<<g, 256, 0, s>>>(w, win.p, su, sv, res.p, ends.p, state.p);
    PCAMG_LAUNCHED();
    compact_i32(win.p, state.p, surv.p, cnt.p, w, s);
    ns = read_scalar(cnt.p, s);
    std::swap(win, surv);  // survivors first in the next window
    ++rounds;
    require(rounds <= 4 * m + 8, PCAMG_EHIP, "path cover did not terminate");
  }
  return rounds;
}

// ---------------------------------------------------------------------------
// Orientation of the paths by pointer jumping on half-edges h = 2v + d
// ("leave v through nb[v][d]"): each half-edge learns the end it reaches and
// its distance.  Path start = smaller end, pos = distance from the start.
// ---------------------------------------------------------------------------
__global__ void pj_init_kernel(int32_t n, const int32_t* __restrict__ nb, int32_t* __restrict__ nxt,
                               int32_t* __restrict__ dist, int32_t* __restrict__ end) {
  int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 2 * n) return;
  const int32_t v = h >> 1;
  const int32_t w = nb[h];
  if (w < 0) {
    nxt[h] = -1;
    dist[h] = 0;
    end[h] = -1;
    return;
  }
  const int32_t dd = nb[2 * w] == v ? 1 : 0;  // leave w away from v
  dist[h] = 1;
  if (nb[2 * w + dd] < 0) {
    nxt[h] = -1;
    end[h] = w;
  } else {
    nxt[h] = 2 * w + dd;
    end[h] = -1;
  }
}

__global__ void pj_jump_kernel(int32_t nh, const int32_t* __restrict__ nxt, const int32_t* __restrict__ dist,
                               const int32_t* __restrict__ end, int32_t* __restrict__ nxt2,
                               int32_t* __restrict__ dist2, int32_t* __restrict__ end2, int32_t* __restrict__ active) {
  int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  const int32_t j = nxt[h];
  if (j < 0) {
    nxt2[h] = -1;
    dist2[h] = dist[h];
    end2[h] = end[h];
    return;
  }
  nxt2[h] = nxt[j];
  dist2[h] = dist[h] + dist[j];
  end2[h] = end[j];
  if (nxt[j] >= 0) *active = 1;
}

__global__ void pj_final_kernel(int32_t n, const int32_t* __restrict__ nb, const int32_t* __restrict__ dist,
                                const int32_t* __restrict__ end, int32_t* __restrict__ path_id,
                                int32_t* __restrict__ pos, int32_t* __restrict__ plen) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const bool h0 = nb[2 * v] >= 0, h1 = nb[2 * v + 1] >= 0;
  if (!h0 && !h1) {
    path_id[v] = -1;
    pos[v] = -1;
    plen[v] = 0;
    return;
  }
  int32_t e0, d0, e1, d1;
  if (h0 && h1) {
    e0 = end[2 * v];
    d0 = dist[2 * v];
    e1 = end[2 * v + 1];
    d1 = dist[2 * v + 1];
  } else {
    const int32_t h = h0 ? 2 * v : 2 * v + 1;
    e0 = v;
    d0 = 0;
    e1 = end[h];
    d1 = dist[h];
  }
  const bool first = e0 < e1;
  path_id[v] = first ? e0 : e1;
  pos[v] = first ? d0 : d1;
  plen[v] = d0 + d1 + 1;
}

void orient_paths_ws(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen, int32_t* ws,
                     hipStream_t s) {
  if (n <= 0) return;
  const size_t nh = 2 * (size_t)n;
  // workspace: six half-edge arrays (next, distance, end; double-buffered) and
  // the "still jumping" flag, which is cleared before every round
  int32_t *nx = ws, *ds = ws + nh, *en = ws + 2 * nh, *nx2 = ws + 3 * nh, *ds2 = ws + 4 * nh, *en2 = ws + 5 * nh;
  int32_t* act = ws + 6 * nh;
  pj_init_kernel<<<grid_for(nh, 256), 256, 0, s>>>(n, nb, nx, ds, en);
  PCAMG_LAUNCHED();
  for (int it = 0; it < 64; ++it) {
    fill_i32(act, 0, 1, s);
    pj_jump_kernel<<<grid_for(nh, 256), 256, 0, s>>>((int32_t)nh, nx, ds, en, nx2, ds2, en2, act);
    PCAMG_LAUNCHED();
    std::swap(nx, nx2);
    std::swap(ds, ds2);
    std::swap(en, en2);
    if (!read_scalar(act, s)) break;
  }
  pj_final_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, nb, ds, en, path_id, pos, plen);
  PCAMG_LAUNCHED();
}

void orient_paths(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen, hipStream_t s) {
  if (n <= 0) return;
  DVec<int32_t> ws(orient_ws_ints(n));
  orient_paths_ws(n, nb, path_id, pos, plen, ws.p, s);
}

// ---------------------------------------------------------------------------
// Aggregation along the cover (Alg. 3).  Aggregate objects are identified by
// the vertex that created them; obj[v] = object of v.  An object keeps its
// size, its centre (the vertex it grew at past three members, else -1) and
// its members as a doubly linked list through the vertices (head, next, prev),
// so that members join and leave in O(1).
// ---------------------------------------------------------------------------
struct AggObjs {
  int32_t* obj;
  int32_t* size;
  int32_t* centre;
  int32_t* head;
  int32_t* next;
  int32_t* prev;
};

__device__ void obj_new2(const AggObjs& o, int32_t u, int32_t v) {  // {u, v}, or {u} when v < 0
  o.obj[u] = u;
  o.size[u] = v >= 0 ? 2 : 1;
  o.centre[u] = -1;
  o.head[u] = u;
  o.prev[u] = -1;
  o.next[u] = v;
  if (v >= 0) {
    o.obj[v] = u;
    o.prev[v] = u;
    o.next[v] = -1;
  }
}

__device__ void obj_push(const AggObjs& o, int32_t T, int32_t u) {
  const int32_t h = o.head[T];
  o.obj[u] = T;
  o.prev[u] = -1;
  o.next[u] = h;
  if (h >= 0) o.prev[h] = u;
  o.head[T] = u;
  o.size[T] += 1;
}

__device__ void obj_remove(const AggObjs& o, int32_t T, int32_t v) {
  const int32_t p = o.prev[v], q = o.next[v];
  if (p >= 0) o.next[p] = q;
  else o.head[T] = q;
  if (q >= 0) o.prev[q] = p;
  o.size[T] -= 1;
}

__global__ void pair_kernel(int32_t n, const int32_t* __restrict__ nb, const int32_t* __restrict__ pid,
                            const int32_t* __restrict__ pos, const int32_t* __restrict__ plen, AggObjs o) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (pid[v] < 0) return;
  const int32_t p = pos[v];
  if ((p & 1) == 0 && p + 1 < plen[v]) {
    int32_t w = nb[2 * v];
    if (w < 0 || pos[w] != p + 1) w = nb[2 * v + 1];
    obj_new2(o, v, w);
  }
}

// best neighbour: smallest (key, id) with keys; else largest weight, ties smaller id
constexpr int32_t BEST_LONG = 256;

__global__ void long_row_flag_kernel(int32_t n, const int32_t* __restrict__ obj, const int32_t* __restrict__ grp,
                                     uint8_t* __restrict__ flag) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  flag[u] = obj[u] < 0 && grp[u + 1] - grp[u] > BEST_LONG;
}

__global__ void best_kernel(int32_t n, const int32_t* __restrict__ obj, const int32_t* __restrict__ grp,
                            const int32_t* __restrict__ gci, const double* __restrict__ gw,
                            const double* __restrict__ gkey, int32_t* __restrict__ best, uint8_t* __restrict__ unagg) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  unagg[u] = obj[u] < 0;
  if (obj[u] >= 0) {
    best[u] = -1;
    return;
  }
  if (grp[u + 1] - grp[u] > BEST_LONG) {  // long rows: best_long_kernel, a wavefront each
    best[u] = -2;
    return;
  }
  int32_t b = -1;
  double bv = 0.0;
  for (int32_t k = grp[u]; k < grp[u + 1]; ++k) {
    if (gkey) {
      double key = gkey[k];
      if (b < 0 || key < bv) { b = gci[k]; bv = key; }
    } else {
      double w = gw[k];
      if (b < 0 || w > bv) { b = gci[k]; bv = w; }
    }
  }
  best[u] = b;
}

// The same for rows of more than BEST_LONG entries, one wavefront per row of
// the list: each lane keeps the best of a strided share, then the lanes'
// candidates are reduced by (weight or key, then column id) -- the unique
// first best of the row in stored (ascending column) order, as above.
__global__ void __launch_bounds__(256)
    best_long_kernel(int32_t m, const int32_t* __restrict__ rows, const int32_t* __restrict__ grp,
                     const int32_t* __restrict__ gci, const double* __restrict__ gw, const double* __restrict__ gkey,
                     int32_t* __restrict__ best) {
  const int32_t t = (int32_t)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);  // uniform per wavefront
  if (t >= m) return;
  const int lane = (int)(threadIdx.x & 63);
  const int32_t u = rows[t];
  int32_t b = -1;
  double bv = 0.0;
  for (int32_t k = grp[u] + lane; k < grp[u + 1]; k += 64) {
    const int32_t c = gci[k];
    if (gkey) {
      const double key = gkey[k];
      if (b < 0 || key < bv) { b = c; bv = key; }
    } else {
      const double w = gw[k];
      if (b < 0 || w > bv) { b = c; bv = w; }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t ob = __shfl_xor(b, o, 64);
    const double ov = __shfl_xor(bv, o, 64);
    bool take;
    if (ob < 0) take = false;
    else if (b < 0) take = true;
    else if (gkey) take = ov < bv || (ov == bv && ob < b);
    else take = ov > bv || (ov == bv && ob < b);
    if (take) { b = ob; bv = ov; }
  }
  if (lane == 0) best[u] = b;
}

enum { ST_SINGLETON = 0, ST_CASE1, ST_CASE2, ST_CASE3, ST_MIDDLE, ST_COUNT };

__global__ void rp_reserve_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ obj,
                                  const int32_t* __restrict__ best, uint32_t* __restrict__ resV,
                                  uint32_t* __restrict__ resO, int2* __restrict__ plan, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  const int32_t u = win[x];
  if (obj[u] >= 0) {  // aggregated by an earlier vertex (Case 1 or 3)
    state[x] = 0;
    return;
  }
  const int32_t v = best[u];
  const int32_t T = v >= 0 ? obj[v] : -1;
  atomicMin(&resV[u], (uint32_t)u);
  if (v >= 0) atomicMin(&resV[v], (uint32_t)u);
  if (T >= 0) atomicMin(&resO[T], (uint32_t)u);
  plan[x] = make_int2(v, T);
  state[x] = 1;
}

__device__ bool adjacent(const int32_t* grp, const int32_t* gci, int32_t a, int32_t b) {
  int32_t lo = grp[a], hi = grp[a + 1];
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    int32_t c = gci[mid];
    if (c == b) return true;
    if (c < b) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

// A winner owns u, v and v's object T for the round: every list link it
// touches belongs to u, v or a member of T.
__global__ void rp_commit_kernel(int32_t w, const int32_t* __restrict__ win, AggObjs o,
                                 const uint32_t* __restrict__ resV, const uint32_t* __restrict__ resO,
                                 const int2* __restrict__ plan, uint8_t* __restrict__ state,
                                 const int32_t* __restrict__ grp, const int32_t* __restrict__ gci,
                                 int32_t* __restrict__ stats, int32_t case3) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w || state[x] != 1) return;
  const uint32_t u = (uint32_t)win[x];
  const int32_t v = plan[x].x, T = plan[x].y;
  if (resV[u] != u || (v >= 0 && resV[v] != u) || (T >= 0 && resO[T] != u)) return;
  state[x] = 2;
  if (v < 0) {  // no neighbour
    obj_new2(o, u, -1);
    atomicAdd(&stats[ST_SINGLETON], 1);
    return;
  }
  if (T < 0) {  // Case 1
    obj_new2(o, u, v);
    atomicAdd(&stats[ST_CASE1], 1);
    return;
  }
  const int32_t sz = o.size[T];
  if (sz <= 2) {  // Case 2
    obj_push(o, T, u);
    atomicAdd(&stats[ST_CASE2], 1);
    return;
  }
  // Case 3: v leaves T unless that disconnects it (v the middle of a 3-chain,
  // or the centre of a star); then u joins T at v.  case3 = 1: as printed,
  // v always leaves.
  bool take_out;
  if (case3 == 1) {
    take_out = true;
  } else if (sz == 3) {
    int32_t rest[2] = {-1, -1}, k = 0;
    for (int32_t m = o.head[T], c = 0; m >= 0 && c < 3; m = o.next[m], ++c)
      if (m != v && k < 2) rest[k++] = m;
    take_out = k == 2 && adjacent(grp, gci, rest[0], rest[1]);
  } else {
    take_out = v != o.centre[T];
  }
  if (take_out) {
    obj_remove(o, T, v);
    obj_new2(o, u, v);
    atomicAdd(&stats[ST_CASE3], 1);
  } else {
    obj_push(o, T, u);
    o.centre[T] = v;
    atomicAdd(&stats[ST_MIDDLE], 1);
  }
}

__global__ void rp_reset_kernel(int32_t w, const int32_t* __restrict__ win, uint32_t* __restrict__ resV,
                                uint32_t* __restrict__ resO, const int2* __restrict__ plan, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  const uint8_t st = state[x];
  if (st == 0) return;
  const int32_t u = win[x];
  resV[u] = UINT_MAX;
  if (plan[x].x >= 0) resV[plan[x].x] = UINT_MAX;
  if (plan[x].y >= 0) resO[plan[x].y] = UINT_MAX;
  state[x] = st == 1 ? 1 : 0;
}

// canonical numbering by smallest member: the smallest member of every object
__global__ void objmin_kernel(int32_t n, const int32_t* __restrict__ obj, int32_t* __restrict__ omin,
                              int32_t* __restrict__ bad) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t T = obj[v];
  if (T < 0 || T >= n) {  // every vertex is aggregated after the repair; guard anyway
    atomicOr(bad, 1);
    return;
  }
  atomicMin(&omin[T], v);
}

__global__ void isroot_kernel(int32_t n, const int32_t* __restrict__ obj, const int32_t* __restrict__ omin,
                              int32_t* __restrict__ isroot) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  isroot[v] = omin[obj[v]] == v;
}

__global__ void canon_kernel(int32_t n, const int32_t* __restrict__ obj, const int32_t* __restrict__ osz,
                             const int32_t* __restrict__ omin, const int32_t* __restrict__ cpos,
                             int32_t* __restrict__ agg, uint32_t* __restrict__ aggu, int32_t* __restrict__ msz) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t T = obj[v];
  const int32_t I = cpos[omin[T]];
  agg[v] = I;
  aggu[v] = (uint32_t)I;
  if (omin[T] == v) msz[I] = osz[T];
}

int32_t number_aggregates(int32_t n, const int32_t* obj, const int32_t* osz, int32_t* agg, int32_t* moff,
                          int32_t* mem, hipStream_t s);

int32_t aggregate_level(int32_t n, const int32_t* grp, const int32_t* gci, const double* gw, const double* gkey,
                        const int32_t* nb, const int32_t* path_id, const int32_t* pos, const int32_t* plen,
                        int32_t* agg, int32_t* moff, int32_t* mem, AggStats& st, hipStream_t s, int32_t case3) {
  DVec<int32_t> obj(n), osz(n), ocen(n), ohead(n), onext(n), oprev(n), best(n), pend(n), cnt(1), stats(ST_COUNT);
  DVec<uint8_t> unagg(n);
  const AggObjs o{obj.p, osz.p, ocen.p, ohead.p, onext.p, oprev.p};
  fill_i32(obj.p, -1, n, s);
  fill_i32(osz.p, 0, n, s);
  fill_i32(stats.p, 0, ST_COUNT, s);
  pair_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, nb, path_id, pos, plen, o);
  PCAMG_LAUNCHED();
  best_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, obj.p, grp, gci, gw, gkey, best.p, unagg.p);
  PCAMG_LAUNCHED();
  {  // rows of more than BEST_LONG entries still unaggregated: a wavefront each
    DVec<uint8_t> lflag(n);
    DVec<int32_t> lrows(n), lcnt(1);
    long_row_flag_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, obj.p, grp, lflag.p);
    PCAMG_LAUNCHED();
    compact_i32(nullptr, lflag.p, lrows.p, lcnt.p, n, s);
    const int32_t nl = read_scalar(lcnt.p, s);
    if (nl > 0) {
      best_long_kernel<<<grid_for((size_t)nl * 64, 256), 256, 0, s>>>(nl, lrows.p, grp, gci, gw, gkey, best.p);
      PCAMG_LAUNCHED();
    }
  }
  compact_i32(nullptr, unagg.p, pend.p, cnt.p, n, s);
  const int32_t npend = read_scalar(cnt.p, s);
  st.n_unagg = npend;
  if (npend > 0) {
    DVec<uint32_t> resV(n), resO(n);
    fill_u32(resV.p, UINT_MAX, n, s);
    fill_u32(resO.p, UINT_MAX, n, s);
    const int32_t WIN = std::max<int32_t>(1 << 14, std::min<int32_t>(1 << 20, npend));
    DVec<int32_t> win(WIN), surv(WIN);
    DVec<int2> plan(WIN);
    DVec<uint8_t> state(WIN);
    int32_t ns = 0, next = 0, rounds = 0;
    while (ns > 0 || next < npend) {
      // the survivors of the last round are already at the front of win
      const int32_t take = std::min<int32_t>(WIN - ns, npend - next);
      if (take > 0) copy_d2d(win.p + ns, pend.p + next, take, s);
      const int32_t w = ns + take;
      next += take;
      const unsigned g = grid_for(w, 256);
      rp_reserve_kernel<<<g, 256, 0, s>>>(w, win.p, obj.p, best.p, resV.p, resO.p, plan.p, state.p);
      PCAMG_LAUNCHED();
      rp_commit_kernel<<<g, 256, 0, s>>>(w, win.p, o, resV.p, resO.p, plan.p, state.p, grp, gci, stats.p, case3);
      PCAMG_LAUNCHED();
      rp_reset_kernel<<<g, 256, 0, s>>>(w, win.p, resV.p, resO.p, plan.p, state.p);
      PCAMG_LAUNCHED();
      compact_i32(win.p, state.p, surv.p, cnt.p, w, s);
      ns = read_scalar(cnt.p, s);
      std::swap(win, surv);  // survivors first in the next window
      ++rounds;
      require(rounds <= 4 * npend + 8, PCAMG_EHIP, "isolated-vertex repair did not terminate");
    }
    st.repair_rounds = rounds;
  }
  auto hs = to_host(stats.p, ST_COUNT, s);
  st.singleton = hs[ST_SINGLETON];
  st.case1 = hs[ST_CASE1];
  st.case2 = hs[ST_CASE2];
  st.case3 = hs[ST_CASE3];
  st.middle = hs[ST_MIDDLE];
  return number_aggregates(n, obj.p, osz.p, agg, moff, mem, s);
}

// Canonical numbering of aggregate objects (object id obj[v] in [0, n), sizes
// osz) by their smallest member, and member lists in ascending id.
// (synchronises)
int32_t number_aggregates(int32_t n, const int32_t* obj, const int32_t* osz, int32_t* agg, int32_t* moff,
                          int32_t* mem, hipStream_t s) {
  DVec<int32_t> omin(n), isroot(n), cpos(n), msz(n), ncd(1), bad(1), vid(n);
  DVec<uint32_t> aggu(n), skeys(n);
  fill_i32(bad.p, 0, 1, s);
  fill_i32(omin.p, INT32_MAX, n, s);
  objmin_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, obj, omin.p, bad.p);
  PCAMG_LAUNCHED();
  require(read_scalar(bad.p, s) == 0, PCAMG_EHIP, "aggregation left a vertex without aggregate");
  isroot_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, obj, omin.p, isroot.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(isroot.p, cpos.p, n, ncd.p, s);
  const int32_t nc = read_scalar(ncd.p, s);
  canon_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, obj, osz, omin.p, cpos.p, agg, aggu.p, msz.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(msz.p, moff, nc, moff + nc, s);
  // members of every aggregate in ascending id: a stable sort of the ids by aggregate
  iota_i32(vid.p, n, s);
  int key_bits = 1;
  while (key_bits < 32 && (1ll << key_bits) < (int64_t)nc) ++key_bits;
  radix_sort_u32_u32(aggu.p, (const uint32_t*)vid.p, skeys.p, (uint32_t*)mem, n, key_bits, s);
  PCAMG_HIP(hipStreamSynchronize(s));
  return nc;
}

// ---------------------------------------------------------------------------
// Level-1 prolongation values (Sec. 3.3): e normalised by a power of two
// (max|e| in [0.5, 1)), centred by its mean measured in fixed point
// (resolution 2^-32, exact integer sum, so independent of summation order);
// an aggregate with max|e| < 2^-26 takes the value 1.
// ---------------------------------------------------------------------------
__global__ void pv_fixed_sum_kernel(const double* __restrict__ e, size_t n, const uint64_t* __restrict__ maxbits,
                                    unsigned long long* __restrict__ sum) {
  int ex;
  frexp(__longlong_as_double((long long)*maxbits), &ex);
  long long acc = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    acc += (long long)rint(ldexp(e[i], 32 - ex));
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(sum, (unsigned long long)acc);
}

__global__ void pv_centre_kernel(const double* __restrict__ e, size_t n, const uint64_t* __restrict__ maxbits,
                                 const unsigned long long* __restrict__ sum, double* __restrict__ ec) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ex;
  frexp(__longlong_as_double((long long)*maxbits), &ex);
  const double c = ldexp((double)(long long)*sum / (double)n, -32);
  ec[i] = ldexp(e[i], -ex) - c;
}

__global__ void pv_assign_kernel(int32_t nc, const int32_t* __restrict__ moff, const int32_t* __restrict__ mem,
                                 const double* __restrict__ ec, double* __restrict__ pval, int32_t* __restrict__ nfb) {
  int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  double m = 0.0;
  for (int32_t t = moff[I]; t < moff[I + 1]; ++t) m = fmax(m, fabs(ec[mem[t]]));
  const bool small = m < 0x1.0p-26;
  if (small) atomicAdd(nfb, 1);
  for (int32_t t = moff[I]; t < moff[I + 1]; ++t) pval[mem[t]] = small ? 1.0 : ec[mem[t]];
}

int32_t smooth_pval(int32_t n, const double* e_raw, int32_t nc, const int32_t* moff, const int32_t* mem,
                    double* pval, hipStream_t s) {
  DVec<uint64_t> mx(1);
  DVec<unsigned long long> sum(1);
  DVec<double> ec(n);
  DVec<int32_t> nfb(1);
  max_abs_bits_f64(e_raw, n, mx.p, s);
  PCAMG_HIP(hipMemsetAsync(sum.p, 0, sizeof(unsigned long long), s));
  fill_i32(nfb.p, 0, 1, s);
  pv_fixed_sum_kernel<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(e_raw, n, mx.p, sum.p);
  PCAMG_LAUNCHED();
  pv_centre_kernel<<<grid_for(n, 256), 256, 0, s>>>(e_raw, n, mx.p, sum.p, ec.p);
  PCAMG_LAUNCHED();
  pv_assign_kernel<<<grid_for(nc, 256), 256, 0, s>>>(nc, moff, mem, ec.p, pval, nfb.p);
  PCAMG_LAUNCHED();
  return read_scalar(nfb.p, s);
}

// ---------------------------------------------------------------------------
// Galerkin product (Alg. 4, Step 8): one wavefront per coarse row I.  The
// row's terms arrive in the defined order -- members k of I ascending; for
// each k the diagonal term, then row k in CSR order -- and are gathered into
// LDS with their sequence number t, bitonic-sorted by (column J, t), and each
// run of equal J is summed by one lane in t order (fma(p_k a_kl, p_l, acc)).
// The reweighted graph is coarsened with boolean P, diagonal dropped, plain
// sums.  Rows with more than GAL_T terms take the long-row path.
// ---------------------------------------------------------------------------
constexpr int GAL_WAVES = 4;   // rows per block
constexpr int GAL_T = 256;     // terms per row held in LDS

__global__ void __launch_bounds__(64 * GAL_WAVES)
    galerkin_kernel(int32_t nc, const int32_t* __restrict__ moff, const int32_t* __restrict__ mem,
                    const int32_t* __restrict__ agg, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const double* __restrict__ av, const double* __restrict__ d, const double* __restrict__ pval,
                    bool graph_mode, const int32_t* __restrict__ rpc, int32_t* __restrict__ count,
                    int32_t* __restrict__ cic, double* __restrict__ vc, double* __restrict__ dc,
                    double* __restrict__ dinvc, uint8_t* __restrict__ overflow) {
  __shared__ uint64_t K[GAL_WAVES][GAL_T];
  __shared__ double TV[GAL_WAVES][GAL_T];
  __shared__ double TP[GAL_WAVES][GAL_T];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t I = blockIdx.x * GAL_WAVES + w;
  if (I >= nc) return;  // whole wave leaves together
  const bool fill = rpc != nullptr;
  const int32_t q0 = moff[I], q1 = moff[I + 1];
  // term count and per-member offsets (at most a handful of members)
  int T = 0;
  for (int32_t q = q0; q < q1; ++q) {
    const int32_t k = mem[q];
    T += (graph_mode ? 0 : 1) + rp[k + 1] - rp[k];
  }
  if (T > GAL_T) {
    if (lane == 0) {
      overflow[I] = 1;
      if (!fill) count[I] = 0;
    }
    return;
  }
  uint64_t* Kw = K[w];
  double* TVw = TV[w];
  double* TPw = TP[w];
  int base = 0;
  for (int32_t q = q0; q < q1; ++q) {
    const int32_t k = mem[q];
    const double pk = pval ? pval[k] : 1.0;
    if (!graph_mode) {
      if (lane == 0) {
        Kw[base] = ((uint64_t)(uint32_t)I << 32) | (uint32_t)base;
        if (fill) {
          TVw[base] = pk * d[k];
          TPw[base] = pk;
        }
      }
      ++base;
    }
    const int32_t e0 = rp[k], e1 = rp[k + 1];
    for (int32_t e = e0 + lane; e < e1; e += 64) {
      const int32_t l = ci[e];
      const int t = base + (e - e0);
      Kw[t] = ((uint64_t)(uint32_t)agg[l] << 32) | (uint32_t)t;
      if (fill) {
        if (graph_mode) {
          TVw[t] = av[e];
        } else {
          TVw[t] = pk * av[e];
          TPw[t] = pval ? pval[l] : 1.0;
        }
      }
    }
    base += e1 - e0;
  }
  int S = 1;
  while (S < T) S <<= 1;
  for (int t = T + lane; t < S; t += 64) Kw[t] = ~0ull;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < S; t += 64) {
        const int ixj = t ^ j;
        if (ixj > t) {
          const uint64_t a = Kw[t], b = Kw[ixj];
          const bool up = (t & k) == 0;
          if ((a > b) == up) {
            Kw[t] = b;
            Kw[ixj] = a;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  }
  // runs of equal column: one lane sums each run in sequence order
  int32_t written = 0;
  const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int p0 = 0; p0 < T; p0 += 64) {
    const int p = p0 + lane;
    bool start = false, counted = false;
    int32_t J = -1;
    double acc = 0.0;
    if (p < T) {
      const uint64_t kp = Kw[p];
      J = (int32_t)(kp >> 32);
      start = p == 0 || (Kw[p - 1] >> 32) != (kp >> 32);
      counted = start && J != I;
      if (start && fill) {
        for (int u = p; u < T && (Kw[u] >> 32) == (kp >> 32); ++u) {
          const int t = (int)(uint32_t)Kw[u];
          acc = graph_mode ? acc + TVw[t] : fma(TVw[t], TPw[t], acc);
        }
      }
    }
    const unsigned long long m = __ballot(counted);
    if (fill) {
      if (start && J == I && !graph_mode) {
        dc[I] = acc;
        dinvc[I] = 1.0 / acc;
      }
      if (counted) {
        const int32_t o = rpc[I] + written + __popcll(m & lt);
        cic[o] = J;
        vc[o] = acc;
      }
    }
    written += __popcll(m);
  }
  if (!fill && lane == 0) count[I] = written;
}

// Long coarse rows (more distinct columns than the LDS list holds): all terms
// of these rows are written out in their defined order, stably sorted by (row,
// column), and every run of equal column is summed in that order.
__global__ void gal_terms_count_kernel(int32_t nL, const int32_t* __restrict__ rows, const int32_t* __restrict__ moff,
                                       const int32_t* __restrict__ mem, const int32_t* __restrict__ rp, bool graph_mode,
                                       int32_t* __restrict__ lc) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nL) return;
  const int32_t I = rows[r];
  int32_t c = 0;
  for (int32_t q = moff[I]; q < moff[I + 1]; ++q) {
    const int32_t k = mem[q];
    c += (graph_mode ? 0 : 1) + rp[k + 1] - rp[k];
  }
  lc[r] = c;
}

__global__ void gal_terms_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
                                 const int32_t* __restrict__ moff, const int32_t* __restrict__ mem,
                                 const int32_t* __restrict__ agg, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ ci, const double* __restrict__ av,
                                 const double* __restrict__ d, const double* __restrict__ pval, bool graph_mode,
                                 uint64_t* __restrict__ keys, double* __restrict__ tv, double* __restrict__ tp) {
  const int32_t r = blockIdx.x;
  const int32_t I = rows[r];
  const uint64_t hi = (uint64_t)r << 32;
  int64_t seq = off[r];
  for (int32_t q = moff[I]; q < moff[I + 1]; ++q) {
    const int32_t k = mem[q];
    const double pk = pval ? pval[k] : 1.0;
    // tv == nullptr: counting pass, keys only (av, d may be null then)
    if (!graph_mode) {
      if (threadIdx.x == 0) {
        if (keys) keys[seq] = hi | (uint32_t)I;
        if (tv) {
          tv[seq] = pk * d[k];
          tp[seq] = pk;
        }
      }
      ++seq;
    }
    const int32_t e0 = rp[k], e1 = rp[k + 1];
    for (int32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
      const int32_t l = ci[e];
      const int64_t t = seq + (e - e0);
      if (keys) keys[t] = hi | (uint32_t)agg[l];
      if (!tv) continue;
      if (graph_mode) {
        tv[t] = av[e];
        tp[t] = 1.0;
      } else {
        tv[t] = pk * av[e];
        tp[t] = pval ? pval[l] : 1.0;
      }
    }
    seq += e1 - e0;
  }
}

__global__ void __launch_bounds__(LONG_BLOCK)
    gal_runs_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ off, const uint64_t* __restrict__ keys,
                    const uint32_t* __restrict__ perm, const double* __restrict__ tv, const double* __restrict__ tp,
                    bool graph_mode, const int32_t* __restrict__ rpc, int32_t* __restrict__ count,
                    int32_t* __restrict__ cic, double* __restrict__ vc, double* __restrict__ dc,
                    double* __restrict__ dinvc) {
  __shared__ int32_t tot;
  const int32_t r = blockIdx.x;
  const int32_t I = rows[r];
  const int64_t a = off[r], b = off[r + 1];
  int32_t written = 0;
  for (int64_t base = a; base < b; base += LONG_BLOCK) {
    const int64_t t = base + threadIdx.x;
    bool start = false;
    int32_t J = -1;
    double acc = 0.0;
    if (t < b) {
      start = t == a || keys[t - 1] != keys[t];
      J = (int32_t)(uint32_t)keys[t];
      if (start && rpc) {
        // the run's terms in order, eight loads in flight at a time (keys
        // are sorted: once a key differs the run has ended); the loads are
        // unconditional (past the row's end: its last term again, not added)
        // so that they issue together
        constexpr int U = 8;
        const uint64_t kt = keys[t];
        for (int64_t u = t;; u += U) {
          bool in[U];
          uint64_t ku[U];
          uint32_t xs[U];
          double v[U], pv[U];
#pragma unroll
          for (int j = 0; j < U; ++j) {
            const int64_t uj = min(u + j, b - 1);
            ku[j] = keys[uj];
            xs[j] = perm[uj];
          }
#pragma unroll
          for (int j = 0; j < U; ++j) in[j] = u + j < b && ku[j] == kt;
#pragma unroll
          for (int j = 0; j < U; ++j) {
            v[j] = tv[xs[j]];
            pv[j] = graph_mode ? 0.0 : tp[xs[j]];
          }
#pragma unroll
          for (int j = 0; j < U; ++j)
            if (in[j]) acc = graph_mode ? acc + v[j] : fma(v[j], pv[j], acc);
          if (!in[U - 1]) break;
        }
      }
    }
    const bool counted = start && J != I;
    if (rpc && start && J == I && !graph_mode) {
      dc[I] = acc;
      dinvc[I] = 1.0 / acc;
    }
    const int32_t pos = block_scan_excl(counted ? 1 : 0, &tot);
    if (rpc && counted) {
      cic[rpc[I] + written + pos] = J;
      vc[rpc[I] + written + pos] = acc;
    }
    written += tot;
  }
  if (!rpc && threadIdx.x == 0) count[I] = written;
}

static void galerkin_long_rows(int32_t nc, const uint8_t* ovf, const int32_t* moff, const int32_t* mem,
                               const int32_t* agg, const int32_t* rp, const int32_t* ci, const double* av,
                               const double* d, const double* pval, bool graph_mode, const int32_t* rpc,
                               int32_t* count, int32_t* cic, double* vc, double* dc, double* dinvc,
                               GalerkinCache* cache, hipStream_t s) {
  const bool values = rpc != nullptr;  // fill pass
  if (values && cache && cache->nL >= 0) {
    // the count pass's sorted terms: the same long rows in the same order
    // (the overflow test is the same), so only the values are generated
    const int32_t nL = cache->nL;
    {
      DVec<int32_t> rows(nc), cnt(1);
      compact_i32(nullptr, ovf, rows.p, cnt.p, nc, s);
      require(read_scalar(cnt.p, s) == nL, PCAMG_EHIP, "Galerkin fill: long rows differ from the count pass");
    }
    if (nL > 0) {
      const int64_t total = cache->total;
      DVec<double> tv(total), tp(total);
      gal_terms_kernel<<<nL, LONG_BLOCK, 0, s>>>(cache->rows.p, cache->off.p, moff, mem, agg, rp, ci, av, d, pval,
                                                 graph_mode, nullptr, tv.p, tp.p);
      PCAMG_LAUNCHED();
      gal_runs_kernel<<<nL, LONG_BLOCK, 0, s>>>(cache->rows.p, cache->off.p, cache->ks.p, cache->perm.p, tv.p, tp.p,
                                                graph_mode, rpc, count, cic, vc, dc, dinvc);
      PCAMG_LAUNCHED();
      PCAMG_HIP(hipStreamSynchronize(s));
    }
    cache->nL = -1;
    return;
  }
  DVec<int32_t> rows(nc), cnt(1);
  compact_i32(nullptr, ovf, rows.p, cnt.p, nc, s);
  const int32_t nL = read_scalar(cnt.p, s);
  if (cache) {
    cache->nL = nL;
    cache->total = 0;
  }
  if (nL == 0) return;
  DVec<int32_t> lc(nL);
  gal_terms_count_kernel<<<grid_for(nL, 256), 256, 0, s>>>(nL, rows.p, moff, mem, rp, graph_mode, lc.p);
  PCAMG_LAUNCHED();
  DVec<int64_t> off(nL + 1);
  scan_exclusive_i64(lc.p, off.p, nL, s);
  int64_t total = read_scalar(off.p + (nL - 1), s) + read_scalar(lc.p + (nL - 1), s);
  require(total < ((int64_t)1 << 31), PCAMG_EUNSUPPORTED, "Galerkin product: long rows exceed 2^31 terms");
  copy_h2d(off.p + nL, &total, 1, s);
  DVec<uint64_t> keys(total), ks(total);
  DVec<double> tv(values ? total : 0), tp(values ? total : 0);
  DVec<uint32_t> idx(total), perm(total);
  gal_terms_kernel<<<nL, LONG_BLOCK, 0, s>>>(rows.p, off.p, moff, mem, agg, rp, ci, av, d, pval, graph_mode, keys.p,
                                             tv.p, tp.p);
  PCAMG_LAUNCHED();
  iota_i32((int32_t*)idx.p, total, s);
  radix_sort_u64_u32(keys.p, idx.p, ks.p, perm.p, total, s);
  gal_runs_kernel<<<nL, LONG_BLOCK, 0, s>>>(rows.p, off.p, ks.p, perm.p, tv.p, tp.p, graph_mode, rpc, count, cic, vc,
                                            dc, dinvc);
  PCAMG_LAUNCHED();
  PCAMG_HIP(hipStreamSynchronize(s));  // `total` is read by the async copy above
  if (cache && !values) {  // kept for the fill pass
    cache->total = total;
    cache->rows = std::move(rows);
    cache->off = std::move(off);
    cache->ks = std::move(ks);
    cache->perm = std::move(perm);
  }
}

int64_t galerkin_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t nc, const int32_t* moff,
                       const int32_t* mem, const int32_t* agg, int32_t* rpc, bool graph_mode, hipStream_t s,
                       GalerkinCache* cache) {
  (void)n;
  if (nc <= 0) return 0;
  DVec<int32_t> cnt(nc);
  DVec<uint8_t> ovf(nc);
  PCAMG_HIP(hipMemsetAsync(ovf.p, 0, nc, s));
  galerkin_kernel<<<grid_for(nc, GAL_WAVES), 64 * GAL_WAVES, 0, s>>>(nc, moff, mem, agg, rp, ci, nullptr, nullptr,
                                                                      nullptr, graph_mode, nullptr, cnt.p, nullptr,
                                                                      nullptr, nullptr, nullptr, ovf.p);
  PCAMG_LAUNCHED();
  galerkin_long_rows(nc, ovf.p, moff, mem, agg, rp, ci, nullptr, nullptr, nullptr, graph_mode, nullptr, cnt.p,
                     nullptr, nullptr, nullptr, nullptr, cache, s);
  DVec<int64_t> off64(nc);
  scan_exclusive_i64(cnt.p, off64.p, nc, s);
  int64_t total = read_scalar(off64.p + (nc - 1), s) + read_scalar(cnt.p + (nc - 1), s);
  require(total < INT32_MAX, PCAMG_EUNSUPPORTED, "coarse operator larger than 2^31 entries");
  scan_exclusive_i32(cnt.p, rpc, nc, rpc + nc, s);
  return total;
}

void galerkin_fill(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, const double* d, int32_t nc,
                   const int32_t* moff, const int32_t* mem, const int32_t* agg, const double* pval, const int32_t* rpc,
                   int32_t* cic, double* vc, double* dc, double* dinvc, bool graph_mode, hipStream_t s,
                   GalerkinCache* cache) {
  (void)n;
  if (nc <= 0) return;
  DVec<uint8_t> ovf(nc);
  PCAMG_HIP(hipMemsetAsync(ovf.p, 0, nc, s));
  galerkin_kernel<<<grid_for(nc, GAL_WAVES), 64 * GAL_WAVES, 0, s>>>(nc, moff, mem, agg, rp, ci, av, d, pval,
                                                                      graph_mode, rpc, nullptr, cic, vc, dc, dinvc,
                                                                      ovf.p);
  PCAMG_LAUNCHED();
  galerkin_long_rows(nc, ovf.p, moff, mem, agg, rp, ci, av, d, pval, graph_mode, rpc, nullptr, cic, vc, dc, dinvc,
                     cache, s);
}

// ---------------------------------------------------------------------------
// Path shortening (Alg. 4, Step 7).  first[I] = smallest (path, position) of a
// member of I on a path; a run of consecutive vertices of I on a path is kept
// only if it starts at first[I]; consecutive kept runs are linked.
// ---------------------------------------------------------------------------
__global__ void sh_first_kernel(int32_t n, const int32_t* __restrict__ pid, const int32_t* __restrict__ pos,
                                const int32_t* __restrict__ agg, unsigned long long* __restrict__ first) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || pid[v] < 0) return;
  unsigned long long key = ((unsigned long long)(uint32_t)pid[v] << 32) | (uint32_t)pos[v];
  atomicMin(&first[agg[v]], key);
}

__device__ int32_t cover_step(const int32_t* nb, const int32_t* pos, int32_t v, int32_t want) {
  int32_t a = nb[2 * v], b = nb[2 * v + 1];
  if (a >= 0 && pos[a] == want) return a;
  if (b >= 0 && pos[b] == want) return b;
  return -1;
}

__device__ bool run_owned(const int32_t* nb, const int32_t* pid, const int32_t* pos, const int32_t* agg,
                          const unsigned long long* first, int32_t v) {
  const int32_t I = agg[v];
  int32_t s = v;
  for (int q = 0; q < 4; ++q) {  // runs are at most 3 long
    int32_t p = pos[s] > 0 ? cover_step(nb, pos, s, pos[s] - 1) : -1;
    if (p < 0 || agg[p] != I) break;
    s = p;
  }
  unsigned long long key = ((unsigned long long)(uint32_t)pid[s] << 32) | (uint32_t)pos[s];
  return first[I] == key;
}

__global__ void sh_link_kernel(int32_t n, const int32_t* __restrict__ nb, const int32_t* __restrict__ pid,
                               const int32_t* __restrict__ pos, const int32_t* __restrict__ agg,
                               const unsigned long long* __restrict__ first, int32_t* __restrict__ nbc) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || pid[v] < 0) return;
  const int32_t w = cover_step(nb, pos, v, pos[v] + 1);
  if (w < 0) return;
  const int32_t I = agg[v], J = agg[w];
  if (I == J) return;
  if (!run_owned(nb, pid, pos, agg, first, w) || !run_owned(nb, pid, pos, agg, first, v)) return;
  nbc[2 * (size_t)I + 1] = J;  // next
  nbc[2 * (size_t)J] = I;      // previous
}

__global__ void sh_canon_kernel(int32_t nc, int32_t* __restrict__ nbc) {
  int32_t I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  if (nbc[2 * (size_t)I] < 0 && nbc[2 * (size_t)I + 1] >= 0) {
    nbc[2 * (size_t)I] = nbc[2 * (size_t)I + 1];
    nbc[2 * (size_t)I + 1] = -1;
  }
}

void shorten_paths(int32_t n, const int32_t* nb, const int32_t* path_id, const int32_t* pos, int32_t nc,
                   const int32_t* agg, int32_t* nbc, hipStream_t s) {
  fill_i32(nbc, -1, 2 * (size_t)nc, s);
  if (n <= 0 || nc <= 0) return;
  DVec<uint64_t> first(nc);
  fill_u64(first.p, ~0ull, nc, s);
  sh_first_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, path_id, pos, agg, (unsigned long long*)first.p);
  PCAMG_LAUNCHED();
  sh_link_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, nb, path_id, pos, agg, (const unsigned long long*)first.p, nbc);
  PCAMG_LAUNCHED();
  sh_canon_kernel<<<grid_for(nc, 256), 256, 0, s>>>(nc, nbc);
  PCAMG_LAUNCHED();
}

// ---------------------------------------------------------------------------
// MWM aggregation (Sec. 2.1) of a level on its weighted adjacency w = -a_ij.
// Upper entries (i < j) in row-major order are the edges in lexicographic
// index order; a stable radix sort on ~bits(w) (w > 0, so the bit pattern
// grows with w) puts them heaviest first with ties by index.  The greedy
// matching runs by deterministic reservations: a pending edge dies once an
// end is matched (a permanent fact), else it reserves both ends with its rank
// and matches them iff it holds both -- every earlier edge at those ends has
// then been decided, so this is the sequential greedy matching.  Left-over
// vertices have only matched neighbours (the matching is maximal) and join
// the aggregate of the heaviest one (ties to the smaller id): independent
// choices, one thread each.
// ---------------------------------------------------------------------------
__global__ void mwm_upper_count_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                       int32_t* __restrict__ ucnt) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t k1 = rp[i + 1];
  ucnt[i] = k1 - first_upper(i, rp[i], k1, ci);
}

__global__ void __launch_bounds__(256)
    mwm_keys_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const double* __restrict__ av, const int32_t* __restrict__ uoff, int32_t* __restrict__ eu,
                    int32_t* __restrict__ ev, uint64_t* __restrict__ ekey) {
  const int32_t i = (int32_t)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);  // uniform per wavefront
  if (i >= n) return;
  const int lane = (int)(threadIdx.x & 63);
  const int32_t k0 = rp[i], k1 = rp[i + 1];
  const int32_t fu = first_upper(i, k0, k1, ci);
  const int32_t ubase = uoff[i];
  for (int32_t k = fu + lane; k < k1; k += 64) {
    const int32_t u = ubase + (k - fu);
    eu[u] = i;
    ev[u] = ci[k];
    ekey[u] = ~(uint64_t)__double_as_longlong(-av[k]);
  }
}

__global__ void mm_reserve_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                  const int32_t* __restrict__ sv, const int32_t* __restrict__ mate,
                                  uint32_t* __restrict__ res, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  const int32_t t = win[x];
  const int32_t u = su[t], v = sv[t];
  if (mate[u] >= 0 || mate[v] >= 0) {
    state[x] = 0;
    return;
  }
  atomicMin(&res[u], (uint32_t)t);
  atomicMin(&res[v], (uint32_t)t);
  state[x] = 1;
}

__global__ void mm_commit_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                 const int32_t* __restrict__ sv, int32_t* __restrict__ mate,
                                 const uint32_t* __restrict__ res, uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w || state[x] != 1) return;
  const uint32_t t = (uint32_t)win[x];
  const int32_t u = su[t], v = sv[t];
  if (res[u] != t || res[v] != t) return;
  mate[u] = v;
  mate[v] = u;
  state[x] = 2;
}

__global__ void mm_reset_kernel(int32_t w, const int32_t* __restrict__ win, const int32_t* __restrict__ su,
                                const int32_t* __restrict__ sv, uint32_t* __restrict__ res,
                                uint8_t* __restrict__ state) {
  int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= w) return;
  const uint8_t st = state[x];
  if (st == 0) return;
  const int32_t t = win[x];
  res[su[t]] = UINT_MAX;
  res[sv[t]] = UINT_MAX;
  state[x] = st == 1 ? 1 : 0;  // keep only the still-pending edges
}

// Objects: a matched pair is named by its smaller end; a left-over vertex
// takes its heaviest neighbour's object (no neighbour: its own).
__global__ void mwm_join_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ av, const int32_t* __restrict__ mate,
                                int32_t* __restrict__ obj, int32_t* __restrict__ osz, int32_t* __restrict__ stats) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t m = mate[u];
  if (m >= 0) {
    const int32_t T = u < m ? u : m;
    obj[u] = T;
    atomicAdd(&osz[T], 1);
    return;
  }
  int32_t b = -1;
  double bw = 0.0;
  for (int32_t k = rp[u]; k < rp[u + 1]; ++k) {
    const double w = -av[k];
    if (b < 0 || w > bw) { b = ci[k]; bw = w; }
  }
  atomicAdd(&stats[0], 1);
  if (b < 0) {
    obj[u] = u;
    atomicAdd(&osz[u], 1);
    atomicAdd(&stats[2], 1);
    return;
  }
  const int32_t mb = mate[b];  // >= 0: the matching is maximal
  const int32_t T = mb < 0 ? b : (b < mb ? b : mb);
  obj[u] = T;
  atomicAdd(&osz[T], 1);
  atomicAdd(&stats[1], 1);
}

int32_t mwm_aggregate_level(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, int32_t* agg,
                            int32_t* moff, int32_t* mem, AggStats& st, hipStream_t s) {
  DVec<int32_t> ucnt(n), uoff(n), tot(1), mate(n), obj(n), osz(n), stats(3);
  mwm_upper_count_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, ucnt.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(ucnt.p, uoff.p, n, tot.p, s);
  const int32_t m = read_scalar(tot.p, s);
  fill_i32(mate.p, -1, n, s);
  if (m > 0) {
    DVec<int32_t> eu(m), ev(m), su(m), sv(m);
    DVec<uint64_t> ekey(m), ksorted(m);
    DVec<uint32_t> idx(m), order(m);
    mwm_keys_kernel<<<grid_for((size_t)n * 64, 256), 256, 0, s>>>(n, rp, ci, av, uoff.p, eu.p, ev.p, ekey.p);
    PCAMG_LAUNCHED();
    iota_i32((int32_t*)idx.p, m, s);
    radix_sort_u64_u32(ekey.p, idx.p, ksorted.p, order.p, m, s);
    sorted_endpoints(m, order.p, eu.p, ev.p, su.p, sv.p, s);
    DVec<uint32_t> res(n);
    fill_u32(res.p, UINT_MAX, n, s);
    const int32_t WIN = std::max<int32_t>(1 << 16, std::min<int32_t>(1 << 20, m / 8 + 1));
    DVec<int32_t> win(WIN), surv(WIN), cnt(1);
    DVec<uint8_t> state(WIN);
    int32_t ns = 0, next = 0, rounds = 0;
    while (ns > 0 || next < m) {
      const int32_t take = std::min<int32_t>(WIN - ns, m - next);
      if (take > 0) {
        window_kernel<<<grid_for(take, 256), 256, 0, s>>>(ns, next, take, win.p);
        PCAMG_LAUNCHED();
      }
      const int32_t w = ns + take;
      next += take;
      const unsigned g = grid_for(w, 256);
      mm_reserve_kernel<<<g, 256, 0, s>>>(w, win.p, su.p, sv.p, mate.p, res.p, state.p);
      PCAMG_LAUNCHED();
      mm_commit_kernel<<<g, 256, 0, s>>>(w, win.p, su.p, sv.p, mate.p, res.p, state.p);
      PCAMG_LAUNCHED();
      mm_reset_kernel<<<g, 256, 0, s>>>(w, win.p, su.p, sv.p, res.p, state.p);
      PCAMG_LAUNCHED();
      compact_i32(win.p, state.p, surv.p, cnt.p, w, s);
      ns = read_scalar(cnt.p, s);
      std::swap(win, surv);  // survivors first in the next window
      ++rounds;
      require(rounds <= 4 * m + 8, PCAMG_EHIP, "MWM matching did not terminate");
    }
    st.cover_rounds = rounds;
  }
  fill_i32(osz.p, 0, n, s);
  fill_i32(stats.p, 0, 3, s);
  mwm_join_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, av, mate.p, obj.p, osz.p, stats.p);
  PCAMG_LAUNCHED();
  auto hs = to_host(stats.p, 3, s);
  st.n_unagg = hs[0];
  st.case2 = hs[1];
  st.singleton = hs[2];
  return number_aggregates(n, obj.p, osz.p, agg, moff, mem, s);
}

}  // namespace pcamg
