// Laplacian, multicolouring, Gauss-Seidel passes, residual, transfers and the
// vector kernels of the outer iterations.  Floating-point sums follow a fixed
// order (fma chains in CSR order) so results are reproducible bit for bit.
#include <algorithm>

#include "internal.hpp"
#include "rowchain.hpp"

namespace pcamg {

// SplitMix64 counter stream (Steele, Lea & Flood 2014): word k of stream seed
// is mix(seed + k * 0x9E3779B97F4A7C15).
__host__ __device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64_word(uint64_t seed, uint64_t k) {
  return sm64_mix(seed + k * 0x9E3779B97F4A7C15ull);
}

// ---------------------------------------------------------------------------
// Laplacian A = D - W (Sec. 2.2): one thread per row.
// ---------------------------------------------------------------------------
__global__ void laplacian_kernel(int32_t n, const int32_t* __restrict__ rp, const double* __restrict__ w,
                                 double* __restrict__ aval, double* __restrict__ d, double* __restrict__ dinv) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    double x = w[k];
    s = s + x;
    aval[k] = -x;
  }
  d[i] = s;
  dinv[i] = 1.0 / s;
}

void laplacian(int32_t n, const int32_t* rp, const double* w, double* aval, double* d, double* dinv, size_t,
               hipStream_t s) {
  if (n <= 0) return;
  laplacian_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, w, aval, d, dinv);
  PCAMG_LAUNCHED();
}

// ---------------------------------------------------------------------------
// Jones-Plassmann colouring: a vertex is coloured in the first round in which
// all its higher-priority neighbours are coloured, with the smallest colour
// none of them has.  This equals sequential first-fit in descending
// (priority, id) order; priority = degree, then a random word (largest degree
// first takes fewer colours on the coarse operators).
// ---------------------------------------------------------------------------
// Keys of the colouring order: largest degree first (capped at 2^24 - 1, top
// 24 bits), then the top 40 bits of word (level << 32) + v + 1 of the stream.
__global__ void jp_prio_kernel(int32_t n, const int32_t* __restrict__ rp, uint64_t seed, uint64_t lvl,
                               uint64_t* __restrict__ prio) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t deg = (uint64_t)min(rp[v + 1] - rp[v], (1 << 24) - 1);
  prio[v] = (deg << 40) | (sm64_word(seed, lvl + (uint64_t)v + 1ull) >> 24);
}

// Colour v if all its higher-priority neighbours are coloured; returns true if
// v is still uncoloured afterwards.  Reading a neighbour coloured in the same
// round is harmless either way: its colour is final once written.  Neighbours
// are examined in batches of eight with independent loads.
// prio / colour may point to global memory or LDS.
template <typename PP, typename PC>
__device__ __forceinline__ bool jp_try(int32_t v, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                       PP prio, PC colour) {
  constexpr int U = 8;
  const uint64_t pv = prio[v];
  const int32_t k0 = rp[v], k1 = rp[v + 1];
  unsigned long long used = 0ull;
  for (int32_t k = k0; k < k1; k += U) {
    int32_t u[U];
    uint64_t pu[U];
    int32_t cu[U];
    // unconditional loads (past the row's end: its last entry again, then
    // skipped), so that a batch's loads issue together
#pragma unroll
    for (int j = 0; j < U; ++j) u[j] = ci[min(k + j, k1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      pu[j] = prio[u[j]];
      cu[j] = __atomic_load_n(&colour[u[j]], __ATOMIC_RELAXED);
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (k + j >= k1) continue;  // padding
      if (pu[j] > pv || (pu[j] == pv && u[j] > v)) {
        if (cu[j] < 0) return true;
        if (cu[j] < 64) used |= 1ull << cu[j];
      }
    }
  }
  int32_t c;
  if (~used != 0ull) {  // a free colour below 64 (colours above do not matter)
    c = __ffsll((long long)~used) - 1;
  } else {  // colours 0..63 all taken: the next windows of 64, one row scan each
    c = -1;
    for (int32_t base = 64; c < 0; base += 64) {
      unsigned long long win = 0ull;
      for (int32_t k = k0; k < k1; ++k) {
        const int32_t w = ci[k];
        const uint64_t pw = prio[w];
        if (pw > pv || (pw == pv && w > v)) {
          const int32_t cw = __atomic_load_n(&colour[w], __ATOMIC_RELAXED) - base;
          if (cw >= 0 && cw < 64) win |= 1ull << cw;
        }
      }
      if (~win != 0ull) c = base + __ffsll((long long)~win) - 1;
    }
  }
  __atomic_store_n(&colour[v], c, __ATOMIC_RELAXED);
  return false;
}

// All rounds in one workgroup (small graphs): priorities, colours and the
// shrinking worklist of uncoloured vertices in LDS.
constexpr int JP_SMALL_THREADS = 1024;
constexpr int32_t JP_SMALL_MAX = 4096;
__global__ void __launch_bounds__(JP_SMALL_THREADS)
    jp_small_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const uint64_t* __restrict__ prio, int32_t* colour, int32_t* __restrict__ rounds_out) {
  __shared__ uint64_t pr[JP_SMALL_MAX];
  __shared__ int32_t col[JP_SMALL_MAX];
  __shared__ int32_t wl[2][JP_SMALL_MAX];
  __shared__ int32_t cnt[2];
  for (int32_t v = threadIdx.x; v < n; v += JP_SMALL_THREADS) {
    pr[v] = prio[v];
    col[v] = -1;
    wl[0][v] = v;
  }
  if (threadIdx.x == 0) {
    cnt[0] = n;
    cnt[1] = 0;
  }
  __syncthreads();
  int cur = 0;
  int32_t rounds = 0;
  for (;;) {
    const int32_t m = cnt[cur];
    if (m == 0 || rounds > n + 1) break;
    for (int32_t t = threadIdx.x; t < m; t += JP_SMALL_THREADS) {
      const int32_t v = wl[cur][t];
      if (jp_try(v, rp, ci, (const uint64_t*)pr, (int32_t*)col)) wl[cur ^ 1][atomicAdd(&cnt[cur ^ 1], 1)] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) cnt[cur] = 0;
    cur ^= 1;
    ++rounds;
    __syncthreads();
  }
  for (int32_t v = threadIdx.x; v < n; v += JP_SMALL_THREADS) colour[v] = col[v];
  if (threadIdx.x == 0) *rounds_out = rounds;
}

// Greedy first-fit in descending (priority, id) order, one vertex at a time in
// one workgroup -- the same colouring as the Jones-Plassmann rounds (a
// vertex's already coloured neighbours are exactly its higher-priority ones).
// For near-dense levels, where the rounds degenerate to a few vertices each.
// The order is sorted beforehand (order, with each row's range k0s/k1s);
// colours live in LDS, and the first free colour comes from stamps: step t
// writes t at seen[c] for every colour c of a coloured neighbour (plain
// stores: lanes that write one slot write the same value), then the lowest c
// without the stamp is taken.  Two barriers per vertex; the row entries of
// the vertex two steps ahead are loaded during the current step.
constexpr int32_t SEQ_MAX = 20000;
constexpr int SEQ_T = 1024;
constexpr int SEQ_E = 8;  // row entries per thread loaded ahead (rows beyond SEQ_E * SEQ_T: the rest after)

__global__ void __launch_bounds__(SEQ_T)
    greedy_seq_kernel(int32_t n, int32_t nnz, const int32_t* __restrict__ ci, const int32_t* __restrict__ order,
                      const int32_t* __restrict__ k0s, const int32_t* __restrict__ k1s,
                      int32_t* __restrict__ colour) {
  __shared__ int32_t col[SEQ_MAX];
  __shared__ int32_t seen[SEQ_MAX + 1];
  __shared__ int32_t cand[SEQ_T / 64];
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int32_t i = tid; i <= n; i += SEQ_T) {
    if (i < n) col[i] = -1;
    seen[i] = -1;
  }
  __syncthreads();
  const int32_t last = nnz - 1;  // nnz > 0 on the levels taken here
  // rows of steps t, t + 1 and t + 2 in registers (the last one in flight)
  int32_t r0[SEQ_E], r1[SEQ_E], r2[SEQ_E];
  int32_t va = order[0], a0 = k0s[0], a1 = k1s[0];
  const int32_t s1 = min(1, n - 1), s2 = min(2, n - 1);
  int32_t vb = order[s1], b0 = k0s[s1], b1 = k1s[s1];
  int32_t vc = order[s2], c0 = k0s[s2], c1 = k1s[s2];
#pragma unroll
  for (int e = 0; e < SEQ_E; ++e) {
    r0[e] = ci[min(a0 + tid + e * SEQ_T, last)];
    r1[e] = ci[min(b0 + tid + e * SEQ_T, last)];
  }
  int32_t vprev = -1, cprev = -1, cmax = -1;
  for (int32_t t = 0; t < n; ++t) {
    // two steps ahead: the row of step t + 2, the vertex and range of t + 3
#pragma unroll
    for (int e = 0; e < SEQ_E; ++e) r2[e] = ci[min(c0 + tid + e * SEQ_T, last)];
    const int32_t t3 = min(t + 3, n - 1);
    const int32_t vd = order[t3], d0 = k0s[t3], d1 = k1s[t3];
    // stamp the colours of the coloured neighbours of va (the previous
    // vertex's colour may not be visible yet: taken from the register)
#pragma unroll
    for (int e = 0; e < SEQ_E; ++e) {
      if (a0 + tid + e * SEQ_T < a1) {
        const int32_t u = r0[e];
        const int32_t c = u == vprev ? cprev : col[u];
        if (c >= 0) seen[c] = t;
      }
    }
    for (int32_t k = a0 + SEQ_E * SEQ_T + tid; k < a1; k += SEQ_T) {  // rows longer than the prefetch
      const int32_t u = ci[k];
      const int32_t c = u == vprev ? cprev : col[u];
      if (c >= 0) seen[c] = t;
    }
    __syncthreads();
    // the lowest colour not stamped (cmax + 1 is always free)
    int32_t first = INT32_MAX;
    for (int32_t base = 0; base <= cmax; base += SEQ_T) {  // uniform
      const int32_t c = base + tid;
      const unsigned long long fb = __ballot(c <= cmax && seen[c] != t);
      if (fb) {
        first = base + wave * 64 + __ffsll((long long)fb) - 1;
        break;
      }
    }
    if (lane == 0) cand[wave] = first;
    __syncthreads();
    int32_t mex = cmax + 1;
#pragma unroll
    for (int w = 0; w < SEQ_T / 64; ++w) mex = min(mex, cand[w]);
    if (tid == 0) col[va] = mex;
    vprev = va;
    cprev = mex;
    cmax = max(cmax, mex);
    va = vb, a0 = b0, a1 = b1;
    vb = vc, b0 = c0, b1 = c1;
    vc = vd, c0 = d0, c1 = d1;
#pragma unroll
    for (int e = 0; e < SEQ_E; ++e) {
      r0[e] = r1[e];
      r1[e] = r2[e];
    }
  }
  __syncthreads();
  for (int32_t i = tid; i < n; i += SEQ_T) colour[i] = col[i];
}

// Sort input for greedy_seq_kernel: keys ~priority, ids in descending order,
// so that a stable ascending sort gives descending (priority, id).
__global__ void seq_keys_kernel(int32_t n, const uint64_t* __restrict__ prio, uint64_t* __restrict__ keys,
                                uint32_t* __restrict__ ids) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const int32_t v = n - 1 - i;
  keys[i] = ~prio[v];
  ids[i] = (uint32_t)v;
}

__global__ void seq_ranges_kernel(int32_t n, const int32_t* __restrict__ order, const int32_t* __restrict__ rp,
                                  int32_t* __restrict__ k0s, int32_t* __restrict__ k1s) {
  const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= n) return;
  k0s[t] = rp[order[t]];
  k1s[t] = rp[order[t] + 1];
}

__global__ void row_len_max_kernel(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ out) {
  int32_t m = 0;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    m = max(m, rp[i + 1] - rp[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// The higher-priority neighbours of every vertex (larger (priority, id)), in
// column order: the only ones its first-fit colour depends on.  A blocked
// hub then checks its few higher neighbours, not its whole row.
// Rows of more than ROW_LONG entries are left by the thread-per-row kernels
// below to a workgroup each (a power-law level's hubs have thousands).
constexpr int32_t ROW_LONG = 256;

__device__ __forceinline__ bool prio_higher(uint64_t pu, int32_t u, uint64_t pv, int32_t v) {
  return pu > pv || (pu == pv && u > v);
}

__global__ void higher_count_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const uint64_t* __restrict__ prio, int32_t* __restrict__ cnt) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || rp[v + 1] - rp[v] > ROW_LONG) return;
  const uint64_t pv = prio[v];
  int32_t c = 0;
  for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
    const int32_t u = ci[k];
    c += prio_higher(prio[u], u, pv, v);
  }
  cnt[v] = c;
}

__global__ void __launch_bounds__(256)
    higher_count_long_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                             const int32_t* __restrict__ ci, const uint64_t* __restrict__ prio,
                             int32_t* __restrict__ cnt) {
  __shared__ int32_t wsum[4];
  const int32_t v = rows[blockIdx.x];
  const uint64_t pv = prio[v];
  int32_t c = 0;
  for (int32_t k = rp[v] + (int32_t)threadIdx.x; k < rp[v + 1]; k += 256) {
    const int32_t u = ci[k];
    c += prio_higher(prio[u], u, pv, v);
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[v] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ void higher_fill_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                   const uint64_t* __restrict__ prio, const int32_t* __restrict__ hrp,
                                   int32_t* __restrict__ hci) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || rp[v + 1] - rp[v] > ROW_LONG) return;
  const uint64_t pv = prio[v];
  int32_t o = hrp[v];
  for (int32_t k = rp[v]; k < rp[v + 1]; ++k) {
    const int32_t u = ci[k];
    if (prio_higher(prio[u], u, pv, v)) hci[o++] = u;
  }
}

// The same for the long rows: 256 entries per step, kept in column order by
// a ballot prefix within each wavefront and the wavefronts' counts in LDS.
__global__ void __launch_bounds__(256)
    higher_fill_long_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ ci, const uint64_t* __restrict__ prio,
                            const int32_t* __restrict__ hrp, int32_t* __restrict__ hci) {
  __shared__ int32_t wsum[4];
  const int32_t v = rows[blockIdx.x];
  const uint64_t pv = prio[v];
  const int lane = (int)(threadIdx.x & 63), wid = (int)(threadIdx.x >> 6);
  const unsigned long long below = (1ull << lane) - 1ull;
  const int32_t k1 = rp[v + 1];
  int32_t o = hrp[v];
  for (int32_t base = rp[v]; base < k1; base += 256) {
    const int32_t k = base + (int32_t)threadIdx.x;
    int32_t u = 0;
    bool f = false;
    if (k < k1) {
      u = ci[k];
      f = prio_higher(prio[u], u, pv, v);
    }
    const unsigned long long bal = __ballot(f);
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wid ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (f) hci[o + off + __popcll(bal & below)] = u;
    o += tot;
    __syncthreads();
  }
}

// jp_try_h resuming where the vertex's last attempt stopped: cur[v] is the
// first higher-priority neighbour not yet seen coloured and usedm[v] the set
// of colours below 64 of those before it.  Colours are final once set, so the
// accumulated set equals a fresh scan, and the colour chosen is the same; a
// vertex blocked for many rounds no longer rescans its coloured prefix.
__device__ __forceinline__ bool jp_try_hc(int32_t v, const int32_t* __restrict__ hrp,
                                          const int32_t* __restrict__ hci, int32_t* colour, int32_t* __restrict__ cur,
                                          unsigned long long* __restrict__ usedm) {
  constexpr int U = 8;
  const int32_t k1 = hrp[v + 1];
  unsigned long long used = usedm[v];
  for (int32_t k = cur[v]; k < k1; k += U) {
    int32_t cu[U];
    // unconditional loads (past the list's end: its last entry again), then
    // padding made a colour that neither blocks nor takes a slot
    int32_t hj[U];
#pragma unroll
    for (int j = 0; j < U; ++j) hj[j] = hci[min(k + j, k1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j) cu[j] = __atomic_load_n(&colour[hj[j]], __ATOMIC_RELAXED);
#pragma unroll
    for (int j = 0; j < U; ++j) cu[j] = k + j < k1 ? cu[j] : INT32_MAX;
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (cu[j] < 0) {
        cur[v] = k + j;
        usedm[v] = used;
        return true;
      }
      if (cu[j] < 64) used |= 1ull << cu[j];
    }
  }
  int32_t c;
  if (~used != 0ull) {  // a free colour below 64 (colours above do not matter)
    c = __ffsll((long long)~used) - 1;
  } else {  // colours 0..63 all taken: the next windows of 64, one list scan each
    const int32_t k0 = hrp[v];
    c = -1;
    for (int32_t base = 64; c < 0; base += 64) {
      unsigned long long win = 0ull;
      for (int32_t k = k0; k < k1; ++k) {
        const int32_t cw = __atomic_load_n(&colour[hci[k]], __ATOMIC_RELAXED) - base;
        if (cw >= 0 && cw < 64) win |= 1ull << cw;
      }
      if (~win != 0ull) c = base + __ffsll((long long)~win) - 1;
    }
  }
  __atomic_store_n(&colour[v], c, __ATOMIC_RELAXED);
  return false;
}

// 64-bit words of the per-wavefront colour bitmap of jp_try_wave
constexpr int JP_BM_WORDS = 32;

// OR of a 64-bit mask over the wavefront
__device__ __forceinline__ unsigned long long wave_or64(unsigned long long m) {
  for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o, 64);
  return m;
}

// jp_try_hc for a vertex with a long higher-priority list, by the whole
// wavefront (v is uniform): 64 entries per step from the cursor, the first
// uncoloured one (if any) found by a ballot, the colours below 64 of the
// entries before it OR-ed into the mask; with every higher neighbour
// coloured, the windows of 64 colours above are scanned the same way.  The
// same cursor, mask and colour as jp_try_hc.
__device__ __forceinline__ bool jp_try_wave(int32_t v, const int32_t* __restrict__ hrp,
                                            const int32_t* __restrict__ hci, int32_t* colour,
                                            int32_t* __restrict__ cur, unsigned long long* __restrict__ usedm,
                                            unsigned long long* bm, int lane) {
  const int32_t k1 = hrp[v + 1];
  unsigned long long used = usedm[v];
  for (int32_t k = cur[v]; k < k1; k += 64) {
    const int32_t kk = k + lane;
    const int32_t cu = kk < k1 ? __atomic_load_n(&colour[hci[kk]], __ATOMIC_RELAXED) : INT32_MAX;
    const unsigned long long blk = __ballot(cu < 0);
    const int first = blk ? __ffsll((long long)blk) - 1 : 64;
    used |= wave_or64(lane < first && cu >= 0 && cu < 64 ? 1ull << cu : 0ull);
    if (blk) {
      if (lane == 0) {
        cur[v] = k + first;
        usedm[v] = used;
      }
      return true;
    }
  }
  int32_t c;
  if (~used != 0ull) {
    c = __ffsll((long long)~used) - 1;
  } else {
    // colours 64 .. 64 + 64 JP_BM_WORDS - 1 in one pass over the list: a
    // bitmap in the wavefront's LDS, then its first free bit
    const int32_t k0 = hrp[v];
    if (lane < JP_BM_WORDS) bm[lane] = 0ull;
    __builtin_amdgcn_wave_barrier();
    for (int32_t k = k0 + lane; k < k1; k += 64) {
      const int32_t cw = __atomic_load_n(&colour[hci[k]], __ATOMIC_RELAXED) - 64;
      if (cw >= 0 && cw < 64 * JP_BM_WORDS) atomicOr(&bm[cw >> 6], 1ull << (cw & 63));
    }
    __builtin_amdgcn_wave_barrier();
    const unsigned long long word = lane < JP_BM_WORDS ? bm[lane] : ~0ull;
    __builtin_amdgcn_wave_barrier();
    const unsigned long long fw = __ballot(~word != 0ull);
    if (fw) {
      const int fl = __ffsll((long long)fw) - 1;
      const unsigned long long wfl = __shfl(word, fl, 64);
      c = 64 + 64 * fl + __ffsll((long long)~wfl) - 1;
    } else {  // beyond the bitmap: windows of 64, one list scan each
      c = -1;
      for (int32_t base = 64 + 64 * JP_BM_WORDS; c < 0; base += 64) {
        unsigned long long win = 0ull;
        for (int32_t k = k0; k < k1; k += 64) {
          const int32_t kk = k + lane;
          const int32_t cw = kk < k1 ? __atomic_load_n(&colour[hci[kk]], __ATOMIC_RELAXED) - base : -1;
          win |= cw >= 0 && cw < 64 ? 1ull << cw : 0ull;
        }
        win = wave_or64(win);
        if (~win != 0ull) c = base + __ffsll((long long)~win) - 1;
      }
    }
  }
  if (lane == 0) __atomic_store_n(&colour[v], c, __ATOMIC_RELAXED);
  return false;
}

// Higher-priority lists longer than this go to jp_try_wave.
constexpr int32_t JP_LANE_MAX = 64;

// Wakes the uncoloured vertex w (a lane's entry, if `act`) for round `next`
// unless already queued for it: one atomic per wavefront step for the slots.
__device__ __forceinline__ void jp_wake_push(bool act, int32_t w, const int32_t* colour, int32_t* __restrict__ stamp,
                                             int32_t next, int32_t* __restrict__ cnt_out, int32_t* __restrict__ out,
                                             int lane) {
  const bool push = act && __atomic_load_n(&colour[w], __ATOMIC_RELAXED) < 0 && atomicMax(&stamp[w], next) < next;
  const unsigned long long pb = __ballot(push);
  if (!pb) return;
  const int lead = __ffsll((long long)pb) - 1;
  int32_t at = 0;
  if (lane == lead) at = atomicAdd(cnt_out, __popcll(pb));
  at = __shfl(at, lead, 64);
  if (push) out[at + __popcll(pb & ((1ull << lane) - 1ull))] = w;
}

// Rows longer than this are pushed by jp_push_long_kernel; rows of at most
// JP_PUSH_LANE_MAX entries by their own lane.
constexpr int32_t JP_PUSH_WAVE_MAX = 256;
// No-op stamp slots (after the n stamps) for lanes without an entry to push.
constexpr int32_t JP_SPARE = 4096;
constexpr int32_t JP_PUSH_LANE_MAX = 32;
// Worklists of at most this many vertices per wavefront of the grid are
// taken a vertex per wavefront, longer ones a vertex per lane.
constexpr int32_t JP_WAVE_MODE_PER_WAVE = 4;

// One round over the worklist of all uncoloured vertices (levels without
// hub rows: a few dozen rounds of many vertices each, where the rounds of
// jp_wake_kernel cost more in wake-ups than they save); the ones still
// uncoloured go to the next list (in any order: the colouring does not
// depend on it).
__global__ void __launch_bounds__(256)
    jp_list_kernel(const int32_t* __restrict__ cnt_in, const int32_t* __restrict__ in, int32_t* __restrict__ cnt_out,
                   int32_t* __restrict__ out, const int32_t* __restrict__ hrp, const int32_t* __restrict__ hci,
                   int32_t* colour, int32_t* __restrict__ cur, unsigned long long* __restrict__ usedm) {
  const int32_t m = *cnt_in;
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t base = blockIdx.x * blockDim.x; base < m; base += stride) {
    const int32_t t = base + threadIdx.x;
    const int32_t v = t < m ? in[t] : -1;
    const bool left =
        v >= 0 && __atomic_load_n(&colour[v], __ATOMIC_RELAXED) < 0 && jp_try_hc(v, hrp, hci, colour, cur, usedm);
    const unsigned long long bal = __ballot(left);
    if (!bal) continue;
    const int lane = threadIdx.x & 63;
    const int lead = __ffsll((long long)bal) - 1;
    int32_t at = 0;
    if (lane == lead) at = atomicAdd(cnt_out, __popcll(bal));
    at = __shfl(at, lead, 64);
    if (left) out[at + __popcll(bal & ((1ull << lane) - 1ull))] = v;
  }
}

// One data-driven round: try the vertices of the worklist; every vertex that
// takes its colour here wakes its uncoloured neighbours (all of lower
// priority) for round `next`, each at most once per round (stamp[w] = the
// last round it was queued for).  A vertex that stays blocked waits on an
// uncoloured higher neighbour, which wakes it when coloured, so a round costs
// the vertices around the previous round's colours, not the whole pending
// set (on a power-law level the hub core needs about a thousand rounds of a
// few dozen vertices each).  The colouring is the same function of the
// priorities whatever the schedule.  A wavefront pushes the rows of its newly
// coloured vertices one at a time, 64 entries per step, and lists the ones
// with rows of more than JP_PUSH_WAVE_MAX entries for jp_push_long_kernel;
// vertices with more than JP_LANE_MAX higher-priority neighbours are tried
// by the wavefront too, and a short worklist is taken a vertex per wavefront.
__global__ void __launch_bounds__(256)
    jp_wake_kernel(const int32_t* __restrict__ cnt_in, const int32_t* __restrict__ in, int32_t* __restrict__ cnt_out,
                   int32_t* __restrict__ out, const int32_t* __restrict__ rbase, int32_t r1,
                   const int32_t* __restrict__ rp,
                   const int32_t* __restrict__ ci, const int32_t* __restrict__ hrp, const int32_t* __restrict__ hci,
                   int32_t* colour, int32_t* __restrict__ cur, unsigned long long* __restrict__ usedm,
                   int32_t* __restrict__ stamp, int32_t* __restrict__ spare, int32_t* __restrict__ cnt_hubs,
                   int32_t* __restrict__ hubs) {
  __shared__ unsigned long long bms[4][JP_BM_WORDS];
  const int32_t m = *cnt_in;
  const int32_t next = *rbase + r1;  // the round being filled
  // the stamp atomic of a lane without an entry to push: a no-op on a slot
  // of its own, so that the atomics of a batch issue unconditionally (an
  // atomic under a condition waits for its result before the next issues)
  int32_t* const idle = spare + ((blockIdx.x * blockDim.x + threadIdx.x) & (JP_SPARE - 1));
  const int lane = (int)(threadIdx.x & 63);
  unsigned long long* bm = bms[threadIdx.x >> 6];
  // the wavefront pushes the row of u, or lists it as a hub
  // (at most JP_PUSH_WAVE_MAX / 64 steps of 64 entries, all their loads and
  // stamps in flight together, one append for the row)
  auto wake_row = [&](int32_t u) {
    const int32_t k0 = rp[u], k1 = rp[u + 1];
    if (k1 - k0 > JP_PUSH_WAVE_MAX) {
      if (lane == 0) hubs[atomicAdd(cnt_hubs, 1)] = u;
      return;
    }
    if (k1 <= k0) return;
    constexpr int Q = JP_PUSH_WAVE_MAX / 64;
    int32_t w[Q], cw[Q], old[Q];
    bool act[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      act[q] = k0 + q * 64 + lane < k1;
      w[q] = ci[min(k0 + q * 64 + lane, k1 - 1)];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) cw[q] = __atomic_load_n(&colour[w[q]], __ATOMIC_RELAXED);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      act[q] = act[q] && cw[q] < 0;
      old[q] = atomicMax(act[q] ? &stamp[w[q]] : idle, act[q] ? next : INT32_MIN);
    }
    unsigned long long pb[Q];
    int32_t tot = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pb[q] = __ballot(act[q] && old[q] < next);
      tot += __popcll(pb[q]);
    }
    if (!tot) return;
    int32_t at = 0;
    if (lane == 0) at = atomicAdd(cnt_out, tot);
    at = __shfl(at, 0, 64);
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (pb[q] >> lane & 1ull) out[at + __popcll(pb[q] & below)] = w[q];
      at += __popcll(pb[q]);
    }
  };
  const int32_t nwaves = (int32_t)gridDim.x * 4;
  if (m <= JP_WAVE_MODE_PER_WAVE * nwaves) {
    // short lists: a wavefront per listed vertex, so that the vertices with
    // long lists are not queued behind each other in a few wavefronts
    for (int32_t t = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6); t < m; t += nwaves) {
      const int32_t v = in[t];
      if (__atomic_load_n(&colour[v], __ATOMIC_RELAXED) >= 0) continue;
      if (!jp_try_wave(v, hrp, hci, colour, cur, usedm, bm, lane)) wake_row(v);
    }
    return;
  }
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t base = blockIdx.x * blockDim.x; base < m; base += stride) {  // uniform per workgroup
    const int32_t t = base + (int32_t)threadIdx.x;
    const int32_t v = t < m ? in[t] : -1;
    const bool open = v >= 0 && __atomic_load_n(&colour[v], __ATOMIC_RELAXED) < 0;
    const bool wide = open && hrp[v + 1] - hrp[v] > JP_LANE_MAX;
    bool now = open && !wide && !jp_try_hc(v, hrp, hci, colour, cur, usedm);
    // long higher-priority lists: the wavefront tries them one at a time
    unsigned long long wb = __ballot(wide);
    while (wb) {
      const int j = __ffsll((long long)wb) - 1;
      wb &= wb - 1ull;
      const bool got = !jp_try_wave(__shfl(v, j, 64), hrp, hci, colour, cur, usedm, bm, lane);
      if (lane == j) now = got;
    }
    // short rows: each lane pushes its own row, four entries per step (their
    // colour loads and stamp atomics in flight together, one append for
    // the four); the others a row at a time by the wavefront (or as hubs)
    const int32_t pk0 = now ? rp[v] : 0;
    const int32_t plen = now ? rp[v + 1] - pk0 : 0;
    const bool mine = now && plen <= JP_PUSH_LANE_MAX;
    const int32_t span = wave_max_len(mine ? plen : 0);
    for (int32_t j = 0; j < span; j += 4) {
      int32_t w[4];
      bool act[4];
      // unconditional loads (past the row's end, and for lanes without a row
      // of their own: an entry of the row, or entry 0, again), then masked
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        act[u] = mine && j + u < plen;
        w[u] = ci[pk0 + max(0, min(j + u, plen - 1))];
      }
      int32_t cw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cw[u] = __atomic_load_n(&colour[w[u]], __ATOMIC_RELAXED);
#pragma unroll
      for (int u = 0; u < 4; ++u) act[u] = act[u] && cw[u] < 0;
      int32_t old[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) old[u] = atomicMax(act[u] ? &stamp[w[u]] : idle, act[u] ? next : INT32_MIN);
      unsigned long long pb[4];
      int32_t tot = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pb[u] = __ballot(act[u] && old[u] < next);
        tot += __popcll(pb[u]);
      }
      if (!tot) continue;
      int32_t at = 0;
      if (lane == 0) at = atomicAdd(cnt_out, tot);
      at = __shfl(at, 0, 64);
      const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (pb[u] >> lane & 1ull) out[at + __popcll(pb[u] & below)] = w[u];
        at += __popcll(pb[u]);
      }
    }
    unsigned long long bal = __ballot(now && !mine);
    while (bal) {
      const int j = __ffsll((long long)bal) - 1;
      bal &= bal - 1ull;
      wake_row(__shfl(v, j, 64));
    }
  }
}

// The rows of the vertices with long rows coloured in this round (hubs), each
// spread over the blocks of one grid row (gridDim.x blocks of 256 entries at
// a time), the vertices over the grid rows.
__global__ void __launch_bounds__(256)
    jp_push_long_kernel(const int32_t* __restrict__ cnt_hubs, const int32_t* __restrict__ hubs,
                        const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, const int32_t* colour,
                        int32_t* __restrict__ stamp, const int32_t* __restrict__ rbase, int32_t r1,
                        int32_t* __restrict__ cnt_out, int32_t* __restrict__ out) {
  const int32_t m = *cnt_hubs;
  const int32_t next = *rbase + r1;
  const int lane = (int)(threadIdx.x & 63);
  for (int32_t h = (int32_t)blockIdx.y; h < m; h += (int32_t)gridDim.y) {
    const int32_t u = hubs[h];
    const int32_t k0 = rp[u], k1 = rp[u + 1];
    for (int32_t base = k0 + (int32_t)blockIdx.x * 256; base < k1; base += (int32_t)gridDim.x * 256) {
      const int32_t k = base + (int32_t)threadIdx.x;
      jp_wake_push(k < k1, k < k1 ? ci[k] : 0, colour, stamp, next, cnt_out, out, lane);
    }
  }
}

// counts of the next batch: cnt[0] = cnt[last], the others zero
// The same for a batch of data-driven rounds: also advances the round base
// and clears the hub counts of the batch.
__global__ void jp_wake_carry_kernel(int32_t* cnt, int32_t last, int32_t* rbase, int32_t* cnt_hubs) {
  const int32_t c = cnt[last];
  __syncthreads();
  for (int32_t i = threadIdx.x; i <= last; i += blockDim.x) cnt[i] = i == 0 ? c : 0;
  for (int32_t i = threadIdx.x; i < last; i += blockDim.x) cnt_hubs[i] = 0;
  if (threadIdx.x == 0) *rbase += last;
}

__global__ void jp_carry_kernel(int32_t* cnt, int32_t last) {
  const int32_t c = cnt[last];
  __syncthreads();
  for (int32_t i = threadIdx.x; i <= last; i += blockDim.x) cnt[i] = i == 0 ? c : 0;
}

__global__ void min_i32_kernel(const int32_t* a, int32_t n, int32_t* out) {
  int32_t m = INT32_MAX;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = min(m, a[i]);
  for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(out, m);
}

__global__ void max_i32_kernel(const int32_t* a, int32_t n, int32_t* out) {
  int32_t m = -1;
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = max(m, a[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Mean row length above which levels are coloured one vertex at a time.
constexpr int64_t JP_SEQ_DEG = 48;
// Fewest threads a data-driven colouring round is launched with (8192
// wavefronts: worklists of up to 32768 vertices go a vertex per wavefront),
// and the grid of its hub pushes (blocks per row x rows at a time).
constexpr int32_t WAKE_MIN_THREADS = 1 << 19;
constexpr unsigned PUSH_GRID_X = 16, PUSH_GRID_Y = 64;

// A non-blocking stream of this host thread for capturing launch sequences
// (capture is not allowed on the legacy stream); kept for the thread's life.
hipStream_t capture_stream() {
  thread_local hipStream_t cs = nullptr;
  if (!cs) PCAMG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  return cs;
}

// An instantiated graph, destroyed with its scope.
struct GraphExec {
  hipGraphExec_t e = nullptr;
  GraphExec() = default;
  GraphExec(const GraphExec&) = delete;
  GraphExec& operator=(const GraphExec&) = delete;
  ~GraphExec() {
    if (e) (void)hipGraphExecDestroy(e);
  }
};

int32_t max_row_len(int32_t n, const int32_t* rp, hipStream_t s) {
  DVec<int32_t> mx(1);
  fill_i32(mx.p, 0, 1, s);
  row_len_max_kernel<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(n, rp, mx.p);
  PCAMG_LAUNCHED();
  return read_scalar(mx.p, s);
}

int32_t colour_jp(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level, int32_t* colour,
                  hipStream_t s) {
  if (n <= 0) return 0;
  fill_i32(colour, -1, n, s);
  const uint64_t lvl = (uint64_t)(uint32_t)level << 32;
  DVec<uint64_t> prio(n);
  jp_prio_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, seed, lvl, prio.p);
  PCAMG_LAUNCHED();
  const int64_t nnz = n > 0 ? (int64_t)read_scalar(rp + n, s) : 0;
  // small near-dense levels (more than JP_SEQ_DEG entries per row, at most
  // SEQ_MAX vertices): the priority chains are about as long as the level,
  // so colour one vertex at a time in one workgroup, from LDS.  Other levels:
  // data-driven rounds (below), or the one-workgroup rounds when small.
  const bool dense_rows = nnz > JP_SEQ_DEG * (int64_t)n;
  if (dense_rows && n <= SEQ_MAX) {
    DVec<uint64_t> keys(n), skeys(n);
    DVec<uint32_t> ids(n);
    DVec<int32_t> order(n), k0s(n), k1s(n);
    seq_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, prio.p, keys.p, ids.p);
    PCAMG_LAUNCHED();
    radix_sort_u64_u32(keys.p, ids.p, skeys.p, (uint32_t*)order.p, n, s);
    seq_ranges_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, order.p, rp, k0s.p, k1s.p);
    PCAMG_LAUNCHED();
    greedy_seq_kernel<<<1, SEQ_T, 0, s>>>(n, (int32_t)nnz, ci, order.p, k0s.p, k1s.p, colour);
    PCAMG_LAUNCHED();
  } else if (n <= JP_SMALL_MAX) {
    DVec<int32_t> rounds(1);
    jp_small_kernel<<<1, JP_SMALL_THREADS, 0, s>>>(n, rp, ci, prio.p, colour, rounds.p);
    PCAMG_LAUNCHED();
  } else {
    // data-driven rounds (jp_wake_kernel) in batches of R; the host reads
    // the worklist size after each batch.  The highest-priority uncoloured
    // vertex is always on the current list (its last higher neighbour to be
    // coloured woke it for the next round), so every round colours a vertex
    // until the list is empty, and at most n rounds are run.
    constexpr int R = 16;
    DVec<int32_t> hcnt(n), hrp(n + 1), lrows;
    const int32_t nl = rows_longer_than(n, rp, nullptr, ROW_LONG, lrows, s);
    higher_count_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, prio.p, hcnt.p);
    PCAMG_LAUNCHED();
    if (nl > 0) {
      higher_count_long_kernel<<<nl, 256, 0, s>>>(lrows.p, rp, ci, prio.p, hcnt.p);
      PCAMG_LAUNCHED();
    }
    scan_exclusive_i32(hcnt.p, hrp.p, n, hrp.p + n, s);
    const int32_t htot = read_scalar(hrp.p + n, s);  // nnz / 2 on a symmetric pattern
    DVec<int32_t> hci(std::max<int32_t>(htot, 1));
    higher_fill_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, prio.p, hrp.p, hci.p);
    PCAMG_LAUNCHED();
    if (nl > 0) {
      higher_fill_long_kernel<<<nl, 256, 0, s>>>(lrows.p, rp, ci, prio.p, hrp.p, hci.p);
      PCAMG_LAUNCHED();
    }
    DVec<int32_t> list0(n), list1(n), cnt(R + 1), cur(n), stamp((size_t)n + JP_SPARE), hubs(n), cnt_hubs(R);
    DVec<uint64_t> usedm(n);
    copy_d2d(cur.p, hrp.p, n, s);
    fill_u64(usedm.p, 0ull, n, s);
    fill_i32(stamp.p, 0, (size_t)n + JP_SPARE, s);
    fill_i32(cnt_hubs.p, 0, R, s);
    iota_i32(list0.p, n, s);
    fill_i32(cnt.p, 0, R + 1, s);
    fill_i32(cnt.p, n, 1, s);
    int32_t pending = n;  // worklist size at the start of the next batch
    int64_t rounds = 0;
    if (nl == 0) {
      // no hub rows: rounds over all pending vertices in batches of RL (RL is
      // even: the survivors are in list0 after each batch), one captured
      // graph replayed per batch as below
      constexpr int RL = 8;
      const unsigned grid = std::min<unsigned>(grid_for(n, 256), 2048);
      GraphExec ge;
      {
        hipStream_t cs = capture_stream();
        PCAMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
          for (int r = 0; r < RL; ++r) {
            const int32_t* in = (r & 1) ? list1.p : list0.p;
            int32_t* out = (r & 1) ? list0.p : list1.p;
            jp_list_kernel<<<grid, 256, 0, cs>>>(cnt.p + r, in, cnt.p + r + 1, out, hrp.p, hci.p, colour, cur.p,
                                                 (unsigned long long*)usedm.p);
            PCAMG_LAUNCHED();
          }
          jp_carry_kernel<<<1, 64, 0, cs>>>(cnt.p, RL);
          PCAMG_LAUNCHED();
        } catch (...) {
          hipGraph_t tmp = nullptr;
          (void)hipStreamEndCapture(cs, &tmp);
          if (tmp) (void)hipGraphDestroy(tmp);
          throw;
        }
        hipGraph_t g = nullptr;
        PCAMG_HIP(hipStreamEndCapture(cs, &g));
        const hipError_t err = hipGraphInstantiate(&ge.e, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        PCAMG_HIP(err);
      }
      for (;;) {
        PCAMG_HIP(hipGraphLaunch(ge.e, s));
        rounds += RL;
        pending = read_scalar(cnt.p, s);
        if (pending == 0) break;
        require(rounds <= (int64_t)n + RL, PCAMG_EHIP, "colouring made no progress");
      }
    }
    if (pending > 0) {
      // a batch of R rounds (each a wake and a hub-push launch) and the carry
      // is captured once and replayed until the worklist is empty: the
      // launches of a graph cost less than stream launches, and the round
      // numbers come from a device counter.  Lists grow and shrink within a
      // batch: a grid of at least WAKE_MIN_THREADS threads, grid-stride loops
      // beyond it.
      DVec<int32_t> rbase(1);
      fill_i32(rbase.p, 0, 1, s);
      const unsigned grid = std::min<unsigned>(grid_for(std::max<int32_t>(n, WAKE_MIN_THREADS), 256), 2048);
      GraphExec ge;
      {
        hipStream_t cs = capture_stream();
        PCAMG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
          for (int r = 0; r < R; ++r) {
            const int32_t* in = (r & 1) ? list1.p : list0.p;
            int32_t* out = (r & 1) ? list0.p : list1.p;
            jp_wake_kernel<<<grid, 256, 0, cs>>>(cnt.p + r, in, cnt.p + r + 1, out, rbase.p, r + 1, rp, ci, hrp.p,
                                                 hci.p, colour, cur.p, (unsigned long long*)usedm.p, stamp.p,
                                                 stamp.p + n, cnt_hubs.p + r, hubs.p);
            PCAMG_LAUNCHED();
            jp_push_long_kernel<<<dim3(PUSH_GRID_X, PUSH_GRID_Y), 256, 0, cs>>>(
                cnt_hubs.p + r, hubs.p, rp, ci, colour, stamp.p, rbase.p, r + 1, cnt.p + r + 1, out);
            PCAMG_LAUNCHED();
          }
          jp_wake_carry_kernel<<<1, 64, 0, cs>>>(cnt.p, R, rbase.p, cnt_hubs.p);
          PCAMG_LAUNCHED();
        } catch (...) {
          hipGraph_t tmp = nullptr;
          (void)hipStreamEndCapture(cs, &tmp);
          if (tmp) (void)hipGraphDestroy(tmp);
          throw;
        }
        hipGraph_t g = nullptr;
        PCAMG_HIP(hipStreamEndCapture(cs, &g));
        const hipError_t err = hipGraphInstantiate(&ge.e, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        PCAMG_HIP(err);
      }
      for (;;) {
        PCAMG_HIP(hipGraphLaunch(ge.e, s));
        rounds += R;
        pending = read_scalar(cnt.p, s);  // R is even: that list is in list0 again
        if (pending == 0) break;
        require(rounds <= (int64_t)n + R, PCAMG_EHIP, "colouring made no progress");
      }
    }
  }
  DVec<int32_t> mx(1);
  fill_i32(mx.p, -1, 1, s);
  max_i32_kernel<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(colour, n, mx.p);
  PCAMG_LAUNCHED();
  const int32_t nc = read_scalar(mx.p, s) + 1;
  // every vertex must be coloured: the smallest colour is then 0, and -1 never appears
  DVec<int32_t> mn(1);
  fill_i32(mn.p, 1, 1, s);
  min_i32_kernel<<<std::min<unsigned>(grid_for(n, 256), 1024), 256, 0, s>>>(colour, n, mn.p);
  PCAMG_LAUNCHED();
  require(read_scalar(mn.p, s) >= 0, PCAMG_EHIP, "colouring left a vertex uncoloured");
  return nc;
}

// ---------------------------------------------------------------------------
// Red-black colouring of a connected bipartite graph: colour = parity of the
// breadth-first depth from vertex 0.  Breadth-first search in frontier rounds;
// round d expands the vertices of depth d, claiming unvisited neighbours for
// depth d + 1 with a compare-and-swap (the frontier order is irrelevant).  An
// edge between two vertices of depth d closes an odd cycle: every such edge is
// seen while depth d is expanded, so the graph is bipartite exactly when no
// round sees one.
// ---------------------------------------------------------------------------
// Neighbour u of a vertex of depth d: an odd cycle if u has depth d too, a
// claim for depth d + 1 if unvisited (depths below d + 1 were set by earlier
// rounds); the claimed vertices go to the next frontier, one atomic per
// wavefront step.
__device__ __forceinline__ void bfs_visit(bool act, int32_t u, int32_t* depth, int32_t d, bool& odd,
                                          int32_t* __restrict__ cnt_out, int32_t* __restrict__ out, int lane) {
  bool claim = false;
  if (act) {
    const int32_t du = depth[u];
    if (du == d) odd = true;
    else if (du < 0) claim = atomicCAS(&depth[u], -1, d + 1) == -1;
  }
  const unsigned long long bal = __ballot(claim);
  if (!bal) return;
  const int first = __ffsll((long long)bal) - 1;
  int32_t at = 0;
  if (lane == first) at = atomicAdd(cnt_out, __popcll(bal));
  at = __shfl(at, first, 64);
  if (claim) out[at + __popcll(bal & ((1ull << lane) - 1ull))] = u;
}

// One round.  Short frontiers (at most BFS_WAVE_MODE_PER_WAVE vertices per
// wavefront of the grid) go a vertex per wavefront, its row 64 entries per
// step; longer ones a vertex per lane for rows of at most 64 entries, the
// longer rows then by the whole wavefront, one at a time (a hub would
// otherwise hold its wavefront for its whole row, one entry per step).  An
// odd cycle is published as soon as a wavefront sees one, and every
// wavefront stops at its next vertex once it is.
constexpr int32_t BFS_WAVE_MODE_PER_WAVE = 4;

__global__ void __launch_bounds__(256)
    bfs_round_kernel(const int32_t* __restrict__ cnt_in, const int32_t* __restrict__ in, int32_t* __restrict__ cnt_out,
                     int32_t* __restrict__ out, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                     int32_t* depth, int32_t d, int32_t* odd_flag) {
  const int32_t m = *cnt_in;
  const int lane = threadIdx.x & 63;
  bool odd = false;
  // publishes this wavefront's odd cycle; true once any wavefront has one
  auto stop = [&]() -> bool {
    if (__ballot(odd)) {
      if (lane == 0) __atomic_store_n(odd_flag, 1, __ATOMIC_RELAXED);
      return true;
    }
    return __builtin_amdgcn_readfirstlane(__atomic_load_n(odd_flag, __ATOMIC_RELAXED)) != 0;
  };
  const int32_t nwaves = (int32_t)gridDim.x * 4;
  if (m <= BFS_WAVE_MODE_PER_WAVE * nwaves) {
    for (int32_t t = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6); t < m; t += nwaves) {
      if (stop()) return;
      const int32_t v = in[t];
      const int32_t a = rp[v], e = rp[v + 1];
      for (int32_t k = a; k < e; k += 64) {
        const bool on = k + lane < e;
        bfs_visit(on, on ? ci[k + lane] : 0, depth, d, odd, cnt_out, out, lane);
      }
    }
    stop();
    return;
  }
  const int32_t stride = gridDim.x * blockDim.x;
  for (int32_t base = blockIdx.x * blockDim.x; base < m; base += stride) {
    if (stop()) return;
    const int32_t t = base + threadIdx.x;
    const bool act = t < m;
    const int32_t v = act ? in[t] : 0;
    const int32_t k0 = act ? rp[v] : 0;
    const int32_t len = act ? rp[v + 1] - k0 : 0;
    const bool longrow = len > 64;
    const int32_t span = wave_max_len(longrow ? 0 : len);
    for (int32_t j = 0; j < span; ++j) {
      const bool on = !longrow && j < len;
      bfs_visit(on, on ? ci[k0 + j] : 0, depth, d, odd, cnt_out, out, lane);
    }
    unsigned long long lb = __ballot(longrow);
    while (lb) {
      const int src = __ffsll((long long)lb) - 1;
      lb &= lb - 1ull;
      const int32_t a = __shfl(k0, src, 64), e = a + __shfl(len, src, 64);
      for (int32_t k = a; k < e; k += 64) {
        const bool on = k + lane < e;
        bfs_visit(on, on ? ci[k + lane] : 0, depth, d, odd, cnt_out, out, lane);
      }
    }
  }
  stop();
}

__global__ void parity_kernel(int32_t n, const int32_t* __restrict__ depth, int32_t* __restrict__ colour) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) colour[v] = depth[v] & 1;
}

bool colour_bipartite(int32_t n, const int32_t* rp, const int32_t* ci, int32_t* colour, hipStream_t s) {
  if (n <= 0) return false;
  // st[0..RMAX]: frontier sizes of the rounds of one batch; st[RMAX + 1]: odd cycle seen
  constexpr int RMAX = 16;
  DVec<int32_t> depth(n), list0(n), list1(n), st(RMAX + 2);
  fill_i32(depth.p, -1, n, s);
  fill_i32(depth.p, 0, 1, s);
  fill_i32(list0.p, 0, 1, s);
  fill_i32(st.p, 0, RMAX + 2, s);
  fill_i32(st.p, 1, 1, s);
  const unsigned grid = std::min<unsigned>(grid_for(n, 256), 2048);
  int64_t reached = 1;
  int32_t d = 0;
  // batches of R rounds (R even, non-decreasing: the frontier is in list0 after
  // each batch and counters beyond R are still zero); the first batches are
  // short so that a non-bipartite graph is rejected after few rounds
  for (int R = 2;; R = std::min(2 * R, RMAX)) {
    for (int r = 0; r < R; ++r, ++d) {
      const int32_t* in = (r & 1) ? list1.p : list0.p;
      int32_t* out = (r & 1) ? list0.p : list1.p;
      bfs_round_kernel<<<grid, 256, 0, s>>>(st.p + r, in, st.p + r + 1, out, rp, ci, depth.p, d, st.p + RMAX + 1);
      PCAMG_LAUNCHED();
    }
    const std::vector<int32_t> h = to_host(st.p, RMAX + 2, s);
    if (h[RMAX + 1]) return false;
    for (int r = 1; r <= R; ++r) reached += h[r];
    if (h[R] == 0) break;
    require(d <= n + RMAX, PCAMG_EHIP, "breadth-first search made no progress");
    jp_carry_kernel<<<1, 64, 0, s>>>(st.p, R);
    PCAMG_LAUNCHED();
  }
  if (reached != n) return false;
  parity_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, depth.p, colour);
  PCAMG_LAUNCHED();
  return true;
}

int32_t colour_level(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level, int32_t* colour,
                     hipStream_t s) {
  if (colour_bipartite(n, rp, ci, colour, s)) return n > 1 ? 2 : 1;
  return colour_jp(n, rp, ci, seed, level, colour, s);
}

// ---------------------------------------------------------------------------
// Gauss-Seidel pass over the rows of one colour (rows row0..row1-1 of a
// colour-sorted matrix): s = sum_j a_ij x_j as an fma chain in CSR order,
// x_i = (b_i - s) * dinv_i.  Rows of one colour are independent.  G lanes per
// row (G = 1: one thread per row); the row sums come from rowchain.hpp.
// ---------------------------------------------------------------------------
template <typename T, int G>
__global__ void __launch_bounds__(256)
    gs_kernel(int32_t row0, int32_t row1, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
              const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x) {
  const int32_t i = row0 + (int32_t)((xcd_block() * blockDim.x + threadIdx.x) / G);
  if constexpr (G == 1) {
    if (i >= row1) return;
    const T s = row_chain1<T>(rp[i], rp[i + 1], ci, av, x, (T)0);
    x[i] = (b[i] - s) * dinv[i];
  } else {
    const bool ok = i < row1;
    const int32_t k0 = ok ? rp[i] : 0;
    const int32_t len = ok ? rp[i + 1] - k0 : 0;
    const T s = row_chain_g<T, G>(k0, len, ci, av, x, (T)0);
    if (ok && (threadIdx.x & (G - 1)) == 0) x[i] = (b[i] - s) * dinv[i];
  }
}

// rows per launch of lanes-per-row G: the grid covers (row1 - row0) * G threads
template <typename T, int G>
void gs_launch(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av, const T* dinv,
               const T* b, T* x, hipStream_t s) {
  gs_kernel<T, G><<<grid_for((size_t)(row1 - row0) * G, 256), 256, 0, s>>>(row0, row1, rp, ci, av, dinv, b, x);
  PCAMG_LAUNCHED();
}

template <typename T>
void gs_colour(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av, const T* dinv,
               const T* b, T* x, hipStream_t s, int lanes) {
  if (row1 <= row0) return;
  switch (lanes) {
    case 1: gs_launch<T, 1>(row0, row1, rp, ci, av, dinv, b, x, s); break;
    case 4: gs_launch<T, 4>(row0, row1, rp, ci, av, dinv, b, x, s); break;
    case 16: gs_launch<T, 16>(row0, row1, rp, ci, av, dinv, b, x, s); break;
    case 64: gs_launch<T, 64>(row0, row1, rp, ci, av, dinv, b, x, s); break;
    default: throw Error(PCAMG_EINVAL, "lanes per row must be 1, 4, 16 or 64");
  }
}

// Same on the sliced-ELL copy of the matrix (one thread per row).
template <typename T>
__global__ void __launch_bounds__(256)
    gs_sell_kernel(int32_t row0, int32_t row1, const int32_t* __restrict__ rp, const int32_t* __restrict__ woff,
                   const int32_t* __restrict__ sci, const T* __restrict__ sav, const T* __restrict__ dinv,
                   const T* __restrict__ b, T* __restrict__ x) {
  const int32_t i = row0 + (int32_t)(xcd_block() * blockDim.x + threadIdx.x);
  if (i >= row1) return;
  const T s = sell_chain<T>(64 * woff[i >> 6] + (i & 63), rp[i + 1] - rp[i], sci, sav, x, (T)0);
  x[i] = (b[i] - s) * dinv[i];
}

template <typename T>
void gs_colour_sell(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* woff, const int32_t* sci,
                    const T* sav, const T* dinv, const T* b, T* x, hipStream_t s) {
  if (row1 <= row0) return;
  gs_sell_kernel<T><<<grid_for(row1 - row0, 256), 256, 0, s>>>(row0, row1, rp, woff, sci, sav, dinv, b, x);
  PCAMG_LAUNCHED();
}

// Same over an explicit row list (natural-order stage entry point).
template <typename T>
__global__ void gs_rows_kernel(int32_t nrows, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, const T* __restrict__ av, const T* __restrict__ dinv,
                               const T* __restrict__ b, T* __restrict__ x) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  int32_t i = rows[t];
  const T s = row_chain1<T>(rp[i], rp[i + 1], ci, av, x, (T)0);
  x[i] = (b[i] - s) * dinv[i];
}

template <typename T>
void gs_colour_rows(int32_t nrows, const int32_t* rows, const int32_t* rp, const int32_t* ci, const T* av,
                    const T* dinv, const T* b, T* x, hipStream_t s) {
  if (nrows <= 0) return;
  gs_rows_kernel<T><<<grid_for(nrows, 256), 256, 0, s>>>(nrows, rows, rp, ci, av, dinv, b, x);
  PCAMG_LAUNCHED();
}

// y = A x (off-diagonal entries in CSR order after s = d_i x_i); with b, the
// residual r = b - A x.
// long_min > 0: rows of long_min entries or more are left to the long-row
// kernel (skipped here, so they do not hold up their wavefront).
template <typename T, int G>
__global__ void __launch_bounds__(256)
    residual_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const T* __restrict__ av, const T* __restrict__ d, const T* __restrict__ b,
                    const T* __restrict__ x, T* __restrict__ r, int32_t long_min) {
  const int32_t i = (int32_t)((xcd_block() * blockDim.x + threadIdx.x) / G);
  if constexpr (G == 1) {
    if (i >= n) return;
    const int32_t k0 = rp[i], k1 = rp[i + 1];
    if (long_min > 0 && k1 - k0 >= long_min) return;
    const T s = row_chain1<T>(k0, k1, ci, av, x, d[i] * x[i]);
    r[i] = b ? b[i] - s : s;
  } else {
    bool ok = i < n;
    const int32_t k0 = ok ? rp[i] : 0;
    int32_t len = ok ? rp[i + 1] - k0 : 0;
    if (long_min > 0 && len >= long_min) {
      ok = false;
      len = 0;
    }
    const T s = row_chain_g<T, G>(k0, len, ci, av, x, ok ? d[i] * x[i] : (T)0);
    if (ok && (threadIdx.x & (G - 1)) == 0) r[i] = b ? b[i] - s : s;
  }
}

template <typename T, int G>
void residual_launch(int32_t n, const int32_t* rp, const int32_t* ci, const T* av, const T* d, const T* b,
                     const T* x, T* r, int32_t long_min, hipStream_t s) {
  residual_kernel<T, G><<<grid_for((size_t)n * G, 256), 256, 0, s>>>(n, rp, ci, av, d, b, x, r, long_min);
  PCAMG_LAUNCHED();
}

template <typename T>
void residual(int32_t n, const int32_t* rp, const int32_t* ci, const T* av, const T* d, const T* b, const T* x,
              T* r, hipStream_t s, int lanes, int32_t long_min) {
  if (n <= 0) return;
  switch (lanes) {
    case 1: residual_launch<T, 1>(n, rp, ci, av, d, b, x, r, long_min, s); break;
    case 4: residual_launch<T, 4>(n, rp, ci, av, d, b, x, r, long_min, s); break;
    case 16: residual_launch<T, 16>(n, rp, ci, av, d, b, x, r, long_min, s); break;
    case 64: residual_launch<T, 64>(n, rp, ci, av, d, b, x, r, long_min, s); break;
    default: throw Error(PCAMG_EINVAL, "lanes per row must be 1, 4, 16 or 64");
  }
}

// ---------------------------------------------------------------------------
// Long rows (hubs of power-law graphs): one workgroup per row.  Thread t takes
// entries t, t + 256, t + 512, ... of the row in a chain of its own, the 64
// chains of a wavefront are added by a butterfly (every lane ends with the
// same bits: IEEE addition commutes), and the four wavefront sums in order.
// Deterministic, but a different summation order from the single chain of
// shorter rows.  A thread's entries are loaded LONG_U at a time, all of them
// together (past the row's end: its last entry again, never added), so a
// row of up to LONG_U * 256 entries costs one round of index loads and one
// of gathers instead of one per few entries.
// ---------------------------------------------------------------------------
constexpr int LONG_T = 256;
constexpr int LONG_U = 8;

template <typename T>
__device__ __forceinline__ T long_row_sum(int32_t k0, int32_t k1, const int32_t* __restrict__ ci,
                                          const T* __restrict__ av, const T* __restrict__ x) {
  __shared__ T part[LONG_T / 64];
  T s = (T)0;
  const int32_t last = k1 - 1;
  for (int32_t k = k0 + (int32_t)threadIdx.x; k < k1; k += LONG_U * LONG_T) {
    int32_t c[LONG_U];
    T a[LONG_U], v[LONG_U];
#pragma unroll
    for (int u = 0; u < LONG_U; ++u) {
      const int32_t kk = min(k + u * LONG_T, last);
      c[u] = ci[kk];
      a[u] = av[kk];
    }
#pragma unroll
    for (int u = 0; u < LONG_U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < LONG_U; ++u)
      if (k + u * LONG_T < k1) s = fma(a[u], v[u], s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  T t = part[0];
#pragma unroll
  for (int w = 1; w < LONG_T / 64; ++w) t += part[w];
  return t;
}

template <typename T>
__global__ void __launch_bounds__(LONG_T)
    gs_long_kernel(int32_t row0, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                   const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b, T* x) {
  const int32_t i = row0 + (int32_t)blockIdx.x;
  const T s = long_row_sum<T>(rp[i], rp[i + 1], ci, av, x);
  if (threadIdx.x == 0) x[i] = (b[i] - s) * dinv[i];
}

// Long rows by the single fma chain in stored order (the relaxation before a
// build, which must give the chain's bits), one wavefront per row.  Spreading
// a chain over the lanes costs several whole-wavefront instructions per entry
// (the broadcasts of a_k and x_k lane by lane, then the fma); here the
// wavefront stages CHAIN_STAGE entries, each with its gathered x value, in
// LDS with coalesced loads, and lane 0 runs the chain from there -- one paired
// LDS read and one fma per entry -- while the next stage's loads are in
// flight.  The same fma chain, so the same value as row_chain_g.
constexpr int CHAIN_STAGE = 512;
template <typename T>
struct ChainPair {
  T a, v;
};

template <typename T>
__global__ void __launch_bounds__(64)
    gs_chain_long_kernel(int32_t row0, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                         const T* __restrict__ av, const T* __restrict__ dinv, const T* __restrict__ b, T* x) {
  constexpr int P = CHAIN_STAGE / 64;
  __shared__ ChainPair<T> st[CHAIN_STAGE];
  const int lane = (int)threadIdx.x;
  const int32_t i = row0 + (int32_t)blockIdx.x;
  const int32_t k0 = rp[i], k1 = rp[i + 1];  // a long row: not empty
  T a[P], v[P];
  // unconditional loads (past the row's end: its last entry again, never
  // read by the chain), so that a stage's loads issue together
  auto fetch = [&](int32_t base) {
    int32_t c[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int32_t k = min(base + u * 64 + lane, k1 - 1);
      c[u] = ci[k];
      a[u] = av[k];
    }
#pragma unroll
    for (int u = 0; u < P; ++u) v[u] = x[c[u]];
  };
  T s = (T)0;
  fetch(k0);
  for (int32_t base = k0; base < k1; base += CHAIN_STAGE) {  // uniform
#pragma unroll
    for (int u = 0; u < P; ++u) st[u * 64 + lane] = ChainPair<T>{a[u], v[u]};
    __syncthreads();
    const int32_t n = min(CHAIN_STAGE, k1 - base);
    if (base + CHAIN_STAGE < k1) fetch(base + CHAIN_STAGE);
    if (lane == 0) {
#pragma unroll 8
      for (int32_t e = 0; e < n; ++e) {
        const ChainPair<T> q = st[e];
        s = fma(q.a, q.v, s);
      }
    }
    __syncthreads();
  }
  if (lane == 0) x[i] = (b[i] - s) * dinv[i];
}

template <typename T>
void gs_colour_chain_long(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av,
                          const T* dinv, const T* b, T* x, hipStream_t s) {
  if (row1 <= row0) return;
  gs_chain_long_kernel<T><<<row1 - row0, 64, 0, s>>>(row0, rp, ci, av, dinv, b, x);
  PCAMG_LAUNCHED();
}

// One colour's rows in one launch: the first rl - row0 (XCD-ordered) blocks
// take the long rows [row0, rl), a block each, as gs_long_kernel; the other
// blocks the rows [rl, row1) with G lanes each, as gs_kernel -- the same
// arithmetic as the two launches, so the same values.
template <typename T, int G>
__global__ void __launch_bounds__(256)
    gs_fused_kernel(int32_t row0, int32_t rl, int32_t row1, const int32_t* __restrict__ rp,
                    const int32_t* __restrict__ ci, const T* __restrict__ av, const T* __restrict__ dinv,
                    const T* __restrict__ b, T* x) {
  static_assert(LONG_T == 256, "a long row takes one block of 256 threads");
  const int32_t vb = (int32_t)xcd_block(), nlong = rl - row0;
  if (vb < nlong) {  // uniform per block
    const int32_t i = row0 + vb;
    const T s = long_row_sum<T>(rp[i], rp[i + 1], ci, av, x);
    if (threadIdx.x == 0) x[i] = (b[i] - s) * dinv[i];
    return;
  }
  const int32_t i = rl + (int32_t)(((vb - nlong) * 256 + (int32_t)threadIdx.x) / G);
  const bool ok = i < row1;
  const int32_t k0 = ok ? rp[i] : 0;
  const int32_t len = ok ? rp[i + 1] - k0 : 0;
  const T s = row_chain_g<T, G>(k0, len, ci, av, x, (T)0);
  if (ok && (threadIdx.x & (G - 1)) == 0) x[i] = (b[i] - s) * dinv[i];
}

template <typename T>
void gs_colour_fused(int32_t row0, int32_t rl, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av,
                     const T* dinv, const T* b, T* x, hipStream_t s, int lanes) {
  if (row1 <= row0) return;
  if (rl >= row1) {
    gs_colour_long<T>(row0, row1, rp, ci, av, dinv, b, x, s);
    return;
  }
  if (rl <= row0 || lanes < 4) {
    gs_colour_long<T>(row0, rl, rp, ci, av, dinv, b, x, s);
    gs_colour<T>(rl, row1, rp, ci, av, dinv, b, x, s, lanes);
    return;
  }
  const unsigned grid = (unsigned)(rl - row0) + grid_for((size_t)(row1 - rl) * lanes, 256);
  switch (lanes) {
    case 4: gs_fused_kernel<T, 4><<<grid, 256, 0, s>>>(row0, rl, row1, rp, ci, av, dinv, b, x); break;
    case 16: gs_fused_kernel<T, 16><<<grid, 256, 0, s>>>(row0, rl, row1, rp, ci, av, dinv, b, x); break;
    case 64: gs_fused_kernel<T, 64><<<grid, 256, 0, s>>>(row0, rl, row1, rp, ci, av, dinv, b, x); break;
    default: throw Error(PCAMG_EINVAL, "lanes per row must be 1, 4, 16 or 64");
  }
  PCAMG_LAUNCHED();
}

template <typename T>
__global__ void __launch_bounds__(LONG_T)
    residual_long_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ ci, const T* __restrict__ av, const T* __restrict__ d,
                         const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ r) {
  const int32_t i = rows[blockIdx.x];
  const T t = long_row_sum<T>(rp[i], rp[i + 1], ci, av, x);
  if (threadIdx.x == 0) {
    const T s = d[i] * x[i] + t;
    r[i] = b ? b[i] - s : s;
  }
}

// ---------------------------------------------------------------------------
// All colour passes of one sweep of a level in a single workgroup (levels
// with many colours of a few rows each -- the near-dense coarse levels of
// power-law graphs -- where a launch per colour costs more than the colour's
// work).  Four groups of LONG_T threads; in colour c the long rows
// [coff[c], lend[c]) go to the groups in turn, each summed with exactly the
// tree of gs_long_kernel (a group's chains, a butterfly per wavefront, the
// group's four wavefront sums in order), and the other rows [lend[c],
// coff[c+1]) are single fma chains in stored order, a wavefront each (its
// lanes load the entries, as gs_kernel's lane groups do) -- so every value is
// bit-identical to the launch-per-colour path.
// A workgroup barrier separates dependent colours.
// ---------------------------------------------------------------------------
constexpr int SWEEP_GROUPS = 4;

template <typename T>
__global__ void __launch_bounds__(LONG_T * SWEEP_GROUPS)
    gs_sweep_block_kernel(int32_t c0, int32_t c1, int32_t step, const int32_t* __restrict__ coff,
                          const int32_t* __restrict__ lend, const int32_t* __restrict__ rp,
                          const int32_t* __restrict__ ci, const T* __restrict__ av, const T* __restrict__ dinv,
                          const T* __restrict__ b, T* x) {
  __shared__ T part[SWEEP_GROUPS][LONG_T / 64];
  const int tid = (int)threadIdx.x, grp = tid / LONG_T, gt = tid % LONG_T;
  for (int32_t c = c0; c != c1; c += step) {
    const int32_t r0 = coff[c], rl = lend[c], r1 = coff[c + 1];
    // long rows, SWEEP_GROUPS at a time (every group takes part in the barriers)
    for (int32_t base = r0; base < rl; base += SWEEP_GROUPS) {
      const int32_t i = base + grp;
      T sum = (T)0;
      if (i < rl) {
        constexpr int U = 4;
        const int32_t k0 = rp[i], k1 = rp[i + 1];
        int32_t k = k0 + gt;
        for (; k + (U - 1) * LONG_T < k1; k += U * LONG_T) {
          int32_t cc[U];
          T a[U], v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            cc[u] = ci[k + u * LONG_T];
            a[u] = av[k + u * LONG_T];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) v[u] = x[cc[u]];
#pragma unroll
          for (int u = 0; u < U; ++u) sum = fma(a[u], v[u], sum);
        }
        for (; k < k1; k += LONG_T) sum = fma(av[k], x[ci[k]], sum);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if ((gt & 63) == 0) part[grp][gt >> 6] = sum;
      }
      __syncthreads();
      if (i < rl && gt == 0) {
        T t = part[grp][0];
#pragma unroll
        for (int w = 1; w < LONG_T / 64; ++w) t += part[grp][w];
        x[i] = (b[i] - t) * dinv[i];
      }
      __syncthreads();
    }
    // the other rows: one wavefront each, its lanes loading the entries and
    // all of them running the row's single chain in stored order
    const int wave = tid >> 6;
    for (int32_t i0 = rl; i0 < r1; i0 += (LONG_T * SWEEP_GROUPS) / 64) {
      const int32_t i = i0 + wave;  // uniform per wavefront
      const bool ok = i < r1;
      const int32_t k0 = ok ? rp[i] : 0;
      const T sum = row_chain_g<T, 64>(k0, ok ? rp[i + 1] - k0 : 0, ci, av, x, (T)0);
      if (ok && (tid & 63) == 0) x[i] = (b[i] - sum) * dinv[i];
    }
    __syncthreads();
  }
}

template <typename T>
void gs_sweep_block(int32_t c_first, int32_t c_end, int32_t step, const int32_t* coff_d, const int32_t* lend_d,
                    const int32_t* rp, const int32_t* ci, const T* av, const T* dinv, const T* b, T* x,
                    hipStream_t s) {
  if (c_first == c_end) return;
  gs_sweep_block_kernel<T><<<1, LONG_T * SWEEP_GROUPS, 0, s>>>(c_first, c_end, step, coff_d, lend_d, rp, ci, av,
                                                                dinv, b, x);
  PCAMG_LAUNCHED();
}

template <typename T>
void gs_colour_long(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av, const T* dinv,
                    const T* b, T* x, hipStream_t s) {
  if (row1 <= row0) return;
  gs_long_kernel<T><<<row1 - row0, LONG_T, 0, s>>>(row0, rp, ci, av, dinv, b, x);
  PCAMG_LAUNCHED();
}

template <typename T>
void residual_long(int32_t nrows, const int32_t* rows, const int32_t* rp, const int32_t* ci, const T* av,
                   const T* d, const T* b, const T* x, T* r, hipStream_t s) {
  if (nrows <= 0) return;
  residual_long_kernel<T><<<nrows, LONG_T, 0, s>>>(rows, rp, ci, av, d, b, x, r);
  PCAMG_LAUNCHED();
}

template <typename T>
void spmv(int32_t n, const int32_t* rp, const int32_t* ci, const T* av, const T* d, const T* x, T* y,
          hipStream_t s, int lanes) {
  residual<T>(n, rp, ci, av, d, nullptr, x, y, s, lanes, 0);
}

// Residual (b != nullptr) or product on the sliced-ELL copy.
template <typename T>
__global__ void __launch_bounds__(256)
    residual_sell_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ woff,
                         const int32_t* __restrict__ sci, const T* __restrict__ sav, const T* __restrict__ d,
                         const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ r) {
  const int32_t i = (int32_t)(xcd_block() * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const T s = sell_chain<T>(64 * woff[i >> 6] + (i & 63), rp[i + 1] - rp[i], sci, sav, x, d[i] * x[i]);
  r[i] = b ? b[i] - s : s;
}

template <typename T>
void residual_sell(int32_t n, const int32_t* rp, const int32_t* woff, const int32_t* sci, const T* sav, const T* d,
                   const T* b, const T* x, T* r, hipStream_t s) {
  if (n <= 0) return;
  residual_sell_kernel<T><<<grid_for(n, 256), 256, 0, s>>>(n, rp, woff, sci, sav, d, b, x, r);
  PCAMG_LAUNCHED();
}

// ---------------------------------------------------------------------------
// Sliced-ELL copy (SELL-64) of a level matrix with short rows: slice q holds
// rows 64q .. 64q + 63, entry j of row 64q + l at 64 woff[q] + 64 j + l, each
// slice padded to its longest row (woff = exclusive sum of the slice widths;
// padding slots are never read).  With CSR rows of a few entries a
// wavefront's load of one entry per row spreads over a dozen cache lines;
// here it is one contiguous segment.  Entries keep their CSR order.
// ---------------------------------------------------------------------------
__global__ void sell_width_kernel(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ width) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;  // blockDim a multiple of 64: wave = slice
  const int32_t w = wave_max_len(i < n ? rp[i + 1] - rp[i] : 0);
  if ((threadIdx.x & 63) == 0 && i < n) width[i >> 6] = w;
}

__global__ void sell_fill_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ av, const float* __restrict__ av32,
                                 const int32_t* __restrict__ woff, int32_t* __restrict__ sci,
                                 double* __restrict__ sav, float* __restrict__ sav32) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t base = 64 * woff[i >> 6] + (i & 63);
  const int32_t k0 = rp[i], len = rp[i + 1] - k0;
  for (int32_t j = 0; j < len; ++j) {
    sci[base + 64 * j] = ci[k0 + j];
    sav[base + 64 * j] = av[k0 + j];
    sav32[base + 64 * j] = av32[k0 + j];
  }
}

bool sell_build(int32_t n, int32_t nnz, const int32_t* rp, const int32_t* ci, const double* av, const float* av32,
                DVec<int32_t>& woff, DVec<int32_t>& sci, DVec<double>& sav, DVec<float>& sav32, hipStream_t s) {
  if (n <= 0 || nnz <= 0) return false;
  const int32_t ns = (n + 63) / 64;
  DVec<int32_t> width(ns), total(1);
  sell_width_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, width.p);
  PCAMG_LAUNCHED();
  // a slice's width is at most the sum of its rows' lengths: the total fits int32
  woff.resize(ns);
  scan_exclusive_i32(width.p, woff.p, ns, total.p, s);
  const int64_t padded = 64ll * read_scalar(total.p, s);
  if (padded > 2ll * nnz || padded > (int64_t)INT32_MAX) {
    woff.resize(0);
    return false;
  }
  sci.resize(padded);
  sav.resize(padded);
  sav32.resize(padded);
  sell_fill_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, av, av32, woff.p, sci.p, sav.p, sav32.p);
  PCAMG_LAUNCHED();
  return true;
}

// ---------------------------------------------------------------------------
// Padded-row (ELL) copy of a level with lane groups: row i's entries at
// i*W + 0 .. i*W + len-1, the slots up to W padded with column i and value 0
// (never in a chain; they keep the speculative loads in bounds).  The pass
// loads a row's entries and its length together, so only the gathers of x
// wait on a load: two memory round trips per row instead of three (row
// pointer, then entries, then x).  The chain is the CSR one: entries in
// stored order, fma by fma.
// ---------------------------------------------------------------------------
__global__ void ell_fill_kernel(int32_t n, int32_t W, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const float* __restrict__ av32, int32_t* __restrict__ eci, float* __restrict__ eav) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t k0 = rp[i], len = rp[i + 1] - k0;
  const size_t o = (size_t)i * W;
  for (int32_t j = 0; j < W; ++j) {
    eci[o + j] = j < len ? ci[k0 + j] : i;
    eav[o + j] = j < len ? av32[k0 + j] : 0.0f;
  }
}

template <int G, int UT>
__global__ void __launch_bounds__(256)
    gs_ell_kernel(int32_t row0, int32_t row1, int32_t W, const int32_t* __restrict__ rp,
                  const int32_t* __restrict__ eci, const float* __restrict__ eav, const float* __restrict__ dinv,
                  const float* __restrict__ b, float* __restrict__ x) {
  const int32_t i = row0 + (int32_t)((xcd_block() * blockDim.x + threadIdx.x) / G);
  const bool ok = i < row1;
  const int32_t ii = ok ? i : row0;  // a valid row for the loads of idle lanes
  const int q = (int)(threadIdx.x & (G - 1));
  // unconditional loads (ii is a valid row), so that none waits in a branch
  const int32_t p0 = rp[ii], p1 = rp[ii + 1];
  const float bi = b[ii], di = dinv[ii];  // issued with the row's loads, not after its chain
  const size_t base = (size_t)ii * W;
  int32_t c[UT];
  float a[UT], v[UT];
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int32_t kk = min(u * G + q, W - 1);  // beyond the width: never in the chain
    c[u] = eci[base + kk];
    a[u] = eav[base + kk];
  }
#pragma unroll
  for (int u = 0; u < UT; ++u) v[u] = x[c[u]];
  // the chain up to the wavefront's longest row (the row pointers were
  // loaded with the entries, so this waits on nothing new)
  const int32_t len = ok ? p1 - p0 : 0;
  const int32_t span = wave_max_len(len);
  float s = 0.0f;
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int32_t e = u * G;
    if (e >= span) break;  // wave-uniform
    if constexpr (G == 4) {
      const float a0 = quad_bcast<0>(a[u]), v0 = quad_bcast<0>(v[u]);
      const float a1 = quad_bcast<1>(a[u]), v1 = quad_bcast<1>(v[u]);
      const float a2 = quad_bcast<2>(a[u]), v2 = quad_bcast<2>(v[u]);
      const float a3 = quad_bcast<3>(a[u]), v3 = quad_bcast<3>(v[u]);
      if (e + 0 < len) s = fma(a0, v0, s);
      if (e + 1 < len) s = fma(a1, v1, s);
      if (e + 2 < len) s = fma(a2, v2, s);
      if (e + 3 < len) s = fma(a3, v3, s);
    } else {
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const float at = __shfl(a[u], t, G);
        const float vt = __shfl(v[u], t, G);
        if (e + t < len) s = fma(at, vt, s);
      }
    }
  }
  if (ok && q == 0) x[i] = (bi - s) * di;
}

int32_t ell_slots(int32_t W, int lanes) {
  const int32_t per = (W + lanes - 1) / lanes;  // entries per lane
  for (int32_t ut : {2, 4, 8, 16})
    if (per <= ut && (lanes == 4 || ut <= 8)) return ut;
  return 0;
}

bool ell_build(int32_t n, int32_t lanes, const int32_t* rp, const int32_t* ci, const float* av32, int32_t& W,
               DVec<int32_t>& eci, DVec<float>& eav, hipStream_t s) {
  if (n <= 0 || (lanes != 4 && lanes != 16)) return false;
  W = max_row_len(n, rp, s);
  if (W <= 0 || ell_slots(W, lanes) == 0) {
    W = 0;
    return false;
  }
  eci.resize((size_t)n * W);
  eav.resize((size_t)n * W);
  ell_fill_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, W, rp, ci, av32, eci.p, eav.p);
  PCAMG_LAUNCHED();
  return true;
}

template <int G, int UT>
void gs_ell_launch(int32_t row0, int32_t row1, int32_t W, const int32_t* rp, const int32_t* eci, const float* eav,
                   const float* dinv, const float* b, float* x, hipStream_t s) {
  gs_ell_kernel<G, UT><<<grid_for((size_t)(row1 - row0) * G, 256), 256, 0, s>>>(row0, row1, W, rp, eci, eav, dinv,
                                                                                b, x);
  PCAMG_LAUNCHED();
}

void gs_colour_ell(int32_t row0, int32_t row1, int32_t W, int lanes, const int32_t* rp, const int32_t* eci,
                   const float* eav, const float* dinv, const float* b, float* x, hipStream_t s) {
  if (row1 <= row0) return;
  const int32_t ut = ell_slots(W, lanes);
  if (lanes == 16 && ut == 2) gs_ell_launch<16, 2>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 16 && ut == 4) gs_ell_launch<16, 4>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 16 && ut == 8) gs_ell_launch<16, 8>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 4 && ut == 2) gs_ell_launch<4, 2>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 4 && ut == 4) gs_ell_launch<4, 4>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 4 && ut == 8) gs_ell_launch<4, 8>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else if (lanes == 4 && ut == 16) gs_ell_launch<4, 16>(row0, row1, W, rp, eci, eav, dinv, b, x, s);
  else throw Error(PCAMG_EINVAL, "padded-row copy: unsupported width");
}

// Restriction b_c = P^T r: fma chain over the members of each aggregate in
// ascending (natural) order.  pval == nullptr: boolean P.  With xc, the
// coarse x is started too: mode 1 zero; mode 2 the coarse level's first
// Gauss-Seidel pass from x = 0 for its colour-0 rows (q < c1), xc = bc * dinvc
// -- from x = 0 that pass's row chains are +0 (each product a signed zero).
template <typename T>
__global__ void restrict_kernel(int32_t nc, const int32_t* __restrict__ moff, const int32_t* __restrict__ mem,
                                const T* __restrict__ pval, const T* __restrict__ r, T* __restrict__ bc,
                                T* __restrict__ xc, const T* __restrict__ dinvc, int32_t c1, int mode) {
  int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  T s = 0;
  for (int32_t t = moff[q]; t < moff[q + 1]; ++t) {
    int32_t k = mem[t];
    s = fma(pval ? pval[k] : (T)1, r[k], s);
  }
  bc[q] = s;
  if (mode == 1) xc[q] = 0;
  else if (mode == 2) xc[q] = q < c1 ? s * dinvc[q] : (T)0;
}

template <typename T>
void restrict_members(int32_t nc, const int32_t* moff, const int32_t* mem, const T* pval, const T* r, T* bc,
                      hipStream_t s, T* xc, const T* dinvc, int32_t c1, int mode) {
  if (nc <= 0) return;
  restrict_kernel<T><<<grid_for(nc, 256), 256, 0, s>>>(nc, moff, mem, pval, r, bc, xc, dinvc, c1, xc ? mode : 0);
  PCAMG_LAUNCHED();
}

// Prolongation x_k += p_k x_c[agg_k].
template <typename T>
__global__ void prolong_kernel(int32_t n, const int32_t* __restrict__ agg, const T* __restrict__ pval,
                               const T* __restrict__ xc, T* __restrict__ x) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  x[k] = fma(pval ? pval[k] : (T)1, xc[agg[k]], x[k]);
}

template <typename T>
void prolong_add(int32_t n, const int32_t* agg, const T* pval, const T* xc, T* x, hipStream_t s) {
  if (n <= 0) return;
  prolong_kernel<T><<<grid_for(n, 256), 256, 0, s>>>(n, agg, pval, xc, x);
  PCAMG_LAUNCHED();
}

#define INSTANTIATE(T)                                                                                          \
  template void gs_colour<T>(int32_t, int32_t, const int32_t*, const int32_t*, const T*, const T*, const T*,   \
                             T*, hipStream_t, int);                                                             \
  template void gs_colour_rows<T>(int32_t, const int32_t*, const int32_t*, const int32_t*, const T*, const T*, \
                                  const T*, T*, hipStream_t);                                                   \
  template void residual<T>(int32_t, const int32_t*, const int32_t*, const T*, const T*, const T*, const T*,   \
                            T*, hipStream_t, int, int32_t);                                                     \
  template void gs_colour_long<T>(int32_t, int32_t, const int32_t*, const int32_t*, const T*, const T*,        \
                                  const T*, T*, hipStream_t);                                                   \
  template void gs_colour_fused<T>(int32_t, int32_t, int32_t, const int32_t*, const int32_t*, const T*,        \
                                   const T*, const T*, T*, hipStream_t, int);                                   \
  template void gs_colour_chain_long<T>(int32_t, int32_t, const int32_t*, const int32_t*, const T*, const T*,  \
                                        const T*, T*, hipStream_t);                                             \
  template void gs_sweep_block<T>(int32_t, int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*,   \
                                  const int32_t*, const T*, const T*, const T*, T*, hipStream_t);               \
  template void residual_long<T>(int32_t, const int32_t*, const int32_t*, const int32_t*, const T*, const T*,  \
                                 const T*, const T*, T*, hipStream_t);                                          \
  template void spmv<T>(int32_t, const int32_t*, const int32_t*, const T*, const T*, const T*, T*, hipStream_t, \
                        int);                                                                                   \
  template void gs_colour_sell<T>(int32_t, int32_t, const int32_t*, const int32_t*, const int32_t*, const T*,  \
                                  const T*, const T*, T*, hipStream_t);                                         \
  template void residual_sell<T>(int32_t, const int32_t*, const int32_t*, const int32_t*, const T*, const T*,  \
                                 const T*, const T*, T*, hipStream_t);                                          \
  template void restrict_members<T>(int32_t, const int32_t*, const int32_t*, const T*, const T*, T*,          \
                                    hipStream_t, T*, const T*, int32_t, int);                                   \
  template void prolong_add<T>(int32_t, const int32_t*, const T*, const T*, T*, hipStream_t);
INSTANTIATE(double)
INSTANTIATE(float)
#undef INSTANTIATE

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------
__global__ void axpy_kernel(double a, const double* __restrict__ x, double* __restrict__ y, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], y[i]);
}
void axpy_f64(double a, const double* x, double* y, size_t n, hipStream_t s) {
  if (!n) return;
  axpy_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, x, y, n);
  PCAMG_LAUNCHED();
}

__global__ void axpy_dev_kernel(const double* __restrict__ a, int sign, const double* __restrict__ x,
                                double* __restrict__ y, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double al = sign < 0 ? -*a : *a;
  if (i < n) y[i] = fma(al, x[i], y[i]);
}
void axpy_dev_f64(const double* a, int sign, const double* x, double* y, size_t n, hipStream_t s) {
  if (!n) return;
  axpy_dev_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, sign, x, y, n);
  PCAMG_LAUNCHED();
}

__global__ void xpby_kernel(const double* __restrict__ z, const double* __restrict__ beta, double* __restrict__ p,
                            size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = fma(*beta, p[i], z[i]);
}
void xpby_dev_f64(const double* z, const double* beta, double* p, size_t n, hipStream_t s) {
  if (!n) return;
  xpby_kernel<<<grid_for(n, 256), 256, 0, s>>>(z, beta, p, n);
  PCAMG_LAUNCHED();
}

__global__ void sub_mean_kernel(double* __restrict__ x, const double* __restrict__ sum, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double mu = *sum / (double)n;
  if (i < n) x[i] = x[i] - mu;
}
void sub_mean_f64(double* x, const double* sum, size_t n, hipStream_t s) {
  if (!n) return;
  sub_mean_kernel<<<grid_for(n, 256), 256, 0, s>>>(x, sum, n);
  PCAMG_LAUNCHED();
}

template <typename T>
__global__ void gather_kernel(const T* __restrict__ src, const int32_t* __restrict__ idx, T* __restrict__ dst,
                              size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}
template <typename T>
__global__ void scatter_kernel(const T* __restrict__ src, const int32_t* __restrict__ idx, T* __restrict__ dst,
                               size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[idx[i]] = src[i];
}
void gather_f64(const double* src, const int32_t* idx, double* dst, size_t n, hipStream_t s) {
  if (!n) return;
  gather_kernel<double><<<grid_for(n, 256), 256, 0, s>>>(src, idx, dst, n);
  PCAMG_LAUNCHED();
}
void scatter_f64(const double* src, const int32_t* idx, double* dst, size_t n, hipStream_t s) {
  if (!n) return;
  scatter_kernel<double><<<grid_for(n, 256), 256, 0, s>>>(src, idx, dst, n);
  PCAMG_LAUNCHED();
}
void gather_f32(const float* src, const int32_t* idx, float* dst, size_t n, hipStream_t s) {
  if (!n) return;
  gather_kernel<float><<<grid_for(n, 256), 256, 0, s>>>(src, idx, dst, n);
  PCAMG_LAUNCHED();
}
void scatter_f32(const float* src, const int32_t* idx, float* dst, size_t n, hipStream_t s) {
  if (!n) return;
  scatter_kernel<float><<<grid_for(n, 256), 256, 0, s>>>(src, idx, dst, n);
  PCAMG_LAUNCHED();
}
void gather_i32(const int32_t* src, const int32_t* idx, int32_t* dst, size_t n, hipStream_t s) {
  if (!n) return;
  gather_kernel<int32_t><<<grid_for(n, 256), 256, 0, s>>>(src, idx, dst, n);
  PCAMG_LAUNCHED();
}

__global__ void cast_d2f_kernel(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void cast_f2d_kernel(const float* __restrict__ a, double* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}
void cast_f64_f32(const double* a, float* b, size_t n, hipStream_t s) {
  if (!n) return;
  cast_d2f_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, b, n);
  PCAMG_LAUNCHED();
}
void cast_f32_f64(const float* a, double* b, size_t n, hipStream_t s) {
  if (!n) return;
  cast_f2d_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, b, n);
  PCAMG_LAUNCHED();
}

// Start vector of build r: xi_i = 2u - 1, u = top 53 bits of word
// (r << 32) + i + 1 times 2^-53; out[p] = xi_{perm[p]} (perm may be null).
__global__ void xi_kernel(uint64_t seed, uint64_t rbase, const int32_t* __restrict__ perm, double* __restrict__ out,
                          size_t n) {
  size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint64_t i = perm ? (uint64_t)(uint32_t)perm[p] : (uint64_t)p;
  uint64_t w = sm64_word(seed, rbase + i + 1ull);
  double u = (double)(w >> 11) * 0x1.0p-53;
  out[p] = 2.0 * u - 1.0;
}
void xi_fill(uint64_t seed, int32_t r, const int32_t* perm, double* out, size_t n, hipStream_t s) {
  if (!n) return;
  xi_kernel<<<grid_for(n, 256), 256, 0, s>>>(seed, (uint64_t)(uint32_t)r << 32, perm, out, n);
  PCAMG_LAUNCHED();
}

__global__ void sub_kernel(const double* a, const double* b, double* o, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] - b[i];
}
void sub_f64(const double* a, const double* b, double* out, size_t n, hipStream_t s) {
  if (!n) return;
  sub_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, b, out, n);
  PCAMG_LAUNCHED();
}

// out = z . (rn - r), deterministic
void zsub_dot_f64(const double* z, const double* rn, const double* r, size_t n, double* out, hipStream_t s) {
  DVec<double> t(n);
  sub_f64(rn, r, t.p, n, s);
  dot_f64(z, t.p, n, out, s);
}

}  // namespace pcamg
