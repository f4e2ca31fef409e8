// Fills, prefix sums, deterministic reductions, compaction and a stable LSD
// radix sort for gfx950 (wave64).
#include <algorithm>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace pcamg {

// ---------------------------------------------------------------------------
// Device memory cache.  Blocks are bucketed to 1/16-octave sizes and kept for
// reuse.  A freed block is tagged with the stream the freeing thread works on
// (StreamScope): work enqueued on that stream may still use it, so it is
// handed out again only on the same stream, where later work is ordered after
// that use.  Blocks of a stream the caller has synchronised return to a
// shared pool (dev_cache_idle).
// ---------------------------------------------------------------------------
namespace {
std::mutex g_mem_mu;
const hipStream_t kIdle = reinterpret_cast<hipStream_t>(~uintptr_t(0));
std::multimap<std::pair<hipStream_t, size_t>, void*> g_free;
std::map<void*, size_t> g_size;
thread_local hipStream_t tl_stream = nullptr;

size_t bucket(size_t bytes) {
  if (bytes <= 4096) return 4096;
  size_t p = 1;
  while (p < bytes) p <<= 1;
  size_t step = p / 16;
  return (bytes + step - 1) / step * step;
}
}  // namespace

StreamScope::StreamScope(hipStream_t s) : prev(tl_stream) { tl_stream = s; }
StreamScope::~StreamScope() { tl_stream = prev; }

void* dev_alloc(size_t bytes) {
  size_t b = bucket(bytes);
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    for (hipStream_t tag : {tl_stream, kIdle}) {
      auto it = g_free.find({tag, b});
      if (it != g_free.end()) {
        void* p = it->second;
        g_free.erase(it);
        return p;
      }
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    dev_cache_release();
    e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(PCAMG_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
    }
  }
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_size[p] = b;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_size.find(p);
  if (it == g_size.end()) return;
  g_free.insert({{tl_stream, it->second}, p});
}

void dev_cache_idle(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  for (auto it = g_free.begin(); it != g_free.end();) {
    if (it->first.first == s) {
      g_free.insert({{kIdle, it->first.second}, it->second});
      it = g_free.erase(it);
    } else {
      ++it;
    }
  }
}

void dev_cache_release() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  (void)hipDeviceSynchronize();
  for (auto& kv : g_free) {
    (void)hipFree(kv.second);
    g_size.erase(kv.second);
  }
  g_free.clear();
}

// ---------------------------------------------------------------------------
// Fills
// ---------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(T* a, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) a[i] = v;
}

template <typename T>
static void fill_t(T* a, T v, size_t n, hipStream_t s) {
  if (!n) return;
  unsigned g = std::min<unsigned>(grid_for(n, 256), 8192);
  fill_kernel<T><<<g, 256, 0, s>>>(a, v, n);
  PCAMG_LAUNCHED();
}

void fill_i32(int32_t* a, int32_t v, size_t n, hipStream_t s) { fill_t(a, v, n, s); }
void fill_u32(uint32_t* a, uint32_t v, size_t n, hipStream_t s) { fill_t(a, v, n, s); }
void fill_u64(uint64_t* a, uint64_t v, size_t n, hipStream_t s) { fill_t(a, v, n, s); }
void fill_f64(double* a, double v, size_t n, hipStream_t s) { fill_t(a, v, n, s); }
void fill_f32(float* a, float v, size_t n, hipStream_t s) { fill_t(a, v, n, s); }

__global__ void iota_kernel(int32_t* a, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}
void iota_i32(int32_t* a, size_t n, hipStream_t s) {
  if (!n) return;
  iota_kernel<<<grid_for(n, 256), 256, 0, s>>>(a, n);
  PCAMG_LAUNCHED();
}

// ---------------------------------------------------------------------------
// Prefix sums: 1024 items per block (256 threads x 4), block totals scanned
// recursively, then added back.
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__device__ T block_exclusive_scan(T v, T* total) {
  __shared__ T wsum[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
      T t = wsum[w];
      wsum[w] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  return x - v + wsum[wid];
}

template <typename TI, typename TO>
__global__ void scan_tiles_kernel(const TI* in, TO* out, TO* tile_sums, size_t n) {
  __shared__ TO tot;
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  TO v[SCAN_ITEMS];
  TO sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? (TO)in[base + k] : (TO)0;
    sum += v[k];
  }
  TO ex = block_exclusive_scan<TO>(sum, &tot);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = tot;
}

template <typename TO>
__global__ void add_tile_offsets_kernel(TO* out, const TO* offs, size_t n) {
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  const TO o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) out[base + k] += o;
}

template <typename TO>
__global__ void write_total_kernel(const TO* offs_excl, const TO* sums, size_t ntiles, TO* total) {
  *total = offs_excl[ntiles - 1] + sums[ntiles - 1];
}

template <typename TI, typename TO>
static void scan_exclusive_t(const TI* in, TO* out, size_t n, TO* total, hipStream_t s) {
  if (n == 0) {
    if (total) PCAMG_HIP(hipMemsetAsync(total, 0, sizeof(TO), s));
    return;
  }
  const size_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (ntiles == 1) {  // the one tile's sum is the total
    scan_tiles_kernel<TI, TO><<<1, SCAN_BLOCK, 0, s>>>(in, out, total, n);
    PCAMG_LAUNCHED();
    return;
  }
  DVec<TO> sums(ntiles), offs(ntiles);
  scan_tiles_kernel<TI, TO><<<(unsigned)ntiles, SCAN_BLOCK, 0, s>>>(in, out, sums.p, n);
  PCAMG_LAUNCHED();
  scan_exclusive_t<TO, TO>(sums.p, offs.p, ntiles, (TO*)nullptr, s);
  add_tile_offsets_kernel<TO><<<(unsigned)ntiles, SCAN_BLOCK, 0, s>>>(out, offs.p, n);
  PCAMG_LAUNCHED();
  if (total) {
    write_total_kernel<TO><<<1, 1, 0, s>>>(offs.p, sums.p, ntiles, total);
    PCAMG_LAUNCHED();
  }
}

void scan_exclusive_i32(const int32_t* in, int32_t* out, size_t n, int32_t* total, hipStream_t s) {
  scan_exclusive_t<int32_t, int32_t>(in, out, n, total, s);
}
void scan_exclusive_i64(const int32_t* in, int64_t* out, size_t n, hipStream_t s) {
  scan_exclusive_t<int32_t, int64_t>(in, out, n, (int64_t*)nullptr, s);
}

// ---------------------------------------------------------------------------
// Deterministic reductions: a fixed grid of per-thread strided partial sums,
// block trees, then one block over the block partials in index order.
// ---------------------------------------------------------------------------
constexpr int RED_BLOCK = 256;

__device__ double block_sum_f64(double v) {
  __shared__ double sh[RED_BLOCK / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < RED_BLOCK / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

__global__ void dot_partial_kernel(const double* a, const double* b, size_t n, double* part) {
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * RED_BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * RED_BLOCK)
    acc = fma(a[i], b ? b[i] : 1.0, acc);
  double t = block_sum_f64(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void sum_partials_kernel(const double* part, int np, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += RED_BLOCK) acc += part[i];
  double t = block_sum_f64(acc);
  if (threadIdx.x == 0) *out = t;
}

static unsigned red_grid(size_t n) { return (unsigned)std::min<size_t>(1024, std::max<size_t>(1, (n + 2047) / 2048)); }

void dot_f64(const double* a, const double* b, size_t n, double* out, hipStream_t s) {
  unsigned g = red_grid(n);
  DVec<double> part(g);
  dot_partial_kernel<<<g, RED_BLOCK, 0, s>>>(a, b, n, part.p);
  PCAMG_LAUNCHED();
  sum_partials_kernel<<<1, RED_BLOCK, 0, s>>>(part.p, (int)g, out);
  PCAMG_LAUNCHED();
}

void sum_f64(const double* a, size_t n, double* out, hipStream_t s) { dot_f64(a, nullptr, n, out, s); }

__global__ void max_abs_bits_kernel(const double* a, size_t n, unsigned long long* out) {
  unsigned long long m = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(fabs(a[i]));
    m = b > m ? b : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long y = __shfl_down(m, o, 64);
    m = y > m ? y : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

void max_abs_bits_f64(const double* a, size_t n, uint64_t* out, hipStream_t s) {
  PCAMG_HIP(hipMemsetAsync(out, 0, sizeof(uint64_t), s));
  unsigned g = std::min<unsigned>(grid_for(n, 256), 2048);
  max_abs_bits_kernel<<<g, 256, 0, s>>>(a, n, (unsigned long long*)out);
  PCAMG_LAUNCHED();
}

__global__ void or_and_kernel(const uint64_t* a, size_t n, unsigned long long* out) {
  unsigned long long o = 0, an = ~0ull;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    o |= a[i];
    an &= a[i];
  }
  for (int k = 32; k > 0; k >>= 1) {
    o |= __shfl_down(o, k, 64);
    an &= __shfl_down(an, k, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicOr(&out[0], o);
    atomicAnd(&out[1], an);
  }
}

void or_and_u64(const uint64_t* a, size_t n, uint64_t* out, hipStream_t s) {
  uint64_t init[2] = {0ull, ~0ull};
  PCAMG_HIP(hipMemcpyAsync(out, init, sizeof(init), hipMemcpyHostToDevice, s));
  unsigned g = std::min<unsigned>(grid_for(n, 256), 2048);
  or_and_kernel<<<g, 256, 0, s>>>(a, n, (unsigned long long*)out);
  PCAMG_LAUNCHED();
  PCAMG_HIP(hipStreamSynchronize(s));  // `init` lives on this stack frame
}

// ---------------------------------------------------------------------------
// Compaction
// ---------------------------------------------------------------------------
__global__ void flags_to_i32_kernel(const uint8_t* f, int32_t* o, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = f[i] ? 1 : 0;
}
__global__ void compact_scatter_kernel(const int32_t* in, const uint8_t* f, const int32_t* pos, int32_t* out,
                                       size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && f[i]) out[pos[i]] = in ? in[i] : (int32_t)i;
}

void compact_i32(const int32_t* in, const uint8_t* flags, int32_t* out, int32_t* count, size_t n, hipStream_t s) {
  if (n == 0) {
    PCAMG_HIP(hipMemsetAsync(count, 0, sizeof(int32_t), s));
    return;
  }
  DVec<int32_t> pos(n);
  flags_to_i32_kernel<<<grid_for(n, 256), 256, 0, s>>>(flags, pos.p, n);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(pos.p, pos.p, n, count, s);
  compact_scatter_kernel<<<grid_for(n, 256), 256, 0, s>>>(in, flags, pos.p, out, n);
  PCAMG_LAUNCHED();
}

__global__ void row_longer_flag_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ perm,
                                       int32_t len, uint8_t* __restrict__ f) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = perm ? perm[i] : i;
  f[i] = rp[r + 1] - rp[r] > len;
}

int32_t rows_longer_than(int32_t n, const int32_t* rp, const int32_t* perm, int32_t len, DVec<int32_t>& rows,
                         hipStream_t s) {
  if (n <= 0) return 0;
  DVec<uint8_t> f(n);
  DVec<int32_t> cnt(1);
  row_longer_flag_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, perm, len, f.p);
  PCAMG_LAUNCHED();
  rows.resize(n);
  compact_i32(nullptr, f.p, rows.p, cnt.p, n, s);
  return read_scalar(cnt.p, s);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits.
//  pass k: (1) per-tile digit histograms, stored digit-major so one exclusive
//  scan gives every (digit, tile) its global offset; (2) per tile, each wave
//  ranks its keys in order with 64-bit ballots (peers = lanes with the same
//  digit), waves are combined in wave order, the tile is reordered in LDS
//  and written out digit run by digit run to offset + rank (coalesced).  Keys
//  keep their input order within a digit (stable).
// ---------------------------------------------------------------------------
constexpr int RS_BLOCK = 512;
constexpr int RS_ITEMS = 8;                       // per lane
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;      // 4096 keys per block (runs of 16 keys per digit on average)
constexpr int RS_WAVES = RS_BLOCK / 64;
static_assert(RS_BLOCK >= 256, "a thread per digit in the histogram");

template <typename K>
__global__ void __launch_bounds__(RS_BLOCK) rs_hist_kernel(const K* keys, size_t n, int shift, int32_t* hist, int ntiles) {
  __shared__ int32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * RS_TILE;
  // the tile's keys loaded together (past the end: the last key again, not
  // counted), then counted
  K kk[RS_ITEMS];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r) kk[r] = keys[min(base + (size_t)(r * RS_BLOCK + threadIdx.x), n - 1)];
#pragma unroll
  for (int r = 0; r < RS_ITEMS; ++r)
    if (base + (size_t)(r * RS_BLOCK + threadIdx.x) < n) atomicAdd(&h[(int)((kk[r] >> shift) & 0xFF)], 1);
  __syncthreads();
  if (threadIdx.x < 256) hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <typename K>
__global__ void __launch_bounds__(RS_BLOCK) rs_scatter_kernel(const K* keys, const uint32_t* vals, K* okeys, uint32_t* ovals, size_t n,
                                  int shift, const int32_t* offs, int ntiles) {
  __shared__ int32_t wcount[RS_WAVES][256];
  __shared__ int32_t goff[256];
  __shared__ int32_t tstart[256];
  __shared__ K lkey[RS_TILE];
  __shared__ uint32_t lval[RS_TILE];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 256; d += RS_BLOCK) {
    for (int w = 0; w < RS_WAVES; ++w) wcount[w][d] = 0;
    goff[d] = offs[(size_t)d * ntiles + blockIdx.x];
  }
  __syncthreads();
  const size_t seg = (size_t)blockIdx.x * RS_TILE + (size_t)wid * (64 * RS_ITEMS);
  K kk[RS_ITEMS];
  uint32_t vv[RS_ITEMS];
  int32_t rank[RS_ITEMS];
  int dig[RS_ITEMS];
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    size_t i = seg + (size_t)r * 64 + lane;
    bool valid = i < n;
    K key = valid ? keys[i] : (K)0;
    uint32_t val = valid ? vals[i] : 0u;
    int d = (int)((key >> shift) & 0xFF);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      unsigned long long bb = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bb : ~bb;
    }
    int before = 0;
    if (valid) before = wcount[wid][d];
    // all lanes have read the running count before any leader updates it
    __builtin_amdgcn_wave_barrier();
    int leader = valid ? (__ffsll((long long)peers) - 1) : -1;
    if (valid && lane == leader) wcount[wid][d] = before + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
    kk[r] = key;
    vv[r] = val;
    dig[r] = valid ? d : -1;
    rank[r] = before + __popcll(peers & lt);
  }
  __syncthreads();
  // exclusive prefix over waves for each digit, and the tile's digit counts
  for (int d = threadIdx.x; d < 256; d += RS_BLOCK) {
    int acc = 0;
    for (int w = 0; w < RS_WAVES; ++w) {
      int t = wcount[w][d];
      wcount[w][d] = acc;
      acc += t;
    }
    tstart[d] = acc;
  }
  __syncthreads();
  // tile-local start of every digit (exclusive scan of the 256 counts)
  if (threadIdx.x < 64) {
    int c[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c[q] = tstart[4 * lane + q];
      sum += c[q];
    }
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    int run = incl - sum;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      tstart[4 * lane + q] = run;
      run += c[q];
    }
  }
  __syncthreads();
  // the tile in LDS in its sorted order (stable: wave order, then rank) ...
  for (int r = 0; r < RS_ITEMS; ++r) {
    if (dig[r] < 0) continue;
    const int lp = tstart[dig[r]] + wcount[wid][dig[r]] + rank[r];
    lkey[lp] = kk[r];
    lval[lp] = vv[r];
  }
  __syncthreads();
  // ... then written out in that order: a digit's run is one contiguous
  // segment of the output, so consecutive threads write consecutive addresses
  const size_t base = (size_t)blockIdx.x * RS_TILE;
  const int tn = (int)(n - base < (size_t)RS_TILE ? n - base : (size_t)RS_TILE);
  for (int i = threadIdx.x; i < tn; i += RS_BLOCK) {
    const K key = lkey[i];
    const int d = (int)((key >> shift) & 0xFF);
    const int32_t dst = goff[d] + (i - tstart[d]);
    okeys[dst] = key;
    ovals[dst] = lval[i];
  }
}

template <typename K>
static void radix_sort_t(const K* keys_in, const uint32_t* vals_in, K* keys_out, uint32_t* vals_out, size_t n,
                         uint64_t varying, hipStream_t s) {
  if (n == 0) return;
  require(n < (size_t)INT32_MAX, PCAMG_EUNSUPPORTED, "radix sort: more than 2^31 keys");
  const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  std::vector<int> passes;
  for (int sh = 0; sh < (int)(8 * sizeof(K)); sh += 8)
    if ((varying >> sh) & 0xFFull) passes.push_back(sh);
  if (passes.empty()) {
    copy_d2d(keys_out, keys_in, n, s);
    copy_d2d(vals_out, vals_in, n, s);
    return;
  }
  DVec<K> kb(n);
  DVec<uint32_t> vb(n);
  DVec<int32_t> hist((size_t)256 * ntiles);
  // ping-pong so that the last pass writes keys_out/vals_out
  const K* ksrc = keys_in;
  const uint32_t* vsrc = vals_in;
  const int np = (int)passes.size();
  for (int t = 0; t < np; ++t) {
    bool to_out = ((np - 1 - t) % 2) == 0;
    K* kdst = to_out ? keys_out : kb.p;
    uint32_t* vdst = to_out ? vals_out : vb.p;
    rs_hist_kernel<K><<<ntiles, RS_BLOCK, 0, s>>>(ksrc, n, passes[t], hist.p, ntiles);
    PCAMG_LAUNCHED();
    scan_exclusive_i32(hist.p, hist.p, (size_t)256 * ntiles, nullptr, s);
    rs_scatter_kernel<K><<<ntiles, RS_BLOCK, 0, s>>>(ksrc, vsrc, kdst, vdst, n, passes[t], hist.p, ntiles);
    PCAMG_LAUNCHED();
    ksrc = kdst;
    vsrc = vdst;
  }
}

void radix_sort_u64_u32(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
                        size_t n, hipStream_t s) {
  if (n == 0) return;
  DVec<uint64_t> oa(2);
  or_and_u64(keys_in, n, oa.p, s);  // synchronises
  auto h = to_host(oa.p, 2, s);
  radix_sort_t<uint64_t>(keys_in, vals_in, keys_out, vals_out, n, h[0] ^ h[1], s);
}

void radix_sort_u32_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                        size_t n, int key_bits, hipStream_t s) {
  uint64_t varying = key_bits >= 32 ? 0xFFFFFFFFull : ((1ull << key_bits) - 1);
  radix_sort_t<uint32_t>(keys_in, vals_in, keys_out, vals_out, n, varying, s);
}

}  // namespace pcamg
