// Internal declarations of the HIP library: errors, device memory, and the
// host-side launchers of every kernel.  All launchers enqueue on `s` and do not
// synchronise unless their name says so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pcamg.h"

namespace pcamg {

// ---------------------------------------------------------------------------
// Errors: launchers throw Error; the C ABI converts it to a status.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  pcamg_status code;
  Error(pcamg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PCAMG_HIP(call)                                                                              \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      throw ::pcamg::Error(PCAMG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_) + " at " + \
                                           __FILE__ + ":" + std::to_string(__LINE__));              \
  } while (0)

#define PCAMG_LAUNCHED() PCAMG_HIP(hipGetLastError())

inline void require(bool ok, pcamg_status code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------------------
// Device memory: a size-bucketed cache so rebuilds reuse allocations.  Blocks
// freed while a StreamScope is active are reused only on that stream.
// ---------------------------------------------------------------------------
void* dev_alloc(size_t bytes);
void dev_free(void* p);
void dev_cache_release();             // return cached blocks to the runtime
void dev_cache_idle(hipStream_t s);   // s is synchronised: its blocks may serve any stream
struct StreamScope {                  // the stream this thread's allocations belong to
  explicit StreamScope(hipStream_t s);
  ~StreamScope();
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
  hipStream_t prev;
};

template <typename T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  DVec() = default;
  explicit DVec(size_t count) { resize(count); }
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  DVec(DVec&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DVec& operator=(DVec&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DVec() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  void resize(size_t count) {
    release();
    n = count;
    if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T)));
  }
  size_t bytes() const { return n * sizeof(T); }
  T* get() const { return p; }
};

template <typename T>
std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    PCAMG_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    PCAMG_HIP(hipStreamSynchronize(s));
  }
  return h;
}

template <typename T>
T read_scalar(const T* d, hipStream_t s) {
  T v{};
  PCAMG_HIP(hipMemcpyAsync(&v, d, sizeof(T), hipMemcpyDeviceToHost, s));
  PCAMG_HIP(hipStreamSynchronize(s));
  return v;
}

template <typename T>
void copy_d2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) PCAMG_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

template <typename T>
void copy_h2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) PCAMG_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}

inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  return (unsigned)(g ? g : 1);
}

// ---------------------------------------------------------------------------
// util.hip: fills, scans, reductions, radix sort
// ---------------------------------------------------------------------------
void fill_i32(int32_t* a, int32_t v, size_t n, hipStream_t s);
void fill_u32(uint32_t* a, uint32_t v, size_t n, hipStream_t s);
void fill_u64(uint64_t* a, uint64_t v, size_t n, hipStream_t s);
void fill_f64(double* a, double v, size_t n, hipStream_t s);
void fill_f32(float* a, float v, size_t n, hipStream_t s);
void iota_i32(int32_t* a, size_t n, hipStream_t s);

// Exclusive prefix sum of int32 counts into int32 offsets; out may alias in.
// If total != nullptr the (device) total is written there.  n <= 2^31 - 1.
void scan_exclusive_i32(const int32_t* in, int32_t* out, size_t n, int32_t* total, hipStream_t s);
// Same with 64-bit output (for sizes that can exceed int32).
void scan_exclusive_i64(const int32_t* in, int64_t* out, size_t n, hipStream_t s);

// Deterministic reductions (fixed tree, independent of timing).
// Result written to device `out`.
void dot_f64(const double* a, const double* b, size_t n, double* out, hipStream_t s);
void sum_f64(const double* a, size_t n, double* out, hipStream_t s);
void max_abs_bits_f64(const double* a, size_t n, uint64_t* out, hipStream_t s);  // max |a| as bits
void or_and_u64(const uint64_t* a, size_t n, uint64_t* out_or_and /*[2]*/, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by key.  `bits` = number of low
// key bits that may vary (skips constant 8-bit digits).  Output in keys_out /
// vals_out; temporaries from the cache.
void radix_sort_u64_u32(const uint64_t* keys_in, const uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out,
                        size_t n, hipStream_t s);
void radix_sort_u32_u32(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                        size_t n, int key_bits, hipStream_t s);

// Stable compaction: out[k] = in[i] for flags[i] != 0 in order; *count (device).
void compact_i32(const int32_t* in, const uint8_t* flags, int32_t* out, int32_t* count, size_t n, hipStream_t s);
// The positions i < n (in order) whose row perm[i] (i itself when perm is
// null) has more than len entries: written to rows (resized to n), count
// returned (synchronises).  Kernels that walk a row per thread leave those
// rows to a workgroup each.
int32_t rows_longer_than(int32_t n, const int32_t* rp, const int32_t* perm, int32_t len, DVec<int32_t>& rows,
                         hipStream_t s);

// ---------------------------------------------------------------------------
// vec.hip: vector kernels for the outer iterations
// ---------------------------------------------------------------------------
void axpy_f64(double alpha_host, const double* x, double* y, size_t n, hipStream_t s);     // y += a x
void axpy_dev_f64(const double* alpha, int sign, const double* x, double* y, size_t n, hipStream_t s);
void xpby_dev_f64(const double* z, const double* beta, double* p, size_t n, hipStream_t s);  // p = z + beta p
void sub_mean_f64(double* x, const double* sum, size_t n, hipStream_t s);                   // x -= sum / n
void gather_f64(const double* src, const int32_t* idx, double* dst, size_t n, hipStream_t s);   // dst[i] = src[idx[i]]
void scatter_f64(const double* src, const int32_t* idx, double* dst, size_t n, hipStream_t s);  // dst[idx[i]] = src[i]
void gather_f32(const float* src, const int32_t* idx, float* dst, size_t n, hipStream_t s);
void scatter_f32(const float* src, const int32_t* idx, float* dst, size_t n, hipStream_t s);
void gather_i32(const int32_t* src, const int32_t* idx, int32_t* dst, size_t n, hipStream_t s);
void cast_f64_f32(const double* a, float* b, size_t n, hipStream_t s);
void cast_f32_f64(const float* a, double* b, size_t n, hipStream_t s);
void xi_fill(uint64_t seed, int32_t r, const int32_t* perm, double* out, size_t n, hipStream_t s);
void sub_f64(const double* a, const double* b, double* out, size_t n, hipStream_t s);        // out = a - b
void zsub_dot_f64(const double* z, const double* rn, const double* r, size_t n, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// basic.hip: Laplacian, colouring, smoother, residual, transfers
// ---------------------------------------------------------------------------
void laplacian(int32_t n, const int32_t* rp, const double* w, double* aval, double* d, double* dinv,
               size_t nnz, hipStream_t s);
int32_t colour_jp(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level, int32_t* colour,
                  hipStream_t s);
// Red-black colouring (parity of the breadth-first depth from vertex 0) when
// the graph is connected and bipartite; returns false otherwise.
bool colour_bipartite(int32_t n, const int32_t* rp, const int32_t* ci, int32_t* colour, hipStream_t s);
// The smoother's colouring of a level graph: red-black if connected and
// bipartite, Jones-Plassmann otherwise.  Returns the number of colours.
int32_t colour_level(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level, int32_t* colour,
                     hipStream_t s);  // synchronises; returns number of colours

template <typename T>
void gs_colour(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av, const T* dinv,
               const T* b, T* x, hipStream_t s, int lanes = 1);  // lanes per row: 1, 4, 16, 64
template <typename T>
void gs_colour_rows(int32_t nrows, const int32_t* rows, const int32_t* rp, const int32_t* ci, const T* av,
                    const T* dinv, const T* b, T* x, hipStream_t s);
// long_min > 0: rows of long_min entries or more are skipped (residual_long)
template <typename T>
void residual(int32_t n, const int32_t* rp, const int32_t* ci, const T* av, const T* d, const T* b, const T* x,
              T* r, hipStream_t s, int lanes = 1, int32_t long_min = 0);
// Long rows, one workgroup each (a fixed summation tree instead of the single
// chain): Gauss-Seidel over rows row0..row1-1, residual over a row list.
template <typename T>
void gs_colour_long(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av, const T* dinv,
                    const T* b, T* x, hipStream_t s);
// One launch for both parts of a colour: long rows [row0, rl) as
// gs_colour_long, rows [rl, row1) as gs_colour with `lanes` lanes per row.
template <typename T>
void gs_colour_fused(int32_t row0, int32_t rl, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av,
                     const T* dinv, const T* b, T* x, hipStream_t s, int lanes);
// Gauss-Seidel over long rows [row0, row1) by the single chain in stored
// order (as gs_colour), a wavefront each staging the row through LDS.
template <typename T>
void gs_colour_chain_long(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* ci, const T* av,
                          const T* dinv, const T* b, T* x, hipStream_t s);
template <typename T>
void residual_long(int32_t nrows, const int32_t* rows, const int32_t* rp, const int32_t* ci, const T* av,
                   const T* d, const T* b, const T* x, T* r, hipStream_t s);
// Colour passes c_first, c_first + step, ... (up to, not including, c_end) of
// one sweep in a single workgroup: rows [coff[c], lend[c]) by the long-row
// tree, the rest by single chains; device coff_d[ncol + 1], lend_d[ncol].
// Bit-identical to gs_colour_long + gs_colour per colour.
template <typename T>
void gs_sweep_block(int32_t c_first, int32_t c_end, int32_t step, const int32_t* coff_d, const int32_t* lend_d,
                    const int32_t* rp, const int32_t* ci, const T* av, const T* dinv, const T* b, T* x,
                    hipStream_t s);
template <typename T>
void spmv(int32_t n, const int32_t* rp, const int32_t* ci, const T* av, const T* d, const T* x, T* y,
          hipStream_t s, int lanes = 1);
// Sliced-ELL (SELL-64) copy of a matrix with short rows: slice q = rows
// 64q .. 64q + 63, entry j of row 64q + l at 64 woff[q] + 64 j + l.  Returns
// false (woff emptied, nothing else allocated) when the padded slots would be
// more than twice the entries (padding is never read, so it costs memory, not
// bandwidth).  Synchronises.
bool sell_build(int32_t n, int32_t nnz, const int32_t* rp, const int32_t* ci, const double* av, const float* av32,
                DVec<int32_t>& woff, DVec<int32_t>& sci, DVec<double>& sav, DVec<float>& sav32, hipStream_t s);
// Padded-row (ELL, width W = longest row) FP32 copy of a level with 4 or 16
// lanes per row and W small enough for one batch of loads per lane (W <= 64
// for 4 lanes, <= 128 for 16); false (nothing allocated) otherwise.
// Synchronises.
bool ell_build(int32_t n, int32_t lanes, const int32_t* rp, const int32_t* ci, const float* av32, int32_t& W,
               DVec<int32_t>& eci, DVec<float>& eav, hipStream_t s);
// FP32 Gauss-Seidel colour pass on that copy: the same chains, results identical.
void gs_colour_ell(int32_t row0, int32_t row1, int32_t W, int lanes, const int32_t* rp, const int32_t* eci,
                   const float* eav, const float* dinv, const float* b, float* x, hipStream_t s);
// Gauss-Seidel colour pass and residual (b == nullptr: product) on that copy;
// rp still gives the row lengths.  Same results as the CSR kernels.
template <typename T>
void gs_colour_sell(int32_t row0, int32_t row1, const int32_t* rp, const int32_t* woff, const int32_t* sci,
                    const T* sav, const T* dinv, const T* b, T* x, hipStream_t s);
template <typename T>
void residual_sell(int32_t n, const int32_t* rp, const int32_t* woff, const int32_t* sci, const T* sav, const T* d,
                   const T* b, const T* x, T* r, hipStream_t s);
// with xc: mode 1 also zeroes xc, mode 2 also does the coarse first colour
// pass from zero (rows < c1: xc = bc * dinvc, others 0)
template <typename T>
void restrict_members(int32_t nc, const int32_t* moff, const int32_t* mem, const T* pval, const T* r, T* bc,
                      hipStream_t s, T* xc = nullptr, const T* dinvc = nullptr, int32_t c1 = 0, int mode = 0);
template <typename T>
void prolong_add(int32_t n, const int32_t* agg, const T* pval, const T* xc, T* x, hipStream_t s);


// ---------------------------------------------------------------------------
// setup.hip: hierarchy construction kernels (natural numbering)
// ---------------------------------------------------------------------------
// A^2 pattern; returns nnz2 (synchronises).  Throws PCAMG_EUNSUPPORTED if a
// row has more candidates than the kernel supports.
int64_t a2_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, int32_t* rp2, hipStream_t s);
void a2_fill(int32_t n, const int32_t* rp, const int32_t* ci, int32_t cap, const int32_t* rp2, int32_t* ci2,
             hipStream_t s);
// keys and reweighted values on the pattern; upper edge list (eu, ev, key bits)
// in lexicographic edge order.  Returns m (synchronises).
int32_t a2_keys(int32_t n, const int32_t* rp2, const int32_t* ci2, const double* e, double* gkey, double* gv,
                int32_t* eu, int32_t* ev, uint64_t* ekey, hipStream_t s);
// sorted ranks -> su/sv (edges in processing order)
void sorted_endpoints(int32_t m, const uint32_t* order, const int32_t* eu, const int32_t* ev, int32_t* su,
                      int32_t* sv, hipStream_t s);
// Greedy path cover by deterministic reservations; nb[2n] (synchronises).
int32_t path_cover(int32_t n, int32_t m, const int32_t* su, const int32_t* sv, int32_t* nb, hipStream_t s);
// Pointer-jumping orientation: path_id, pos, plen (synchronises).
void orient_paths(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen, hipStream_t s);
// The same on a caller's device workspace of orient_ws_ints(n) int32 (no
// allocation; every entry the kernels read is written first).
inline size_t orient_ws_ints(int32_t n) { return 12 * (size_t)n + 1; }
void orient_paths_ws(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen, int32_t* ws,
                     hipStream_t s);
// noalloc.hip: device address (current device) of the fixed orientation
// workspace of orient_ws_ints(PCAMG_ORIENT_NOALLOC_MAX_N) int32.
int32_t* orient_noalloc_scratch();

struct AggStats {
  int32_t n_unagg = 0, case1 = 0, case2 = 0, case3 = 0, middle = 0, singleton = 0, p1_fallback = 0;
  int32_t n_paths = 0, n_path_vertices = 0, repair_rounds = 0, cover_rounds = 0;
};
// Alg. 3 on one level; returns nc; agg[n], member CSR moff[nc+1], mem[n]
// (device, allocated by the caller with n+1 / n entries). (synchronises)
// case3 = 1: Case 3 as printed (v always leaves its aggregate).
int32_t aggregate_level(int32_t n, const int32_t* grp, const int32_t* gci, const double* gw, const double* gkey,
                        const int32_t* nb, const int32_t* path_id, const int32_t* pos, const int32_t* plen,
                        int32_t* agg, int32_t* moff, int32_t* mem, AggStats& st, hipStream_t s, int32_t case3 = 0);
// MWM aggregation (Sec. 2.1) of a level with off-diagonal entries av (weights
// -av); returns nc; agg[n], moff[nc+1], mem[n] as for aggregate_level;
// st.n_unagg (left after the matching), st.case2 (joined), st.singleton.
// (synchronises)
int32_t mwm_aggregate_level(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, int32_t* agg,
                            int32_t* moff, int32_t* mem, AggStats& st, hipStream_t s);
// Level-1 prolongation values from e_raw (power-of-two normalisation,
// fixed-point mean, small-aggregate fallback).  Returns fallback count.
int32_t smooth_pval(int32_t n, const double* e_raw, int32_t nc, const int32_t* moff, const int32_t* mem,
                    double* pval, hipStream_t s);
// The sorted terms of the coarse rows too long for the one-pass kernel,
// kept by a count pass for the fill pass of the same product.
struct GalerkinCache {
  int32_t nL = -1;  // -1: nothing kept
  int64_t total = 0;
  DVec<int32_t> rows;
  DVec<int64_t> off;
  DVec<uint64_t> ks;
  DVec<uint32_t> perm;
};
// Galerkin P^T A P (pval == nullptr: boolean).  Count pass then fill pass;
// with a cache, the fill pass right after the count pass of the same
// operands reuses its sort.
int64_t galerkin_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t nc, const int32_t* moff,
                       const int32_t* mem, const int32_t* agg, int32_t* rpc, bool drop_diag, hipStream_t s,
                       GalerkinCache* cache = nullptr);
void galerkin_fill(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, const double* d,
                   int32_t nc, const int32_t* moff, const int32_t* mem, const int32_t* agg, const double* pval,
                   const int32_t* rpc, int32_t* cic, double* vc, double* dc, double* dinvc, bool graph_mode,
                   hipStream_t s, GalerkinCache* cache = nullptr);
// Path shortening: coarse cover nbc[2nc].
void shorten_paths(int32_t n, const int32_t* nb, const int32_t* path_id, const int32_t* pos, int32_t nc,
                   const int32_t* agg, int32_t* nbc, hipStream_t s);

// ---------------------------------------------------------------------------
// layout.hip: colour-permuted solve layout
// ---------------------------------------------------------------------------
void build_perm(int32_t n, const int32_t* colour, int32_t ncol, int32_t* perm, int32_t* iperm,
                std::vector<int32_t>& coff, hipStream_t s);
// Largest row length of a CSR matrix (synchronises).
int32_t max_row_len(int32_t n, const int32_t* rp, hipStream_t s);
// Same with the rows of long_min entries or more first within each colour:
// lend[c] = end of colour c's long rows (coff[c] <= lend[c] <= coff[c + 1]).
void build_perm_long(int32_t n, const int32_t* colour, int32_t ncol, const int32_t* rp, int32_t long_min,
                     int32_t* perm, int32_t* iperm, std::vector<int32_t>& coff, std::vector<int32_t>& lend,
                     hipStream_t s);
void permute_csr(int32_t n, const int32_t* perm, const int32_t* iperm, const int32_t* rp, const int32_t* ci,
                 const double* av, const double* d, const double* dinv, int32_t* rpp, int32_t* cip, double* avp,
                 float* avp32, double* dp, double* dinvp, float* dp32, float* dinvp32, hipStream_t s);
void permute_transfer(int32_t n, const int32_t* perm, const int32_t* iperm, int32_t nc, const int32_t* permc,
                      const int32_t* ipermc, const int32_t* agg, const double* pval, const int32_t* moff,
                      const int32_t* mem, int32_t* aggp, double* pvalp, float* pvalp32, int32_t* moffp,
                      int32_t* memp, hipStream_t s);

// ---------------------------------------------------------------------------
// coarse.hip: dense LDL^T of the coarsest level
// ---------------------------------------------------------------------------
// Dense matrix from CSR (n x n row-major).
void dense_from_csr(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, const double* d, double* A,
                    hipStream_t s);
// Factor the leading m x m block; returns false on a non-positive pivot (synchronises).
bool ldlt_factor(int32_t n, int32_t m, const double* A, double* L, double* D, hipStream_t s);
// x = solve(b); grounded: x[n-1] = 0 then mean removed.
void ldlt_solve(int32_t n, int32_t m, bool grounded, const double* L, const double* D, const double* b, double* x,
                hipStream_t s);
void ldlt_solve32(int32_t n, int32_t m, bool grounded, const double* L, const double* D, const float* b, float* x,
                  hipStream_t s);

}  // namespace pcamg
