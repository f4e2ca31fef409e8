// Tail of a multigrid cycle in one workgroup.  The small levels of a
// hierarchy (and the dense coarsest solve) are visited many times per cycle --
// 2^l times in a W-cycle -- and each visit of a multicoloured level is a long
// chain of tiny steps.  Here the whole sub-cycle from the first small level
// down to the coarsest runs in a single launch of 1024 threads, with a
// workgroup barrier between dependent steps.  All vectors of the sub-cycle sit
// in LDS for the launch, so a step's only global reads are matrix entries,
// which do not depend on the previous step.  Every row and every sum uses the
// same arithmetic and order as the per-step kernels, so results are identical
// bit for bit.
#include <type_traits>
#include "rowchain.hpp"
#include "solver.hpp"

namespace pcamg {

constexpr int TAIL_THREADS = 1024;

template <typename T>
using GP = const PCAMG_GLOBAL T*;
template <typename T>
using GW = PCAMG_GLOBAL T*;
template <typename T>
__device__ __forceinline__ GW<T> gptr_w(T* p) {
  return (GW<T>)p;
}

// sum_j C[j * n + i] * v[j] as one fma chain in j order (C column-major), the
// column entries loaded sixteen ahead of the chain
template <typename T, typename PC, typename PV>
__device__ __forceinline__ T dense_row_dot(int32_t n, PC C, int32_t i, PV v) {
  constexpr int U = 16;
  T s = 0;
  int32_t j = 0;
  for (; j + U <= n; j += U) {
    T c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = C[(size_t)(j + u) * n + i];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(c[u], v[j + u], s);
  }
  for (; j < n; ++j) s = fma(C[(size_t)j * n + i], v[j], s);
  return s;
}

template <typename T>
struct TailOps;
template <>
struct TailOps<double> {
  __device__ static GP<double> av(const TailLevel& L) { return gptr(L.av); }
  __device__ static GP<double> d(const TailLevel& L) { return gptr(L.d); }
  __device__ static GP<double> dinv(const TailLevel& L) { return gptr(L.dinv); }
  __device__ static GP<double> pval(const TailLevel& L) { return gptr(L.pval); }
  __device__ static GW<double> gx(const TailLevel& L) { return gptr_w(L.x); }
  __device__ static GW<double> gb(const TailLevel& L) { return gptr_w(L.b); }
  __device__ static GW<double> gr(const TailLevel& L) { return gptr_w(L.r); }
  __device__ static int32_t off(const TailLevel& L, int j) { return L.o64[j]; }
  __device__ static int32_t oacc(const TailDesc& D) { return D.oacc64; }
  __device__ static int32_t oL(const TailDesc& D) { return D.oL64; }
  __device__ static GP<double> C(const TailDesc& D) { return gptr(D.C64); }
};
template <>
struct TailOps<float> {
  __device__ static GP<float> av(const TailLevel& L) { return gptr(L.av32); }
  __device__ static GP<float> d(const TailLevel& L) { return gptr(L.d32); }
  __device__ static GP<float> dinv(const TailLevel& L) { return gptr(L.dinv32); }
  __device__ static GP<float> pval(const TailLevel& L) { return gptr(L.pval32); }
  __device__ static GW<float> gx(const TailLevel& L) { return gptr_w(L.x32); }
  __device__ static GW<float> gb(const TailLevel& L) { return gptr_w(L.b32); }
  __device__ static GW<float> gr(const TailLevel& L) { return gptr_w(L.r32); }
  __device__ static int32_t off(const TailLevel& L, int j) { return L.o32[j]; }
  __device__ static int32_t oacc(const TailDesc& D) { return D.oacc32; }
  __device__ static int32_t oL(const TailDesc& D) { return D.oL32; }
  __device__ static GP<float> C(const TailDesc& D) { return gptr(D.C32); }
};

// One Gauss-Seidel sweep over the colours of a level (forward or backward), G
// lanes per row (1 or 16).  The vector pointer types carry the address space
// (LDS or global), so each combination compiles to direct LDS or global
// accesses.  With G > 1 all threads take part in every pass (uniform bounds),
// as row_chain_g requires.
template <typename T, int G, typename PB, typename PX>
__device__ __forceinline__ void tail_gs_g(const TailLevel& L, const int32_t* coff, PB b, PX x, bool forward) {
  constexpr int ROWS = TAIL_THREADS / G;
  const GP<T> av = TailOps<T>::av(L), dinv = TailOps<T>::dinv(L);
  const GP<int32_t> rp = gptr(L.rp), ci = gptr(L.ci);
  const int32_t g = (int32_t)(threadIdx.x / G);
  for (int t = 0; t < L.ncol; ++t) {
    const int c = forward ? t : L.ncol - 1 - t;
    const int32_t r0 = coff[c], r1 = coff[c + 1];
    for (int32_t i0 = r0; i0 < r1; i0 += ROWS) {
      const int32_t i = i0 + g;
      if constexpr (G == 1) {
        if (i < r1) {
          const T s = row_chain1<T>(rp[i], rp[i + 1], ci, av, x, (T)0);
          x[i] = (b[i] - s) * dinv[i];
        }
      } else {
        const bool ok = i < r1;
        const int32_t k0 = ok ? rp[i] : 0;
        const int32_t len = ok ? rp[i + 1] - k0 : 0;
        const T s = row_chain_g<T, G>(k0, len, ci, av, x, (T)0);
        if (ok && (threadIdx.x & (G - 1)) == 0) x[i] = (b[i] - s) * dinv[i];
      }
    }
    __syncthreads();
  }
}

template <typename T, int G, typename PB, typename PX, typename PR>
__device__ __forceinline__ void tail_res_g(const TailLevel& L, PB b, PX x, PR r) {
  constexpr int ROWS = TAIL_THREADS / G;
  const GP<T> av = TailOps<T>::av(L), d = TailOps<T>::d(L);
  const GP<int32_t> rp = gptr(L.rp), ci = gptr(L.ci);
  const int32_t g = (int32_t)(threadIdx.x / G);
  for (int32_t i0 = 0; i0 < L.n; i0 += ROWS) {
    const int32_t i = i0 + g;
    if constexpr (G == 1) {
      if (i < L.n) {
        const T s = row_chain1<T>(rp[i], rp[i + 1], ci, av, x, d[i] * x[i]);
        r[i] = b[i] - s;
      }
    } else {
      const bool ok = i < L.n;
      const int32_t k0 = ok ? rp[i] : 0;
      const int32_t len = ok ? rp[i + 1] - k0 : 0;
      const T s = row_chain_g<T, G>(k0, len, ci, av, x, ok ? d[i] * x[i] : (T)0);
      if (ok && (threadIdx.x & (G - 1)) == 0) r[i] = b[i] - s;
    }
  }
  __syncthreads();
}

template <typename T, typename PB, typename PX>
__device__ __forceinline__ void tail_gs(const TailLevel& L, const int32_t* coff, PB b, PX x, bool forward) {
  if (L.lanes == 1) tail_gs_g<T, 1>(L, coff, b, x, forward);
  else tail_gs_g<T, 16>(L, coff, b, x, forward);
}

// pre-smoothing, residual, restriction; the child's x starts at zero, or, with
// a dense operator Cd (nc x nc, column-major), is Cd times the restricted
// right-hand side (fma chain over the columns in order).
template <typename T, typename PB, typename PX, typename PR, typename PBC, typename PXC>
__device__ __forceinline__ void tail_down(const TailLevel& L, const int32_t* coff, PB b, PX x, PR r, PBC bc, PXC xc,
                                          int32_t nc, GP<T> Cd) {
  tail_gs<T>(L, coff, b, x, true);
  if (L.lanes == 1) tail_res_g<T, 1>(L, b, x, r);
  else tail_res_g<T, 16>(L, b, x, r);
  const GP<T> pv = TailOps<T>::pval(L);
  const GP<int32_t> moff = gptr(L.moff), mem = gptr(L.mem);
  for (int32_t q = threadIdx.x; q < nc; q += TAIL_THREADS) {
    T s = 0;
    for (int32_t t = moff[q]; t < moff[q + 1]; ++t) {
      const int32_t k = mem[t];
      s = fma(pv ? pv[k] : (T)1, r[k], s);
    }
    bc[q] = s;
    xc[q] = 0;
  }
  __syncthreads();
  if (Cd) {
    for (int32_t i = threadIdx.x; i < nc; i += TAIL_THREADS) xc[i] = dense_row_dot<T>(nc, Cd, i, bc);
    __syncthreads();
  }
}

// prolongation, post-smoothing
template <typename T, typename PB, typename PX, typename PXC>
__device__ __forceinline__ void tail_up(const TailLevel& L, const int32_t* coff, PB b, PX x, PXC xc) {
  const GP<T> pv = TailOps<T>::pval(L);
  const GP<int32_t> agg = gptr(L.agg);
  for (int32_t k = threadIdx.x; k < L.n; k += TAIL_THREADS) x[k] = fma(pv ? pv[k] : (T)1, xc[agg[k]], x[k]);
  __syncthreads();
  tail_gs<T>(L, coff, b, x, false);
}

template <typename T, typename PB, typename PX, typename PR, typename PBC, typename PXC>
__device__ __forceinline__ void tail_visit(bool down, const TailLevel& L, const int32_t* coff, PB b, PX x, PR r,
                                           PBC bc, PXC xc, int32_t nc, GP<T> Cd) {
  if (down) tail_down<T>(L, coff, b, x, r, bc, xc, nc, Cd);
  else tail_up<T>(L, coff, b, x, xc);
}

// dense coarsest solve (same order as ldlt_solve_kernel), result in x
template <typename T>
__device__ __forceinline__ void tail_coarsest(const TailDesc& D, const double* Lf, const T* b, T* x, double* acc,
                                              double* mu) {
  const int32_t n = D.cn, m = D.cm;
  const GP<double> Dg = gptr(D.D);
  for (int32_t i = threadIdx.x; i < m; i += TAIL_THREADS) acc[i] = (double)b[i];
  __syncthreads();
  for (int32_t k = 0; k < m; ++k) {
    const double yk = acc[k];
    for (int32_t i = k + 1 + threadIdx.x; i < m; i += TAIL_THREADS) acc[i] = fma(-Lf[(size_t)i * m + k], yk, acc[i]);
    __syncthreads();
  }
  for (int32_t i = threadIdx.x; i < m; i += TAIL_THREADS) acc[i] = acc[i] / Dg[i];
  __syncthreads();
  for (int32_t k = m - 1; k >= 0; --k) {
    const double xk = acc[k];
    for (int32_t i = threadIdx.x; i < k; i += TAIL_THREADS) acc[i] = fma(-Lf[(size_t)k * m + i], xk, acc[i]);
    __syncthreads();
  }
  if (D.grounded) {
    if (threadIdx.x == 0) {
      acc[n - 1] = 0.0;
      double s = 0.0;
      for (int32_t i = 0; i < n; ++i) s = s + acc[i];
      *mu = s / (double)n;
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += TAIL_THREADS) x[i] = (T)(acc[i] - *mu);
  } else {
    for (int32_t i = threadIdx.x; i < n; i += TAIL_THREADS) x[i] = (T)acc[i];
  }
  __syncthreads();
}

// Stage the colour offsets and (when it fits) the coarsest factor in LDS.
template <typename T>
__device__ __forceinline__ void tail_prologue(const TailDesc& D, double* pool, int32_t* coffs) {
  const int last = D.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const TailLevel& L = D.lv[l];
    const GP<int32_t> cf = gptr(L.coff);
    for (int32_t c = threadIdx.x; c <= L.ncol; c += TAIL_THREADS) coffs[L.ocoff + c] = cf[c];
  }
  const int32_t oL = TailOps<T>::oL(D);
  if (oL >= 0) {
    const GP<double> Lg = gptr(D.L);
    for (int32_t i = threadIdx.x; i < D.cm * D.cm; i += TAIL_THREADS) pool[oL + i] = Lg[i];
  }
}

// One cycle from tail level 0 to the coarsest: gamma recursive calls per level
// (one when the next level is the coarsest), iteratively; bit l of `again`
// records that level l still owes its second call (gamma <= 2).  Level 0's
// vectors are b0/x0 when they are not in LDS; the other levels outside LDS
// use their global vectors displaced by boff elements (a per-workgroup copy).
template <typename T>
__device__ __forceinline__ void tail_body(const TailDesc& D, double* pool, const int32_t* coffs, GP<T> b0, GW<T> x0,
                                          size_t boff, int gamma, double* mu) {
  T* V = reinterpret_cast<T*>(pool);
  const int last = D.nlev - 1;  // coarsest, relative index
  const int32_t oL = TailOps<T>::oL(D);
  const double* Lf = oL >= 0 ? pool + oL : D.L;
  double* acc = pool + TailOps<T>::oacc(D);
  uint64_t again = 0;
  int l = 0;
  int ph = 0;  // 0: descend into l, 1: returning to l from its child
  while (l >= 0) {
    const TailLevel& L = D.lv[l];
    if (l == last) {  // the coarsest level's vectors are always in LDS
      tail_coarsest<T>(D, Lf, V + TailOps<T>::off(L, 1), V + TailOps<T>::off(L, 0), acc, mu);
      --l;
      ph = 1;
      continue;
    }
    if (ph == 1 && (again & (1ull << l))) {  // second call continues from the child's current x
      again &= ~(1ull << l);
      ++l;
      ph = 0;
      continue;
    }
    const TailLevel& N = D.lv[l + 1];
    const int32_t* coff = coffs + L.ocoff;
    const bool down = ph == 0;
    // both sub-cycles of the child at once through the inner dense operator
    const bool dense = down && gamma > 1 && l + 1 == D.dense_rel && l + 1 < last;
    const GP<T> Cd = dense ? TailOps<T>::C(D) : (GP<T>)nullptr;
    if (L.lds) {
      tail_visit<T>(down, L, coff, (const T*)(V + TailOps<T>::off(L, 1)), V + TailOps<T>::off(L, 0),
                    V + TailOps<T>::off(L, 2), V + TailOps<T>::off(N, 1), V + TailOps<T>::off(N, 0), N.n, Cd);
    } else {
      const GP<T> b = l == 0 ? b0 : (GP<T>)(TailOps<T>::gb(L) + boff);
      const GW<T> x = l == 0 ? x0 : TailOps<T>::gx(L) + boff;
      const GW<T> r = TailOps<T>::gr(L) + boff;
      if (N.lds)
        tail_visit<T>(down, L, coff, b, x, r, V + TailOps<T>::off(N, 1), V + TailOps<T>::off(N, 0), N.n, Cd);
      else
        tail_visit<T>(down, L, coff, b, x, r, TailOps<T>::gb(N) + boff, TailOps<T>::gx(N) + boff, N.n, Cd);
    }
    if (dense) {  // stay at l as if returning from the child's second call
      again &= ~(1ull << l);
      ph = 1;
    } else if (down) {
      if (gamma > 1 && l + 1 < last) again |= 1ull << l;
      else again &= ~(1ull << l);
      ++l;
    } else {
      --l;
    }
  }
}

// Touches one word per 128-byte line of n 4-byte words, so that the steps
// that follow find the array in this XCD's L2 instead of waiting on HBM at
// every dependent load; returns an xor of the words (kept by the caller).
__device__ __forceinline__ uint32_t touch_lines(const void* p, size_t n) {
  uint32_t acc = 0;
  if (!p) return acc;
  const GP<uint32_t> q = gptr(static_cast<const uint32_t*>(p));  // within [p, p + 4n)
  for (size_t i = (size_t)threadIdx.x * 32; i < n; i += (size_t)TAIL_THREADS * 32) acc ^= q[i];
  return acc;
}

// Warm L2 with the matrices and transfer arrays of the tail levels (a few
// hundred KB): each colour step is a short chain of dependent loads, so a cold
// line costs a full memory round trip per step.
template <typename T>
__device__ __forceinline__ uint32_t tail_warm(const TailDesc& D) {
  uint32_t acc = 0;
  const int last = D.nlev - 1;
  const size_t w = sizeof(T) / 4;
  const bool f64 = sizeof(T) == 8;
  for (int l = 0; l < last; ++l) {
    const TailLevel& L = D.lv[l];
    const size_t nnz = (size_t)L.nnz;
    acc ^= touch_lines(L.rp, (size_t)L.n + 1);
    acc ^= touch_lines(L.ci, nnz);
    acc ^= touch_lines(f64 ? (const void*)L.av : (const void*)L.av32, nnz * w);
    acc ^= touch_lines(f64 ? (const void*)L.d : (const void*)L.d32, (size_t)L.n * w);
    acc ^= touch_lines(f64 ? (const void*)L.dinv : (const void*)L.dinv32, (size_t)L.n * w);
    acc ^= touch_lines(f64 ? (const void*)L.pval : (const void*)L.pval32, (size_t)L.n * w);
    acc ^= touch_lines(L.agg, (size_t)L.n);
    acc ^= touch_lines(L.mem, (size_t)L.n);
    acc ^= touch_lines(L.moff, (size_t)D.lv[l + 1].n + 1);
  }
  return acc;
}

// One cycle of the tail on (b0, x0) in global memory.
template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS) tail_kernel(const TailDesc* __restrict__ Dp, const T* __restrict__ b0,
                                                             T* __restrict__ x0, int gamma) {
  __shared__ double pool[TAIL_LDS_BYTES / 8];
  __shared__ int32_t coffs[TAIL_COFF_MAX];
  __shared__ double mu;
  __shared__ uint32_t sink;
  const TailDesc& D = *Dp;
  T* V = reinterpret_cast<T*>(pool);
  const uint32_t warm = tail_warm<T>(D);
  if (threadIdx.x == 0) sink = warm;  // keeps the warming loads
  tail_prologue<T>(D, pool, coffs);
  const TailLevel& L0 = D.lv[0];
  if (L0.lds) {
    T* xs = V + TailOps<T>::off(L0, 0);
    T* bs = V + TailOps<T>::off(L0, 1);
    for (int32_t i = threadIdx.x; i < L0.n; i += TAIL_THREADS) {
      xs[i] = x0[i];
      bs[i] = b0[i];
    }
  }
  __syncthreads();
  tail_body<T>(D, pool, coffs, gptr(b0), gptr_w(x0), 0, gamma, &mu);
  if (L0.lds) {
    const T* xs = V + TailOps<T>::off(L0, 0);
    for (int32_t i = threadIdx.x; i < L0.n; i += TAIL_THREADS) x0[i] = xs[i];
  }
}

// Columns of the operator that two consecutive W-cycles of the tail apply to
// b from x = 0 (what the level above the tail does with gamma = 2): workgroup
// w takes columns w, w + gridDim.x, ..., runs the two cycles on the unit
// vector and stores x as column j of C (column-major, n0 x n0).  Tail levels
// outside LDS use the per-workgroup copies at boff = w * gstride.
template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS)
    tail_dense_kernel(const TailDesc* __restrict__ Dp, T* __restrict__ C, size_t gstride) {
  __shared__ double pool[TAIL_LDS_BYTES / 8];
  __shared__ int32_t coffs[TAIL_COFF_MAX];
  __shared__ double mu;
  const TailDesc& D = *Dp;
  T* V = reinterpret_cast<T*>(pool);
  tail_prologue<T>(D, pool, coffs);
  const TailLevel& L0 = D.lv[0];
  const int32_t n0 = L0.n;
  const size_t boff = (size_t)blockIdx.x * gstride;
  T* xs = L0.lds ? V + TailOps<T>::off(L0, 0) : nullptr;
  T* bs = L0.lds ? V + TailOps<T>::off(L0, 1) : nullptr;
  const GW<T> xg = TailOps<T>::gx(L0) + boff;
  const GW<T> bg = TailOps<T>::gb(L0) + boff;
  for (int32_t j = blockIdx.x; j < n0; j += gridDim.x) {
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n0; i += TAIL_THREADS) {
      if (L0.lds) {
        xs[i] = 0;
        bs[i] = i == j ? (T)1 : (T)0;
      } else {
        xg[i] = 0;
        bg[i] = i == j ? (T)1 : (T)0;
      }
    }
    __syncthreads();
    tail_body<T>(D, pool, coffs, (GP<T>)bg, xg, boff, 2, &mu);
    tail_body<T>(D, pool, coffs, (GP<T>)bg, xg, boff, 2, &mu);
    for (int32_t i = threadIdx.x; i < n0; i += TAIL_THREADS) C[(size_t)j * n0 + i] = L0.lds ? xs[i] : xg[i];
  }
}

// ---------------------------------------------------------------------------
// Multi-column construction of the dense operator: each workgroup carries
// DMC_K unit vectors through the tail recursion at once.  Vectors of the
// non-coarsest levels are rows of DMC_K values in per-workgroup global scratch,
// the coarsest level's in LDS; every (row, column) item follows exactly the
// single-vector arithmetic and order, so each column equals the one-vector
// construction bit for bit while the step latency is shared by DMC_K columns.
// ---------------------------------------------------------------------------
constexpr int DMC_K = 8;
// Threads per workgroup of the construction: with the LDS sized to what the
// coarsest level needs, several workgroups share a CU (the steps are
// latency-bound, so more resident workgroups means more columns in flight).
constexpr int DMC_THREADS = 512;

// One row of a row-major n x DMC_K block (the DMC_K columns' values of a
// vertex) moved as 16-byte vectors: every block starts at a multiple of DMC_K
// elements of an allocation aligned to 256 bytes (global scratch) or of the
// 16-byte aligned LDS pool, so every row is 16-byte aligned.
template <typename T>
struct Row4;
template <>
struct Row4<float> {
  typedef float v __attribute__((ext_vector_type(4)));
};
template <>
struct Row4<double> {
  typedef double v __attribute__((ext_vector_type(4)));
};

template <typename T, typename P>
__device__ __forceinline__ void ld_row(P p, T (&v)[DMC_K]) {
  typedef typename Row4<T>::v V;
  typedef typename std::conditional<std::is_same<P, GP<T>>::value || std::is_same<P, GW<T>>::value,
                                    const PCAMG_GLOBAL V*, const V*>::type VP;
  const VP q = (VP)p;
#pragma unroll
  for (int h = 0; h < DMC_K / 4; ++h) {
    const V t = q[h];
    v[4 * h] = t.x;
    v[4 * h + 1] = t.y;
    v[4 * h + 2] = t.z;
    v[4 * h + 3] = t.w;
  }
}

template <typename T, typename P>
__device__ __forceinline__ void st_row(P p, const T (&v)[DMC_K]) {
  typedef typename Row4<T>::v V;
  typedef typename std::conditional<std::is_same<P, GW<T>>::value, PCAMG_GLOBAL V*, V*>::type VP;
  VP q = (VP)p;
#pragma unroll
  for (int h = 0; h < DMC_K / 4; ++h) {
    V t;
    t.x = v[4 * h];
    t.y = v[4 * h + 1];
    t.z = v[4 * h + 2];
    t.w = v[4 * h + 3];
    q[h] = t;
  }
}

// The DMC_K fma chains of a CSR row against the columns of a row-major
// n x DMC_K block at once: one index and value load per entry feeds DMC_K
// independent chains, each in CSR order as row_chain1 (so each column's sum is
// the single-vector one bit for bit).  Entries past the row end load row 0
// (in bounds) and are not summed.
template <typename T, typename PX>
__device__ __forceinline__ void chain_rows_mc(int32_t k0, int32_t k1, GP<int32_t> ci, GP<T> av, PX x,
                                              T (&s)[DMC_K]) {
  constexpr int U = sizeof(T) == 8 ? 2 : 4;  // gathered values stay in registers
  for (int32_t k = k0; k < k1; k += U) {
    int32_t c[U];
    T a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = k + u < k1 ? ci[k + u] : 0;
      a[u] = k + u < k1 ? av[k + u] : (T)0;
    }
    T v[U][DMC_K];
#pragma unroll
    for (int u = 0; u < U; ++u) ld_row<T>(x + (size_t)c[u] * DMC_K, v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k + u < k1)
#pragma unroll
        for (int j = 0; j < DMC_K; ++j) s[j] = fma(a[u], v[u][j], s[j]);
  }
}

template <typename T>
__device__ __forceinline__ void gs_mc(const TailLevel& L, const int32_t* coff, GW<T> b, GW<T> x, bool forward) {
  const GP<T> av = TailOps<T>::av(L), dinv = TailOps<T>::dinv(L);
  const GP<int32_t> rp = gptr(L.rp), ci = gptr(L.ci);
  for (int t = 0; t < L.ncol; ++t) {
    const int c = forward ? t : L.ncol - 1 - t;
    for (int32_t i = coff[c] + threadIdx.x; i < coff[c + 1]; i += DMC_THREADS) {
      T s[DMC_K], bi[DMC_K];
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = 0;
      chain_rows_mc<T>(rp[i], rp[i + 1], ci, av, (GP<T>)x, s);
      ld_row<T>(b + (size_t)i * DMC_K, bi);
      const T di = dinv[i];
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = (bi[j] - s[j]) * di;
      st_row<T>(x + (size_t)i * DMC_K, s);
    }
    __syncthreads();
  }
}

// pre-smoothing, residual, restriction into the child (bc, xc: LDS pointers
// for the coarsest child, else global), optionally the inner dense product
template <typename T, typename PC>
__device__ __forceinline__ void down_mc(const TailLevel& L, const int32_t* coff, GW<T> b, GW<T> x, GW<T> r, PC bc,
                                        PC xc, int32_t nc, GP<T> Cd) {
  gs_mc<T>(L, coff, b, x, true);
  {
    const GP<T> av = TailOps<T>::av(L), d = TailOps<T>::d(L);
    const GP<int32_t> rp = gptr(L.rp), ci = gptr(L.ci);
    for (int32_t i = threadIdx.x; i < L.n; i += DMC_THREADS) {
      T s[DMC_K], bi[DMC_K];
      ld_row<T>(x + (size_t)i * DMC_K, s);
      const T di = d[i];
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = di * s[j];
      chain_rows_mc<T>(rp[i], rp[i + 1], ci, av, (GP<T>)x, s);
      ld_row<T>(b + (size_t)i * DMC_K, bi);
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = bi[j] - s[j];
      st_row<T>(r + (size_t)i * DMC_K, s);
    }
    __syncthreads();
  }
  const GP<T> pv = TailOps<T>::pval(L);
  const GP<int32_t> moff = gptr(L.moff), mem = gptr(L.mem);
  for (int32_t q = threadIdx.x; q < nc; q += DMC_THREADS) {
    T s[DMC_K], z[DMC_K];
#pragma unroll
    for (int j = 0; j < DMC_K; ++j) s[j] = z[j] = 0;
    for (int32_t t = moff[q]; t < moff[q + 1]; ++t) {
      const int32_t k = mem[t];
      const T p = pv ? pv[k] : (T)1;
      T rk[DMC_K];
      ld_row<T>((GP<T>)r + (size_t)k * DMC_K, rk);
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = fma(p, rk[j], s[j]);
    }
    st_row<T>(bc + (size_t)q * DMC_K, s);
    st_row<T>(xc + (size_t)q * DMC_K, z);
  }
  __syncthreads();
  if (Cd) {
    for (int32_t i = threadIdx.x; i < nc; i += DMC_THREADS) {
      T s[DMC_K];
#pragma unroll
      for (int j = 0; j < DMC_K; ++j) s[j] = 0;
      // column entries of row i loaded eight ahead of the fma chains
      constexpr int U = 8;
      int32_t m = 0;
      for (; m + U <= nc; m += U) {
        T cm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cm[u] = Cd[(size_t)(m + u) * nc + i];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          T bm[DMC_K];
          ld_row<T>(bc + (size_t)(m + u) * DMC_K, bm);
#pragma unroll
          for (int j = 0; j < DMC_K; ++j) s[j] = fma(cm[u], bm[j], s[j]);
        }
      }
      for (; m < nc; ++m) {
        const T cmi = Cd[(size_t)m * nc + i];
        T bm[DMC_K];
        ld_row<T>(bc + (size_t)m * DMC_K, bm);
#pragma unroll
        for (int j = 0; j < DMC_K; ++j) s[j] = fma(cmi, bm[j], s[j]);
      }
      st_row<T>(xc + (size_t)i * DMC_K, s);
    }
    __syncthreads();
  }
}

template <typename T, typename PC>
__device__ __forceinline__ void up_mc(const TailLevel& L, const int32_t* coff, GW<T> b, GW<T> x, PC xc) {
  const GP<T> pv = TailOps<T>::pval(L);
  const GP<int32_t> agg = gptr(L.agg);
  for (int32_t k = threadIdx.x; k < L.n; k += DMC_THREADS) {
    const T p = pv ? pv[k] : (T)1;
    T xk[DMC_K], cq[DMC_K];
    ld_row<T>(x + (size_t)k * DMC_K, xk);
    ld_row<T>(xc + (size_t)agg[k] * DMC_K, cq);
#pragma unroll
    for (int j = 0; j < DMC_K; ++j) xk[j] = fma(p, cq[j], xk[j]);
    st_row<T>(x + (size_t)k * DMC_K, xk);
  }
  __syncthreads();
  gs_mc<T>(L, coff, b, x, false);
}

// dense coarsest solve per column (the order of tail_coarsest)
template <typename T>
__device__ __forceinline__ void coarsest_mc(const TailDesc& D, const double* Lf, const T* b, T* x, double* acc,
                                            double* mu) {
  const int32_t n = D.cn, m = D.cm;
  const GP<double> Dg = gptr(D.D);
  for (int32_t it = threadIdx.x; it < m * DMC_K; it += DMC_THREADS) acc[it] = (double)b[it];
  __syncthreads();
  for (int32_t k = 0; k < m; ++k) {
    for (int32_t it = threadIdx.x; it < (m - k - 1) * DMC_K; it += DMC_THREADS) {
      const int32_t i = k + 1 + it / DMC_K, j = it % DMC_K;
      acc[i * DMC_K + j] = fma(-Lf[(size_t)i * m + k], acc[k * DMC_K + j], acc[i * DMC_K + j]);
    }
    __syncthreads();
  }
  for (int32_t it = threadIdx.x; it < m * DMC_K; it += DMC_THREADS) acc[it] = acc[it] / Dg[it / DMC_K];
  __syncthreads();
  for (int32_t k = m - 1; k >= 0; --k) {
    for (int32_t it = threadIdx.x; it < k * DMC_K; it += DMC_THREADS) {
      const int32_t i = it / DMC_K, j = it % DMC_K;
      acc[i * DMC_K + j] = fma(-Lf[(size_t)k * m + i], acc[k * DMC_K + j], acc[i * DMC_K + j]);
    }
    __syncthreads();
  }
  if (D.grounded) {
    if (threadIdx.x < DMC_K) {
      const int j = threadIdx.x;
      acc[(n - 1) * DMC_K + j] = 0.0;
      double sum = 0.0;
      for (int32_t i = 0; i < n; ++i) sum = sum + acc[i * DMC_K + j];
      mu[j] = sum / (double)n;
    }
    __syncthreads();
    for (int32_t it = threadIdx.x; it < n * DMC_K; it += DMC_THREADS) x[it] = (T)(acc[it] - mu[it % DMC_K]);
  } else {
    for (int32_t it = threadIdx.x; it < n * DMC_K; it += DMC_THREADS) x[it] = (T)acc[it];
  }
  __syncthreads();
}

// One cycle of the multi-column tail (gamma = 2 recursion with the optional
// inner dense operator), level 0's vectors in global memory at boff.
template <typename T>
__device__ __forceinline__ void body_mc(const TailDesc& D, T* cx, T* cb, const int32_t* coffs, const double* Lf,
                                        double* acc, double* mu, size_t boff) {
  const int last = D.nlev - 1;
  uint64_t again = 0;
  int l = 0, ph = 0;
  while (l >= 0) {
    const TailLevel& L = D.lv[l];
    if (l == last) {
      coarsest_mc<T>(D, Lf, cb, cx, acc, mu);
      --l;
      ph = 1;
      continue;
    }
    if (ph == 1 && (again & (1ull << l))) {
      again &= ~(1ull << l);
      ++l;
      ph = 0;
      continue;
    }
    const TailLevel& N = D.lv[l + 1];
    const int32_t* coff = coffs + L.ocoff;
    const bool down = ph == 0;
    const bool dense = down && l + 1 == D.dense_rel && l + 1 < last;
    const GP<T> Cd = dense ? TailOps<T>::C(D) : (GP<T>)nullptr;
    const GW<T> b = TailOps<T>::gb(L) + boff, x = TailOps<T>::gx(L) + boff, r = TailOps<T>::gr(L) + boff;
    if (l + 1 == last) {
      if (down) down_mc<T>(L, coff, b, x, r, cb, cx, N.n, Cd);
      else up_mc<T>(L, coff, b, x, (const T*)cx);
    } else {
      const GW<T> nb = TailOps<T>::gb(N) + boff, nx = TailOps<T>::gx(N) + boff;
      if (down) down_mc<T>(L, coff, b, x, r, nb, nx, N.n, Cd);
      else up_mc<T>(L, coff, b, x, (GP<T>)nx);
    }
    if (dense) {
      again &= ~(1ull << l);
      ph = 1;
    } else if (down) {
      if (l + 1 < last) again |= 1ull << l;
      else again &= ~(1ull << l);
      ++l;
    } else {
      --l;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(DMC_THREADS)
    tail_dense_mc_kernel(const TailDesc* __restrict__ Dp, T* __restrict__ C, size_t gstride) {
  extern __shared__ __attribute__((aligned(16))) double pool[];  // dense_mc_lds_bytes(cn, cm, sizeof(T))
  __shared__ int32_t coffs[TAIL_COFF_MAX];
  __shared__ double mu[DMC_K];
  const TailDesc& D = *Dp;
  const int last = D.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const TailLevel& L = D.lv[l];
    const GP<int32_t> cf = gptr(L.coff);
    for (int32_t c = threadIdx.x; c <= L.ncol; c += DMC_THREADS) coffs[L.ocoff + c] = cf[c];
  }
  // LDS: coarsest x and b (cn x K of T), accumulator (cn x K doubles: the
  // grounded solve sets its last row), factor (cm x cm)
  const int32_t cn = D.cn, cm = D.cm;
  T* cx = reinterpret_cast<T*>(pool);
  T* cb = cx + (size_t)cn * DMC_K;
  const size_t tb = ((size_t)2 * cn * DMC_K * sizeof(T) + 7) / 8;
  double* acc = pool + tb;
  const bool lds_L = cm <= 64;
  if (lds_L) {
    const GP<double> Lg = gptr(D.L);
    for (int32_t i = threadIdx.x; i < cm * cm; i += DMC_THREADS) pool[tb + (size_t)cn * DMC_K + i] = Lg[i];
  }
  const double* Lf = lds_L ? pool + tb + (size_t)cn * DMC_K : D.L;
  const TailLevel& L0 = D.lv[0];
  const int32_t n0 = L0.n;
  const size_t boff = (size_t)blockIdx.x * gstride;
  const GW<T> x0 = TailOps<T>::gx(L0) + boff, b0 = TailOps<T>::gb(L0) + boff;
  for (int32_t j0 = blockIdx.x * DMC_K; j0 < n0; j0 += gridDim.x * DMC_K) {
    __syncthreads();
    for (int32_t it = threadIdx.x; it < n0 * DMC_K; it += DMC_THREADS) {
      const int32_t i = it / DMC_K, j = it % DMC_K;
      x0[it] = 0;
      b0[it] = i == j0 + j ? (T)1 : (T)0;
    }
    __syncthreads();
    body_mc<T>(D, cx, cb, coffs, Lf, acc, mu, boff);
    body_mc<T>(D, cx, cb, coffs, Lf, acc, mu, boff);
    for (int32_t it = threadIdx.x; it < n0 * DMC_K; it += DMC_THREADS) {
      const int32_t i = it % n0, j = it / n0;  // coalesced over i in C
      if (j0 + j < n0) C[(size_t)(j0 + j) * n0 + i] = x0[(size_t)i * DMC_K + j];
    }
  }
}

// LDS bytes the multi-column construction needs for the coarsest level
size_t dense_mc_lds_bytes(int32_t cn, int32_t cm, size_t tsize) {
  return ((size_t)2 * cn * DMC_K * tsize + 7) / 8 * 8 + (size_t)cn * DMC_K * 8 + (cm <= 64 ? (size_t)cm * cm * 8 : 0);
}

int dense_mc_columns() { return DMC_K; }

int dense_mc_threads() { return DMC_THREADS; }

template <typename T>
void tail_dense_mc(const TailDesc* desc, int blocks, T* C, size_t gstride, size_t lds, hipStream_t s) {
  require(lds <= (size_t)TAIL_LDS_BYTES, PCAMG_EINVAL, "dense construction LDS exceeds the pool size");
  PCAMG_HIP(hipFuncSetAttribute((const void*)tail_dense_mc_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
  tail_dense_mc_kernel<T><<<blocks, DMC_THREADS, lds, s>>>(desc, C, gstride);
  PCAMG_LAUNCHED();
}
template void tail_dense_mc<double>(const TailDesc*, int, double*, size_t, size_t, hipStream_t);
template void tail_dense_mc<float>(const TailDesc*, int, float*, size_t, size_t, hipStream_t);

void tail_cycle64(const Hierarchy& H, const double* b, double* x, int gamma, hipStream_t s) {
  tail_kernel<double><<<1, TAIL_THREADS, 0, s>>>(H.tail_desc.p, b, x, gamma);
  PCAMG_LAUNCHED();
}

void tail_cycle32(const Hierarchy& H, const float* b, float* x, int gamma, hipStream_t s) {
  tail_kernel<float><<<1, TAIL_THREADS, 0, s>>>(H.tail_desc.p, b, x, gamma);
  PCAMG_LAUNCHED();
}

template <typename T>
void tail_dense(const TailDesc* desc, int32_t n0, int blocks, T* C, size_t gstride, hipStream_t s) {
  tail_dense_kernel<T><<<blocks, TAIL_THREADS, 0, s>>>(desc, C, gstride);
  PCAMG_LAUNCHED();
}
template void tail_dense<double>(const TailDesc*, int32_t, int, double*, size_t, hipStream_t);
template void tail_dense<float>(const TailDesc*, int32_t, int, float*, size_t, hipStream_t);

// y = C b for a column-major n x n matrix: the columns are split into chunks
// of DENSE_CHUNK; block (row tile, chunk) writes the partial sums of its chunk
// (fma chain in column order), and a second pass adds the chunks in order.
constexpr int DENSE_CHUNK = 128;
template <typename T>
__global__ void __launch_bounds__(256) dense_part_kernel(int32_t n, const T* __restrict__ C, const T* __restrict__ b,
                                                         T* __restrict__ part) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  const int32_t c = blockIdx.y;
  const int32_t j0 = c * DENSE_CHUNK, j1 = min(n, j0 + DENSE_CHUNK);
  __shared__ T bj[DENSE_CHUNK];
  for (int32_t j = j0 + threadIdx.x; j < j1; j += 256) bj[j - j0] = b[j];
  __syncthreads();
  if (i >= n) return;
  // the chunk's column entries loaded sixteen ahead of the fma chain
  constexpr int U = 16;
  T s = 0;
  int32_t j = j0;
  for (; j + U <= j1; j += U) {
    T cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cv[u] = C[(size_t)(j + u) * n + i];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(cv[u], bj[j + u - j0], s);
  }
  for (; j < j1; ++j) s = fma(C[(size_t)j * n + i], bj[j - j0], s);
  part[(size_t)c * n + i] = s;
}
template <typename T>
__global__ void dense_sum_kernel(int32_t n, int32_t nchunk, const T* __restrict__ part, T* __restrict__ y) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = 0;
  for (int32_t c = 0; c < nchunk; ++c) s = s + part[(size_t)c * n + i];
  y[i] = s;
}

template <typename T>
void dense_apply(int32_t n, const T* C, const T* b, T* part, T* y, hipStream_t s) {
  const int32_t nchunk = (n + DENSE_CHUNK - 1) / DENSE_CHUNK;
  dense_part_kernel<T><<<dim3((n + 255) / 256, nchunk), 256, 0, s>>>(n, C, b, part);
  PCAMG_LAUNCHED();
  dense_sum_kernel<T><<<(n + 255) / 256, 256, 0, s>>>(n, nchunk, part, y);
  PCAMG_LAUNCHED();
}
template void dense_apply<double>(int32_t, const double*, const double*, double*, double*, hipStream_t);
template void dense_apply<float>(int32_t, const float*, const float*, float*, float*, hipStream_t);

int32_t dense_chunks(int32_t n) { return (n + DENSE_CHUNK - 1) / DENSE_CHUNK; }

}  // namespace pcamg
