// Tail of a multigrid cycle in one workgroup.  The small levels of a
// hierarchy (and the dense coarsest solve) are visited many times per cycle --
// 2^l times in a W-cycle -- and each visit of a multicoloured level is a long
// chain of tiny steps.  Here the whole sub-cycle from the first small level
// down to the coarsest runs in a single launch of 1024 threads, with a
// workgroup barrier between dependent steps.  The vectors of the smaller
// levels sit in LDS for the launch (the larger ones stay in global memory),
// and the matrices are pulled into L2 at the start.  Every row and every sum uses the
// same arithmetic and order as the per-step kernels, so results are identical
// bit for bit.
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

// pre-smoothing, residual, restriction; the child's x starts at zero
template <typename T, typename PB, typename PX, typename PR, typename PBC, typename PXC>
__device__ __forceinline__ void tail_down(const TailLevel& L, const int32_t* coff, PB b, PX x, PR r, PBC bc, PXC xc,
                                          int32_t nc) {
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
                                           PBC bc, PXC xc, int32_t nc) {
  if (down) tail_down<T>(L, coff, b, x, r, bc, xc, nc);
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
// use their global vectors.
template <typename T>
__device__ __forceinline__ void tail_body(const TailDesc& D, double* pool, const int32_t* coffs, GP<T> b0, GW<T> x0,
                                          int gamma, double* mu) {
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
    if (L.lds) {
      tail_visit<T>(down, L, coff, (const T*)(V + TailOps<T>::off(L, 1)), V + TailOps<T>::off(L, 0),
                    V + TailOps<T>::off(L, 2), V + TailOps<T>::off(N, 1), V + TailOps<T>::off(N, 0), N.n);
    } else {
      const GP<T> b = l == 0 ? b0 : (GP<T>)TailOps<T>::gb(L);
      const GW<T> x = l == 0 ? x0 : TailOps<T>::gx(L);
      const GW<T> r = TailOps<T>::gr(L);
      if (N.lds)
        tail_visit<T>(down, L, coff, b, x, r, V + TailOps<T>::off(N, 1), V + TailOps<T>::off(N, 0), N.n);
      else
        tail_visit<T>(down, L, coff, b, x, r, TailOps<T>::gb(N), TailOps<T>::gx(N), N.n);
    }
    if (down) {
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
  tail_body<T>(D, pool, coffs, gptr(b0), gptr_w(x0), gamma, &mu);
  if (L0.lds) {
    const T* xs = V + TailOps<T>::off(L0, 0);
    for (int32_t i = threadIdx.x; i < L0.n; i += TAIL_THREADS) x0[i] = xs[i];
  }
}

void tail_cycle64(const Hierarchy& H, const double* b, double* x, int gamma, hipStream_t s) {
  tail_kernel<double><<<1, TAIL_THREADS, 0, s>>>(H.tail_desc.p, b, x, gamma);
  PCAMG_LAUNCHED();
}

void tail_cycle32(const Hierarchy& H, const float* b, float* x, int gamma, hipStream_t s) {
  tail_kernel<float><<<1, TAIL_THREADS, 0, s>>>(H.tail_desc.p, b, x, gamma);
  PCAMG_LAUNCHED();
}


// y = C b for a column-major n x n matrix: the columns are split into chunks
// of DENSE_CHUNK; block (row tile, chunk) writes the partial sums of its chunk
// (fma chain in column order), and a second pass adds the chunks in order.
constexpr int DENSE_CHUNK = 64;
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
__global__ void dense_sum_kernel(int32_t n, int32_t nchunk, const T* __restrict__ part, T* __restrict__ y,
                                 int add) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = 0;
  for (int32_t c = 0; c < nchunk; ++c) s = s + part[(size_t)c * n + i];
  y[i] = add ? y[i] + s : s;
}

template <typename T>
void dense_apply(int32_t n, const T* C, const T* b, T* part, T* y, hipStream_t s, bool add) {
  const int32_t nchunk = (n + DENSE_CHUNK - 1) / DENSE_CHUNK;
  dense_part_kernel<T><<<dim3((n + 255) / 256, nchunk), 256, 0, s>>>(n, C, b, part);
  PCAMG_LAUNCHED();
  dense_sum_kernel<T><<<(n + 255) / 256, 256, 0, s>>>(n, nchunk, part, y, add ? 1 : 0);
  PCAMG_LAUNCHED();
}
template void dense_apply<double>(int32_t, const double*, const double*, double*, double*, hipStream_t, bool);
template void dense_apply<float>(int32_t, const float*, const float*, float*, float*, hipStream_t, bool);

int32_t dense_chunks(int32_t n) { return (n + DENSE_CHUNK - 1) / DENSE_CHUNK; }

}  // namespace pcamg
