// Bottom-up construction of the dense W operator.
//
// With gamma = 2 the level above the dense region d calls the cycle of level d
// twice from x = 0: a fixed linear map 2 W_d - W_d A_d W_d of its right-hand
// side, W_d the operator of one call (dense_apply applies it).  Instead of
// running that recursion on every unit vector, the operator of every level l
// of the region is built from the one of level l + 1 as a matrix, all columns
// at once:
//
//   Z        = coarsest solve applied to the identity (FP64, as the cycle does it)
//   C_{l+1}  = Z                       if l + 1 is the coarsest level (one call)
//            = 2 W_{l+1} - W_{l+1} A_{l+1} W_{l+1}   otherwise (second call
//              starts from the first one's result: x1 = x0 + W (b - A x0))
//   W_l      = S_bwd o (I + P C_{l+1} P^T (.. residual ..)) o S_fwd on the
//              identity: forward colour passes from X = 0, R = I - A X,
//              B_c = P^T R, X += P (C_{l+1} B_c), backward colour passes.
//
// The residuals and transfers are the cycle's own row formulas (fma chains
// in CSR / member order) evaluated for all columns; the colour passes sum a
// row in sixteen strided parts added by a fixed tree; the two products with
// dense matrices are GEMMs on the matrix cores (this file's MFMA kernel).
// The result is the same linear map as the recursion with a different
// rounding order.
#include "rowchain.hpp"
#include "solver.hpp"

namespace pcamg {
namespace {

// ---------------------------------------------------------------------------
// Dense GEMM on the matrix cores: P = alpha Q R + beta P, all row-major
// (P: p x r, Q: p x q, R: q x r, each with its column count as stride).
// A workgroup of four wavefronts (2 x 2) computes a BM x BN tile of P; each
// wavefront a (BM/2) x (BN/2) block of 16 x 16 MFMA tiles
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64, 16 x 4 times 4 x 16 per
// instruction).  K advances in slices of 16 staged through LDS, zero-filled
// past the matrix edges; each thread loads the next slice into registers
// while the matrix cores work on the current one.  Lane l of a 16 x 16 x 4 product supplies A[l % 16][l
// / 16] and B[l / 16][l % 16]; its four results v = 0..3 are D[i][l % 16] with
// i = 4 (l / 16) + v for the FP32 instruction and i = l / 16 + 4 v for the FP64
// one (both layouts checked on the device).
// Each entry of P is accumulated by one lane in a fixed order (K ascending,
// four products per instruction), so the result is the same on every run.
// ---------------------------------------------------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using acc_t = f32x4_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct Mfma<double> {
  using acc_t = f64x4_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

template <typename T, int BM, int BN>
__global__ void __launch_bounds__(256)
    gemm_mfma_kernel(int32_t p, int32_t q, int32_t r, T alpha, const T* __restrict__ Q, int32_t ldq,
                     const T* __restrict__ R, int32_t ldr, T beta, T* __restrict__ P, int32_t ldp) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BK * BN / 256;  // elements each thread stages per slice
  __shared__ T As[BK][BM + 4];  // k-major: a lane's A operand is As[k][row]
  __shared__ T Bs[BK][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int32_t row0 = (int32_t)blockIdx.y * BM, col0 = (int32_t)blockIdx.x * BN;
  typename Mfma<T>::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  const int lr = lane & 15, lk = lane >> 4;
  // the next slice's operands are loaded into registers while the matrix
  // cores work on the current one from LDS
  T ra[LA], rb[LB];
  auto load = [&](int32_t k0) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + 256 * u, i = e / BK, k = e % BK;
      const int32_t gi = row0 + i, gk = k0 + k;
      ra[u] = (gi < p && gk < q) ? Q[(size_t)gi * ldq + gk] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e = tid + 256 * u, k = e / BN, j = e % BN;
      const int32_t gk = k0 + k, gj = col0 + j;
      rb[u] = (gk < q && gj < r) ? R[(size_t)gk * ldr + gj] : (T)0;
    }
  };
  load(0);
  for (int32_t k0 = 0; k0 < q; k0 += BK) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + 256 * u;
      As[e % BK][e / BK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e = tid + 256 * u;
      Bs[e / BN][e % BN] = rb[u];
    }
    __syncthreads();
    if (k0 + BK < q) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) av[a] = As[kk + lk][wm * WM + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < FN; ++b) bv[b] = Bs[kk + lk][wn * WN + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int32_t gi = row0 + wm * WM + a * 16 + Mfma<T>::row(lk, v), gj = col0 + wn * WN + b * 16 + lr;
        if (gi < p && gj < r) {
          const size_t o = (size_t)gi * ldp + gj;
          const T t = alpha * acc[a][b][v];
          P[o] = beta == (T)0 ? t : fma(beta, P[o], t);
        }
      }
}

// Row-major P = alpha Q R + beta P (p x q times q x r), each operand with its
// own row stride (ldq, ldr, ldp elements).  128 x 128 tiles when both sides
// fill them (fewer LDS round trips per product), 64 x 64 otherwise; every
// entry is the same fma sequence over K either way.
template <typename T>
void gemm_strided(int32_t p, int32_t q, int32_t r, T alpha, const T* Q, int32_t ldq, const T* R, int32_t ldr,
                  T beta, T* P, int32_t ldp, hipStream_t s) {
  if (p <= 0 || r <= 0) return;
  if (p >= 128 && r >= 128) {
    const dim3 grid((unsigned)((r + 127) / 128), (unsigned)((p + 127) / 128));
    gemm_mfma_kernel<T, 128, 128><<<grid, 256, 0, s>>>(p, q, r, alpha, Q, ldq, R, ldr, beta, P, ldp);
  } else {
    const dim3 grid((unsigned)((r + 63) / 64), (unsigned)((p + 63) / 64));
    gemm_mfma_kernel<T, 64, 64><<<grid, 256, 0, s>>>(p, q, r, alpha, Q, ldq, R, ldr, beta, P, ldp);
  }
  PCAMG_LAUNCHED();
}

// The same with each operand's column count as its stride.
template <typename T>
void gemm_rows(int32_t p, int32_t q, int32_t r, T alpha, const T* Q, const T* R, T beta, T* P, hipStream_t s) {
  gemm_strided<T>(p, q, r, alpha, Q, q, R, r, beta, P, r, s);
}

// Z[i * n + j] = (coarsest solve of e_j)_i: one workgroup per column, the
// arithmetic and order of the cycle's coarsest solve (FP64 accumulator in
// LDS, n doubles; the grounded solve pins the last vertex and removes the mean).
template <typename T>
__global__ void __launch_bounds__(256)
    coarsest_cols_kernel(int32_t n, int32_t m, int grounded, const double* __restrict__ L,
                         const double* __restrict__ D, T* __restrict__ Z) {
  extern __shared__ double acc[];
  __shared__ double mu;
  const int32_t j = blockIdx.x;
  for (int32_t i = threadIdx.x; i < m; i += blockDim.x) acc[i] = i == j ? 1.0 : 0.0;
  __syncthreads();
  for (int32_t k = 0; k < m; ++k) {
    const double yk = acc[k];
    for (int32_t i = k + 1 + threadIdx.x; i < m; i += blockDim.x) acc[i] = fma(-L[(size_t)i * m + k], yk, acc[i]);
    __syncthreads();
  }
  for (int32_t i = threadIdx.x; i < m; i += blockDim.x) acc[i] = acc[i] / D[i];
  __syncthreads();
  for (int32_t k = m - 1; k >= 0; --k) {
    const double xk = acc[k];
    for (int32_t i = threadIdx.x; i < k; i += blockDim.x) acc[i] = fma(-L[(size_t)k * m + i], xk, acc[i]);
    __syncthreads();
  }
  if (grounded) {
    if (threadIdx.x == 0) {
      acc[n - 1] = 0.0;
      double s = 0.0;
      for (int32_t i = 0; i < n; ++i) s = s + acc[i];
      mu = s / (double)n;
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) Z[(size_t)i * n + j] = (T)(acc[i] - mu);
  } else {
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) Z[(size_t)i * n + j] = (T)acc[i];
  }
}

// sum_e a_e Y[c_e, j] over a CSR row as one fma chain from s, entries loaded
// eight ahead (row-major Y with ld columns; the row's indices and values are
// the same for the whole workgroup)
template <typename T>
__device__ __forceinline__ T row_block_chain(int32_t k0, int32_t k1, const int32_t* __restrict__ ci,
                                             const T* __restrict__ av, const T* __restrict__ Y, size_t ld,
                                             int32_t j, T s) {
  constexpr int U = 8;
  int32_t k = k0;
  for (; k + U <= k1; k += U) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = Y[(size_t)ci[k + u] * ld + j];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(av[k + u], v[u], s);
  }
  for (; k < k1; ++k) s = fma(av[k], Y[(size_t)ci[k] * ld + j], s);
  return s;
}

// One Gauss-Seidel colour pass on all columns, right-hand side the identity:
// X[i, j] = (delta_ij - sum_e a_ie X[c_e, j]) * dinv_i for rows r0 + blockIdx.y.
// A workgroup takes 16 columns; its 16 thread rows sum strided sixteenths of
// the row (the near-dense levels' rows have hundreds to thousands of entries),
// added by a fixed tree in LDS.
template <typename T>
__global__ void __launch_bounds__(256)
    blk_gs_kernel(int32_t r0, int32_t nc, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                  const T* __restrict__ av, const T* __restrict__ dinv, T* __restrict__ X) {
  __shared__ T part[16][17];
  const int32_t i = r0 + (int32_t)blockIdx.y;
  const int tx = (int)(threadIdx.x & 15), ty = (int)(threadIdx.x >> 4);
  const int32_t j = (int32_t)blockIdx.x * 16 + tx;
  T s = (T)0;
  if (j < nc) {
    constexpr int U = 4;
    const int32_t k1 = rp[i + 1];
    int32_t k = rp[i] + ty;
    for (; k + 16 * (U - 1) < k1; k += 16 * U) {
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = X[(size_t)ci[k + 16 * u] * nc + j];
#pragma unroll
      for (int u = 0; u < U; ++u) s = fma(av[k + 16 * u], v[u], s);
    }
    for (; k < k1; k += 16) s = fma(av[k], X[(size_t)ci[k] * nc + j], s);
  }
  part[ty][tx] = s;
  __syncthreads();
#pragma unroll
  for (int h = 8; h > 0; h >>= 1) {
    if (ty < h) part[ty][tx] += part[ty + h][tx];
    __syncthreads();
  }
  if (ty == 0 && j < nc) X[(size_t)i * nc + j] = ((i == j ? (T)1 : (T)0) - part[0][tx]) * dinv[i];
}

// Y = A X (identity = 0) or R = I - A X (identity = 1) on all columns, the
// residual's order (s starts from d_i x_i).
template <typename T>
__global__ void __launch_bounds__(256)
    blk_apply_kernel(int32_t nc, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                     const T* __restrict__ av, const T* __restrict__ d, const T* __restrict__ X, T* __restrict__ Y,
                     int identity) {
  const int32_t i = (int32_t)blockIdx.y;
  const int32_t j = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (j >= nc) return;
  const size_t o = (size_t)i * nc + j;
  const T s = row_block_chain<T>(rp[i], rp[i + 1], ci, av, X, (size_t)nc, j, d[i] * X[o]);
  Y[o] = identity ? (i == j ? (T)1 : (T)0) - s : s;
}

// B_c[q, j] = sum over members k of aggregate q (ascending) of p_k R[k, j]
template <typename T>
__global__ void __launch_bounds__(256)
    blk_restrict_kernel(int32_t nc, const int32_t* __restrict__ moff, const int32_t* __restrict__ mem,
                        const T* __restrict__ pval, const T* __restrict__ R, T* __restrict__ Bc) {
  const int32_t q = (int32_t)blockIdx.y;
  const int32_t j = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (j >= nc) return;
  T s = 0;
  for (int32_t t = moff[q]; t < moff[q + 1]; ++t) {
    const int32_t k = mem[t];
    s = fma(pval ? pval[k] : (T)1, R[(size_t)k * nc + j], s);
  }
  Bc[(size_t)q * nc + j] = s;
}

// X[k, j] += p_k Xc[agg_k, j]
template <typename T>
__global__ void __launch_bounds__(256)
    blk_prolong_kernel(int32_t nc, const int32_t* __restrict__ agg, const T* __restrict__ pval,
                       const T* __restrict__ Xc, T* __restrict__ X) {
  const int32_t k = (int32_t)blockIdx.y;
  const int32_t j = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (j >= nc) return;
  const size_t o = (size_t)k * nc + j;
  X[o] = fma(pval ? pval[k] : (T)1, Xc[(size_t)agg[k] * nc + j], X[o]);
}

// C[j * n + i] = X[i * n + j] through 32 x 32 LDS tiles
template <typename T>
__global__ void __launch_bounds__(256) blk_transpose_kernel(int32_t n, const T* __restrict__ X, T* __restrict__ C) {
  __shared__ T tile[32][33];
  const int32_t bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int32_t r = ty; r < 32; r += 8) {
    const int32_t i = by + r, j = bx + tx;
    if (i < n && j < n) tile[r][tx] = X[(size_t)i * n + j];
  }
  __syncthreads();
  for (int32_t r = ty; r < 32; r += 8) {
    const int32_t j = bx + r, i = by + tx;
    if (i < n && j < n) C[(size_t)j * n + i] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
// Near-dense levels (many colours of a few rows each): a colour pass on all
// columns is a launch per colour, each summing long rows.  There a sweep is
// taken instead as a recursive blocked triangular solve on the dense
// off-diagonal part Ad, in the same row order (the colour order of the
// level, in which rows of one colour do not touch each other).  T (n x n)
// holds for every row the sum of a_ik x_k over the rows k outside its block:
// first the side not yet updated in this sweep (the rows after it in a
// forward sweep, from the old X: one GEMM with the strictly upper part; none
// from X = 0), then, as the recursion finishes the first half of a range,
// the GEMM of that half's new values into the second half's rows.  A leaf of
// GS_NB rows then updates its rows one at a time from T and the block's
// current values -- the Gauss-Seidel update of every row, with the sums in
// another order; the GEMMs near the top of the recursion are large.
// ---------------------------------------------------------------------------
constexpr int GS_NB = 32;

// Ad[i, c_e] = a_e (Ad zero on entry), a workgroup per row.
template <typename T>
__global__ void __launch_bounds__(256)
    blk_densify_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const T* __restrict__ av, T* __restrict__ Ad) {
  const int32_t i = (int32_t)blockIdx.x;
  for (int32_t k = rp[i] + (int32_t)threadIdx.x; k < rp[i + 1]; k += 256) Ad[(size_t)i * n + ci[k]] = av[k];
}

// Lo[i, k] = Ad[i, k] for k < i, else 0 (Upper: k > i)
template <typename T, bool Upper>
__global__ void __launch_bounds__(256) blk_triangle_kernel(int32_t n, const T* __restrict__ Ad, T* __restrict__ Tr) {
  const int32_t i = (int32_t)blockIdx.y;
  const int32_t k = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (k >= n) return;
  const size_t o = (size_t)i * n + k;
  Tr[o] = (Upper ? k > i : k < i) ? Ad[o] : (T)0;
}

// The rows r0 .. r0 + nb - 1 of X, one column per thread, in order
// (forward) or reverse: x_i = (delta(r0 + i, j) - T_i - sum over the
// block's rows already updated in this sweep of a_ik x_k) dinv_i; the block
// of Ad in LDS.
template <typename T, bool Forward>
__global__ void __launch_bounds__(256)
    blk_block_gs_kernel(int32_t n, int32_t r0, int32_t nb, const T* __restrict__ Ad, const T* __restrict__ dinv,
                        const T* __restrict__ Tsum, T* __restrict__ X) {
  __shared__ T ab[GS_NB][GS_NB + 1];
  __shared__ T dv[GS_NB];
  for (int e = (int)threadIdx.x; e < GS_NB * GS_NB; e += 256) {
    const int i = e / GS_NB, k = e % GS_NB;
    ab[i][k] = (i < nb && k < nb) ? Ad[(size_t)(r0 + i) * n + r0 + k] : (T)0;
  }
  if (threadIdx.x < GS_NB) dv[threadIdx.x] = (int)threadIdx.x < nb ? dinv[r0 + threadIdx.x] : (T)0;
  __syncthreads();
  const int32_t j = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (j >= n) return;
  T x[GS_NB];
#pragma unroll
  for (int k = 0; k < GS_NB; ++k) x[k] = k < nb ? X[(size_t)(r0 + k) * n + j] : (T)0;
#pragma unroll
  for (int t = 0; t < GS_NB; ++t) {
    const int i = Forward ? t : GS_NB - 1 - t;
    if (i < nb) {
      T acc = (r0 + i == j ? (T)1 : (T)0) - Tsum[(size_t)(r0 + i) * n + j];
#pragma unroll
      for (int k = 0; k < GS_NB; ++k)
        if (Forward ? k < i : k > i) acc = fma(-ab[i][k], x[k], acc);
      x[i] = acc * dv[i];
    }
  }
#pragma unroll
  for (int k = 0; k < GS_NB; ++k)
    if (k < nb) X[(size_t)(r0 + k) * n + j] = x[k];
}

// rows [r0, r1) of one sweep, T holding the contributions from outside
template <typename T>
void dense_gs_range(int32_t n, int32_t r0, int32_t r1, const T* Ad, const T* dinv, T* X, T* Tsum, bool forward,
                    hipStream_t s) {
  const int32_t len = r1 - r0;
  if (len <= GS_NB) {
    const unsigned cols = (unsigned)((n + 255) / 256);
    if (forward) blk_block_gs_kernel<T, true><<<cols, 256, 0, s>>>(n, r0, len, Ad, dinv, Tsum, X);
    else blk_block_gs_kernel<T, false><<<cols, 256, 0, s>>>(n, r0, len, Ad, dinv, Tsum, X);
    PCAMG_LAUNCHED();
    return;
  }
  const int32_t mid = r0 + ((len / 2 + GS_NB - 1) / GS_NB) * GS_NB;  // blocks stay GS_NB-aligned
  if (forward) {
    dense_gs_range<T>(n, r0, mid, Ad, dinv, X, Tsum, true, s);
    gemm_strided<T>(r1 - mid, mid - r0, n, (T)1, Ad + (size_t)mid * n + r0, n, X + (size_t)r0 * n, n, (T)1,
                    Tsum + (size_t)mid * n, n, s);
    dense_gs_range<T>(n, mid, r1, Ad, dinv, X, Tsum, true, s);
  } else {
    dense_gs_range<T>(n, mid, r1, Ad, dinv, X, Tsum, false, s);
    gemm_strided<T>(mid - r0, r1 - mid, n, (T)1, Ad + (size_t)r0 * n + mid, n, X + (size_t)mid * n, n, (T)1,
                    Tsum + (size_t)r0 * n, n, s);
    dense_gs_range<T>(n, r0, mid, Ad, dinv, X, Tsum, false, s);
  }
}

// One sweep on all n columns of X (forward: rows ascending).  old_side: the
// strictly upper (forward) or lower (backward) part of Ad, or null when X =
// 0 on entry.  Tsum: n x n scratch.
template <typename T>
void dense_gs_sweep(int32_t n, const T* Ad, const T* old_side, const T* dinv, T* X, T* Tsum, bool forward,
                    hipStream_t s) {
  if (old_side) gemm_rows<T>(n, n, n, (T)1, old_side, X, (T)0, Tsum, s);
  else PCAMG_HIP(hipMemsetAsync(Tsum, 0, (size_t)n * n * sizeof(T), s));  // all-zero bits: +0
  dense_gs_range<T>(n, 0, n, Ad, dinv, X, Tsum, forward, s);
}

// R[i, j] = delta_ij - (d_i X[i, j] + R[i, j]) with R = Ad X on entry: the
// residual of the identity right-hand side from the GEMM of the
// off-diagonal part.
template <typename T>
__global__ void __launch_bounds__(256)
    blk_resid_dense_kernel(int32_t n, const T* __restrict__ d, const T* __restrict__ X, T* __restrict__ R) {
  const int32_t i = (int32_t)blockIdx.y;
  const int32_t j = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (j >= n) return;
  const size_t o = (size_t)i * n + j;
  R[o] = (i == j ? (T)1 : (T)0) - fma(d[i], X[o], R[o]);
}

// Levels of at most DENSE_GS_MAX_N rows with more than one colour per
// DENSE_GS_ROWS_PER_COLOUR rows take dense_gs_sweep in the build.
constexpr int32_t DENSE_GS_MAX_N = 8192;
constexpr int32_t DENSE_GS_ROWS_PER_COLOUR = 16;

inline dim3 rows_grid(int32_t ncols, int32_t rows) { return dim3((unsigned)((ncols + 255) / 256), (unsigned)rows); }

template <typename T>
struct LevelOf;
template <>
struct LevelOf<double> {
  static const double* av(const LevelMatrix& A) { return A.av.p; }
  static const double* d(const LevelMatrix& A) { return A.d.p; }
  static const double* dinv(const LevelMatrix& A) { return A.dinv.p; }
  static const double* pval(const Transfer& T) { return T.pval.p; }
};
template <>
struct LevelOf<float> {
  static const float* av(const LevelMatrix& A) { return A.av32.p; }
  static const float* d(const LevelMatrix& A) { return A.d32.p; }
  static const float* dinv(const LevelMatrix& A) { return A.dinv32.p; }
  static const float* pval(const Transfer& T) { return T.pval32.p; }
};

// Operator of two consecutive calls of a level's cycle from x = 0, whose single
// call is W (m x m, row-major): x0 = W b, x1 = x0 + W (b - A x0), i.e.
// 2 W - W (A W).
template <typename T>
DVec<T> two_calls(const LevelMatrix& A, const DVec<T>& W, hipStream_t s) {
  const int32_t m = A.n;
  DVec<T> AW((size_t)m * m), Cop((size_t)m * m);
  blk_apply_kernel<T><<<rows_grid(m, m), 256, 0, s>>>(m, A.rp.p, A.ci.p, LevelOf<T>::av(A), LevelOf<T>::d(A), W.p,
                                                       AW.p, 0);
  PCAMG_LAUNCHED();
  copy_d2d(Cop.p, W.p, (size_t)m * m, s);
  gemm_rows<T>(m, m, m, (T)-1, W.p, AW.p, (T)2, Cop.p, s);
  return Cop;
}

}  // namespace

bool dense_bottom_up_fits(const Hierarchy& H, int start) {
  const int nl = (int)H.lv.size();
  if (start < 0) return false;
  for (int l = start; l < nl; ++l)
    if (H.lv[l].A->n > 65535) return false;  // rows of a pass are a grid dimension
  return H.cn <= 4096;
}

template <typename T>
void dense_bottom_up(Hierarchy& H, int d, int gamma, T* C, hipStream_t s, int calls) {
  const int nl = (int)H.lv.size();
  require(d >= 0 && nl - d >= 2 && dense_bottom_up_fits(H, d) && (gamma == 1 || gamma == 2) &&
              (calls == 1 || calls == gamma),
          PCAMG_EINVAL, "no dense region for the bottom-up build");
  // Z: the coarsest operator on the identity
  const int32_t cn = H.cn;
  DVec<T> W(std::max<size_t>((size_t)cn * cn, 1));
  coarsest_cols_kernel<T><<<cn, 256, (size_t)cn * sizeof(double), s>>>(cn, H.cm, H.grounded ? 1 : 0, H.cL.p,
                                                                          H.cD.p, W.p);
  PCAMG_LAUNCHED();
  for (int l = nl - 2; l >= d; --l) {
    const LevelMatrix& A = *H.lv[l].A;
    const Transfer& Tr = H.lv[l].T;
    const int32_t n = A.n, m = Tr.nc;
    require(m == H.lv[l + 1].A->n, PCAMG_EINVAL, "transfer size does not match the next level");
    // coarse operator: Z, one call W (V-cycle), or 2 W - W A W for the two
    // calls of a non-coarsest level (W-cycle)
    DVec<T> Cop;
    const T* Cl = W.p;
    if (gamma == 2 && l + 2 < nl) {
      Cop = two_calls<T>(*H.lv[l + 1].A, W, s);
      Cl = Cop.p;
    }
    // the cycle of level l on the identity
    DVec<T> X((size_t)n * n), R((size_t)n * n), Bc((size_t)m * n), Xc((size_t)m * n);
    PCAMG_HIP(hipMemsetAsync(X.p, 0, X.bytes(), s));  // all-zero bits: +0
    const T* av = LevelOf<T>::av(A);
    const T* dinv = LevelOf<T>::dinv(A);
    // near-dense levels: blocked dense sweeps instead of a launch per colour
    const bool dense_gs = n <= DENSE_GS_MAX_N && (int64_t)A.ncol * DENSE_GS_ROWS_PER_COLOUR > n;
    DVec<T> Ad, Lo, Ts;
    if (dense_gs) {
      Ad.resize((size_t)n * n);
      Lo.resize((size_t)n * n);
      Ts.resize((size_t)n * n);
      PCAMG_HIP(hipMemsetAsync(Ad.p, 0, Ad.bytes(), s));
      blk_densify_kernel<T><<<n, 256, 0, s>>>(n, A.rp.p, A.ci.p, av, Ad.p);
      PCAMG_LAUNCHED();
      blk_triangle_kernel<T, false><<<rows_grid(n, n), 256, 0, s>>>(n, Ad.p, Lo.p);
      PCAMG_LAUNCHED();
      dense_gs_sweep<T>(n, Ad.p, nullptr, dinv, X.p, Ts.p, true, s);  // from X = 0
    }
    for (int k = 0; k < (dense_gs ? 0 : A.ncol); ++k) {
      const int32_t r0 = A.coff[k], r1 = A.coff[k + 1];
      if (r1 <= r0) continue;
      blk_gs_kernel<T><<<dim3((unsigned)((n + 15) / 16), (unsigned)(r1 - r0)), 256, 0, s>>>(r0, n, A.rp.p, A.ci.p,
                                                                                           av, dinv, X.p);
      PCAMG_LAUNCHED();
    }
    if (dense_gs) {  // R = I - A X with the off-diagonal product on the matrix cores
      gemm_rows<T>(n, n, n, (T)1, Ad.p, X.p, (T)0, R.p, s);
      blk_resid_dense_kernel<T><<<rows_grid(n, n), 256, 0, s>>>(n, LevelOf<T>::d(A), X.p, R.p);
    } else {
      blk_apply_kernel<T><<<rows_grid(n, n), 256, 0, s>>>(n, A.rp.p, A.ci.p, av, LevelOf<T>::d(A), X.p, R.p, 1);
    }
    PCAMG_LAUNCHED();
    blk_restrict_kernel<T><<<rows_grid(n, m), 256, 0, s>>>(n, Tr.moff.p, Tr.mem.p, LevelOf<T>::pval(Tr), R.p, Bc.p);
    PCAMG_LAUNCHED();
    gemm_rows<T>(m, m, n, (T)1, Cl, Bc.p, (T)0, Xc.p, s);
    blk_prolong_kernel<T><<<rows_grid(n, n), 256, 0, s>>>(n, Tr.agg.p, LevelOf<T>::pval(Tr), Xc.p, X.p);
    PCAMG_LAUNCHED();
    if (dense_gs) dense_gs_sweep<T>(n, Ad.p, Lo.p, dinv, X.p, Ts.p, false, s);
    for (int k = dense_gs ? -1 : A.ncol - 1; k >= 0; --k) {
      const int32_t r0 = A.coff[k], r1 = A.coff[k + 1];
      if (r1 <= r0) continue;
      blk_gs_kernel<T><<<dim3((unsigned)((n + 15) / 16), (unsigned)(r1 - r0)), 256, 0, s>>>(r0, n, A.rp.p, A.ci.p,
                                                                                           av, dinv, X.p);
      PCAMG_LAUNCHED();
    }
    W = std::move(X);
  }
  // the level above applies `calls` calls of level d's cycle from x = 0
  const int32_t nd = H.lv[d].A->n;
  DVec<T> Cd;
  if (calls == 2) Cd = two_calls<T>(*H.lv[d].A, W, s);
  const T* src = calls == 2 ? Cd.p : W.p;
  blk_transpose_kernel<T><<<dim3((nd + 31) / 32, (nd + 31) / 32), 256, 0, s>>>(nd, src, C);
  PCAMG_LAUNCHED();
  PCAMG_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

template void dense_bottom_up<double>(Hierarchy&, int, int, double*, hipStream_t, int);
template void dense_bottom_up<float>(Hierarchy&, int, int, float*, hipStream_t, int);

namespace {
// deterministic operand values in [-1, 1)
template <typename T>
__global__ void gemm_fill_kernel(size_t n, uint32_t salt, T* __restrict__ a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t h = (uint32_t)i * 2654435761u ^ salt;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  a[i] = (T)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
}

template <typename T>
double bench_gemm_t(int32_t p, int32_t q, int32_t r, int reps, hipStream_t s) {
  DVec<T> Q((size_t)p * q), R((size_t)q * r), P((size_t)p * r);
  gemm_fill_kernel<T><<<(unsigned)(((size_t)p * q + 255) / 256), 256, 0, s>>>((size_t)p * q, 1u, Q.p);
  PCAMG_LAUNCHED();
  gemm_fill_kernel<T><<<(unsigned)(((size_t)q * r + 255) / 256), 256, 0, s>>>((size_t)q * r, 2u, R.p);
  PCAMG_LAUNCHED();
  gemm_rows<T>(p, q, r, (T)1, Q.p, R.p, (T)0, P.p, s);  // warm-up
  hipEvent_t e0, e1;
  PCAMG_HIP(hipEventCreate(&e0));
  PCAMG_HIP(hipEventCreate(&e1));
  float t = 0.0f;
  hipError_t err = hipEventRecord(e0, s);
  for (int k = 0; k < reps && err == hipSuccess; ++k) gemm_rows<T>(p, q, r, (T)1, Q.p, R.p, (T)0, P.p, s);
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  PCAMG_HIP(err);
  return t;
}
}  // namespace

double bench_gemm(int32_t p, int32_t q, int32_t r, int prec, int reps, hipStream_t s) {
  return prec == PCAMG_PREC_F32 ? bench_gemm_t<float>(p, q, r, reps, s) : bench_gemm_t<double>(p, q, r, reps, s);
}

}  // namespace pcamg
