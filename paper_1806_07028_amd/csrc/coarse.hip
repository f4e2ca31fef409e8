// Coarsest level: dense LDL^T (no square roots) in one workgroup, FP64.
// Column j: v_k = L_jk D_k (k < j); D_j = A_jj - sum_k L_jk v_k;
// L_ij = (A_ij - sum_k L_ik v_k) / D_j, every sum an fma chain with k
// ascending.  Solves run column by column so each unknown accumulates its
// terms in the same order as a row-by-row substitution (forward: k ascending,
// backward: k descending).
#include "internal.hpp"

namespace pcamg {

constexpr int LDLT_THREADS = 256;
constexpr int LDLT_LDS_MAX = 4096;  // equals LDLT_MAX of the tail kernel

__global__ void dense_zero_kernel(double* A, size_t nn) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) A[i] = 0.0;
}

__global__ void dense_fill_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const double* __restrict__ av, const double* __restrict__ d, double* __restrict__ A) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  A[(size_t)i * n + i] = d[i];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) A[(size_t)i * n + ci[k]] = av[k];
}

void dense_from_csr(int32_t n, const int32_t* rp, const int32_t* ci, const double* av, const double* d, double* A,
                    hipStream_t s) {
  size_t nn = (size_t)n * n;
  dense_zero_kernel<<<grid_for(nn, 256), 256, 0, s>>>(A, nn);
  PCAMG_LAUNCHED();
  dense_fill_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, ci, av, d, A);
  PCAMG_LAUNCHED();
}

__global__ void __launch_bounds__(LDLT_THREADS)
    ldlt_factor_kernel(int32_t n, int32_t m, const double* __restrict__ A, double* __restrict__ L,
                       double* __restrict__ D, int32_t* __restrict__ fail) {
  __shared__ double v[LDLT_LDS_MAX];
  __shared__ double dj;
  for (int32_t j = 0; j < m; ++j) {
    for (int32_t k = threadIdx.x; k < j; k += blockDim.x) v[k] = L[(size_t)j * m + k] * D[k];
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = A[(size_t)j * n + j];
      for (int32_t k = 0; k < j; ++k) s = fma(-L[(size_t)j * m + k], v[k], s);
      dj = s;
      D[j] = s;
      L[(size_t)j * m + j] = 1.0;
      for (int32_t k = j + 1; k < m; ++k) L[(size_t)j * m + k] = 0.0;
      if (!(s > 0.0)) *fail = 1;
    }
    __syncthreads();
    if (!(dj > 0.0)) return;
    for (int32_t i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
      double t = A[(size_t)i * n + j];
      for (int32_t k = 0; k < j; ++k) t = fma(-L[(size_t)i * m + k], v[k], t);
      L[(size_t)i * m + j] = t / dj;
    }
    __syncthreads();
  }
}

bool ldlt_factor(int32_t n, int32_t m, const double* A, double* L, double* D, hipStream_t s) {
  require(m <= LDLT_LDS_MAX, PCAMG_EUNSUPPORTED, "coarsest level larger than 4096");
  if (m <= 0) return true;
  DVec<int32_t> fail(1);
  fill_i32(fail.p, 0, 1, s);
  ldlt_factor_kernel<<<1, LDLT_THREADS, 0, s>>>(n, m, A, L, D, fail.p);
  PCAMG_LAUNCHED();
  return read_scalar(fail.p, s) == 0;
}

template <typename TB>
__global__ void __launch_bounds__(LDLT_THREADS)
    ldlt_solve_kernel(int32_t n, int32_t m, bool grounded, const double* __restrict__ L, const double* __restrict__ D,
                      const TB* __restrict__ b, TB* __restrict__ x) {
  __shared__ double acc[LDLT_LDS_MAX];
  __shared__ double mu;
  for (int32_t i = threadIdx.x; i < m; i += blockDim.x) acc[i] = (double)b[i];
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
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = (TB)(acc[i] - mu);
  } else {
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) x[i] = (TB)acc[i];
  }
}

void ldlt_solve(int32_t n, int32_t m, bool grounded, const double* L, const double* D, const double* b, double* x,
                hipStream_t s) {
  ldlt_solve_kernel<double><<<1, LDLT_THREADS, 0, s>>>(n, m, grounded, L, D, b, x);
  PCAMG_LAUNCHED();
}

void ldlt_solve32(int32_t n, int32_t m, bool grounded, const double* L, const double* D, const float* b, float* x,
                  hipStream_t s) {
  ldlt_solve_kernel<float><<<1, LDLT_THREADS, 0, s>>>(n, m, grounded, L, D, b, x);
  PCAMG_LAUNCHED();
}

}  // namespace pcamg
