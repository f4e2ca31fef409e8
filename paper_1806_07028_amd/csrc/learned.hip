// Learned smooth-error proposals: a three-layer message-passing network
// (hidden 64) maps a briefly relaxed vector e2 to a smoother vector whose
// level sets give the path-cover keys (Alg. 4, Step 2, Sec. 3.2), replacing
// most of the relaxation sweeps of the first build.
//
//   u = normalise(e2), l = log d - mean(log d), F = [u, Ahat u, l, Ahat l]
//   h0 = relu(F W0 + b0)
//   h_k = relu(bf16([h_{k-1} | Ahat h_{k-1}]) bf16(W_k) + b_k), k = 1..3
//   y = h3 wo + bo + u,    loss = 0.5 mean((y - normalise(t))^2)
// with Ahat = D^{-1} W.  The hidden-layer products and their backward
// products run on MFMA (v_mfma_f32_16x16x16_bf16, float32 accumulation);
// everything else in float32, the normalisations in float64.  Sums over
// nodes (weight and bias gradients, the loss) are partial sums per block
// added in block order, so results are reproducible.
#include <cmath>

#include "solver.hpp"

namespace pcamg {

namespace {

constexpr int HID = 64;
constexpr int NF = 4;
constexpr int NL = 3;
constexpr int ZD = 2 * HID;
// parameter layout: W0 (4x64), b0, (W_k (128x64), b_k) x 3, wo (64), bo (1)
constexpr int OFF_W0 = 0;
constexpr int OFF_B0 = OFF_W0 + NF * HID;
constexpr int OFF_L1 = OFF_B0 + HID;
constexpr int LAYER_SZ = ZD * HID + HID;
constexpr int OFF_WO = OFF_L1 + NL * LAYER_SZ;
constexpr int OFF_BO = OFF_WO + HID;
constexpr int NPAR = OFF_BO + 1;
constexpr int ROWS_PER_CHUNK = 256;  // node chunk of the split-K weight gradients

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// Graph-side kernels
// ---------------------------------------------------------------------------
__global__ void degree_kernel(int32_t n, const int32_t* __restrict__ rp, const double* __restrict__ w,
                              double* __restrict__ d, double* __restrict__ logd) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += w[k];
  d[i] = s;
  logd[i] = log(s);
}

// out_i = sum_j (w_ij / d_i) v_j  (float64)
__global__ void ahat_f64_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ w, const double* __restrict__ d,
                                const double* __restrict__ v, double* __restrict__ out) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += (w[k] / d[i]) * v[ci[k]];
  out[i] = s;
}

// y = (x - sum/n) * scale  with scale = 1 / rms
__global__ void centre_scale_kernel(int32_t n, const double* __restrict__ x, const double* __restrict__ sums,
                                    double* __restrict__ y) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mu = sums[0] / n;
  const double r = sqrt(fmax(sums[1] / n - 0.0, 0.0));
  y[i] = r > 0.0 ? (x[i] - mu) / r : x[i] - mu;
}

__global__ void sub_scalar_kernel(int32_t n, const double* __restrict__ x, const double* __restrict__ sum,
                                  double* __restrict__ y) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] - sum[0] / n;
}

__global__ void features_kernel(int32_t n, const double* __restrict__ u, const double* __restrict__ au,
                                const double* __restrict__ l, const double* __restrict__ al, float* __restrict__ F) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  F[4 * i + 0] = (float)u[i];
  F[4 * i + 1] = (float)au[i];
  F[4 * i + 2] = (float)l[i];
  F[4 * i + 3] = (float)al[i];
}

// Ahat as float32 values in CSR order: a_ij = (float)(w_ij / d_i); and the
// transpose weights (Ahat^T)_ji = a_ij seen from row j: w_ji / d_i.
__global__ void ahat_vals_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ w, const double* __restrict__ d,
                                 float* __restrict__ a, float* __restrict__ at) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    a[k] = (float)(w[k] / d[i]);
    at[k] = (float)(w[k] / d[ci[k]]);
  }
}

// ---------------------------------------------------------------------------
// Network kernels (n rows padded to a multiple of ROWS_PER_CHUNK, pad rows 0)
// ---------------------------------------------------------------------------
// h0 = relu(F W0 + b0), and the bf16 copy of h0 into z's first half
__global__ void layer0_kernel(int32_t n, const float* __restrict__ F, const float* __restrict__ th,
                              float* __restrict__ h) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = t / HID, f = t % HID;
  if (i >= n) return;
  float s = th[OFF_B0 + f];
  for (int c = 0; c < NF; ++c) s = fmaf(F[4 * i + c], th[OFF_W0 + c * HID + f], s);
  h[(size_t)i * HID + f] = fmaxf(s, 0.0f);
}

// z = [h | Ahat h] as bf16 (one wavefront per row, lane = feature)
__global__ void __launch_bounds__(256)
    message_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                   const float* __restrict__ a, const float* __restrict__ h, uint16_t* __restrict__ z) {
  const int32_t i = blockIdx.x * 4 + threadIdx.x / 64;
  const int f = threadIdx.x % 64;
  if (i >= n) return;
  float s = 0.0f;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s = fmaf(a[k], h[(size_t)ci[k] * HID + f], s);
  z[(size_t)i * ZD + f] = to_bf16(h[(size_t)i * HID + f]);
  z[(size_t)i * ZD + HID + f] = to_bf16(s);
}

// weights of layer k as bf16: wt[c][r] = W[r][c] (64 x 128, forward B
// operand) and wn[r][c] = W[r][c] (128 x 64, backward B operand)
__global__ void weights_bf16_kernel(const float* __restrict__ W, uint16_t* __restrict__ wt,
                                    uint16_t* __restrict__ wn) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ZD * HID) return;
  const int r = t / HID, c = t % HID;
  const uint16_t b = to_bf16(W[t]);
  wn[t] = b;
  wt[c * ZD + r] = b;
}

__device__ __forceinline__ bf16x4 load4(const uint16_t* p) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4 r;
  r[0] = (short)(v.x & 0xFFFF);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFF);
  r[3] = (short)(v.y >> 16);
  return r;
}

// Y (rows x NOUT) = A (rows x K, bf16 row-major) * B, with B given as
// Bt (NOUT x K, bf16 row-major: Bt[j][k] = B[k][j]).  One wavefront per 16
// rows; MFMA 16x16x16: lane l holds A[l%16][4(l/16)..+3], B[4(l/16)..+3][l%16],
// and D[4(l/16)..+3][l%16].  mode 0: Y = relu(D + bias) (float32);
// mode 1: Y = D (float32).
// rows: valid rows (written); A is allocated to a multiple of 16 rows beyond.
template <int K, int NOUT>
__global__ void __launch_bounds__(256)
    mfma_rows_kernel(int32_t rows, const uint16_t* __restrict__ A, const uint16_t* __restrict__ Bt,
                     const float* __restrict__ bias, float* __restrict__ Y, int mode) {
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  const int l = threadIdx.x % 64;
  const int32_t r0 = wave * 16;
  if (r0 >= rows) return;  // whole wavefront
  const int rr = l % 16, kq = 4 * (l / 16);
  f32x4 acc[NOUT / 16];
#pragma unroll
  for (int t = 0; t < NOUT / 16; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kk = 0; kk < K; kk += 16) {
    const bf16x4 a = load4(A + (size_t)(r0 + rr) * K + kk + kq);
#pragma unroll
    for (int t = 0; t < NOUT / 16; ++t) {
      const bf16x4 b = load4(Bt + (size_t)(t * 16 + rr) * K + kk + kq);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NOUT / 16; ++t) {
    const int col = t * 16 + rr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t row = r0 + kq + q;
      float v = acc[t][q];
      if (mode == 0) v = fmaxf(v + bias[col], 0.0f);
      if (row < rows) Y[(size_t)row * NOUT + col] = v;
    }
  }
}

// Partial weight gradient of one node chunk: G (ZD x HID) += Z^T dP over the
// chunk's rows, Z (rows x ZD) and dP (rows x HID) bf16.  Four wavefronts, each
// eight 16x16 output tiles; K = the chunk's nodes.
__global__ void __launch_bounds__(256)
    mfma_wgrad_kernel(const uint16_t* __restrict__ Z, const uint16_t* __restrict__ dP, float* __restrict__ part) {
  const int wave = threadIdx.x / 64;
  const int l = threadIdx.x % 64;
  const int rr = l % 16, kq = 4 * (l / 16);
  const size_t node0 = (size_t)blockIdx.x * ROWS_PER_CHUNK;
  f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int kk = 0; kk < ROWS_PER_CHUNK; kk += 16) {
    const size_t nk = node0 + kk + kq;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int tile = wave * 8 + t;          // 32 tiles: 8 along ZD x 4 along HID
      const int tm = tile / 4, tn = tile % 4;
      bf16x4 a, b;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = (short)Z[(nk + q) * ZD + tm * 16 + rr];
        b[q] = (short)dP[(nk + q) * HID + tn * 16 + rr];
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  float* out = part + (size_t)blockIdx.x * ZD * HID;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tile = wave * 8 + t;
    const int tm = tile / 4, tn = tile % 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(size_t)(tm * 16 + kq + q) * HID + tn * 16 + rr] = acc[t][q];
  }
}

// out[c] = sum over blocks b in order of part[b][c]
__global__ void sum_parts_kernel(int32_t nparts, int32_t width, const float* __restrict__ part,
                                 float* __restrict__ out) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= width) return;
  float s = 0.0f;
  for (int32_t b = 0; b < nparts; ++b) s += part[(size_t)b * width + c];
  out[c] = s;
}

// Per-chunk column sums of X (rows x 64) [times v (rows) when given]:
// part[chunk][f] = sum_{i in chunk} X[i][f] (* v[i])
__global__ void colsum_kernel(int32_t rows, const float* __restrict__ X, const float* __restrict__ v,
                              float* __restrict__ part) {
  const int f = threadIdx.x;  // 64 threads
  const int32_t i0 = blockIdx.x * ROWS_PER_CHUNK;
  float s = 0.0f;
  for (int32_t i = i0; i < min(rows, i0 + ROWS_PER_CHUNK); ++i) {
    const float x = X[(size_t)i * HID + f];
    s = v ? fmaf(x, v[i], s) : s + x;
  }
  part[(size_t)blockIdx.x * HID + f] = s;
}

// part[chunk] = sum_{i in chunk} v[i]
__global__ void vsum_kernel(int32_t rows, int32_t chunks, const float* __restrict__ v, float* __restrict__ part) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chunks) return;
  float s = 0.0f;
  for (int32_t i = c * ROWS_PER_CHUNK; i < min(rows, (c + 1) * ROWS_PER_CHUNK); ++i) s += v[i];
  part[c] = s;
}

// Per-chunk W0 gradient: part[chunk][c*64+f] = sum_i F[i][c] dP0[i][f]
__global__ void w0grad_kernel(int32_t rows, const float* __restrict__ F, const float* __restrict__ dP,
                              float* __restrict__ part) {
  const int t = threadIdx.x;  // 256 = 4 x 64
  const int c = t / HID, f = t % HID;
  const int32_t i0 = blockIdx.x * ROWS_PER_CHUNK;
  float s = 0.0f;
  for (int32_t i = i0; i < min(rows, i0 + ROWS_PER_CHUNK); ++i) s = fmaf(F[4 * i + c], dP[(size_t)i * HID + f], s);
  part[(size_t)blockIdx.x * (NF * HID) + t] = s;
}

// y = h3 wo + bo + u
__global__ void output_kernel(int32_t n, const float* __restrict__ h, const float* __restrict__ th,
                              const float* __restrict__ F, float* __restrict__ y) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = th[OFF_BO];
  for (int f = 0; f < HID; ++f) s = fmaf(h[(size_t)i * HID + f], th[OFF_WO + f], s);
  y[i] = s + F[4 * i];
}

// r = y - t (float64 residual for the loss), dy = r / n (float32)
__global__ void loss_grad_kernel(int32_t n, const float* __restrict__ y, const double* __restrict__ t,
                                 double* __restrict__ r, float* __restrict__ dy) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ri = (double)y[i] - t[i];
  r[i] = ri;
  dy[i] = (float)(ri / n);
}

// dh = dy wo^T, then the ReLU mask of h3: dP = dh * (h > 0), bf16 copy
__global__ void out_back_kernel(int32_t n, const float* __restrict__ dy, const float* __restrict__ th,
                                const float* __restrict__ h, float* __restrict__ dP, uint16_t* __restrict__ dPb) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t i = t / HID, f = t % HID;
  if (i >= n) return;
  const float g = dy[i] * th[OFF_WO + f];
  const float v = h[(size_t)i * HID + f] > 0.0f ? g : 0.0f;
  dP[t] = v;
  dPb[t] = to_bf16(v);
}

// dh_{k-1} = dz[:, :64] + Ahat^T dz[:, 64:], masked by h_{k-1} > 0 (the next
// layer's dP); bf16 copy.  One wavefront per row.
__global__ void __launch_bounds__(256)
    msg_back_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                    const float* __restrict__ at, const float* __restrict__ dz, const float* __restrict__ h,
                    float* __restrict__ dP, uint16_t* __restrict__ dPb) {
  const int32_t j = blockIdx.x * 4 + threadIdx.x / 64;
  const int f = threadIdx.x % 64;
  if (j >= n) return;
  float s = dz[(size_t)j * ZD + f];
  for (int32_t k = rp[j]; k < rp[j + 1]; ++k) s = fmaf(at[k], dz[(size_t)ci[k] * ZD + HID + f], s);
  const float v = h[(size_t)j * HID + f] > 0.0f ? s : 0.0f;
  dP[(size_t)j * HID + f] = v;
  dPb[(size_t)j * HID + f] = to_bf16(v);
}

__global__ void adam_kernel(int32_t m, float* __restrict__ th, float* __restrict__ mm, float* __restrict__ vv,
                            const float* __restrict__ g, float lr, float c1, float c2) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float gi = g[i];
  const float mi = 0.9f * mm[i] + 0.1f * gi;
  const float vi = 0.999f * vv[i] + 0.001f * gi * gi;
  mm[i] = mi;
  vv[i] = vi;
  th[i] = th[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Seeded initial parameters: entry k of the flat parameter vector draws word
// k + 1 of the SplitMix64 stream `seed`, u = (word >> 11) 2^-53 in [0, 1), and
// takes (2u - 1) lim rounded to float32, where lim is the Glorot-uniform bound
// sqrt(6 / (fan_in + fan_out)) of its weight matrix (lim0: W0, limh: W1..W3),
// 0.1 for the output weights and 0 for every bias.
__global__ void init_params_kernel(uint64_t seed, double lim0, double limh, float* __restrict__ th) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NPAR) return;
  double lim = 0.0;
  if (k < OFF_B0) {
    lim = lim0;
  } else if (k >= OFF_L1 && k < OFF_WO) {
    lim = (k - OFF_L1) % LAYER_SZ < ZD * HID ? limh : 0.0;
  } else if (k >= OFF_WO && k < OFF_BO) {
    lim = 0.1;
  }
  uint64_t z = seed + (uint64_t)(k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * 0x1.0p-53;
  th[k] = (float)((2.0 * u - 1.0) * lim);
}

__global__ void widen_kernel(int32_t n, const float* __restrict__ y, double* __restrict__ e) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) e[i] = (double)y[i];
}

size_t pad_rows(int32_t n) { return ((size_t)n + ROWS_PER_CHUNK - 1) / ROWS_PER_CHUNK * ROWS_PER_CHUNK; }

}  // namespace

// Per-graph state of one forward (and backward) pass.
struct NetPass {
  int32_t n = 0;
  size_t rows = 0;
  DVec<float> F, a, at, y, dy;
  DVec<float> h[NL + 1];
  DVec<uint16_t> z[NL];
};

// normalise(v): mean removed, unit RMS (float64)
static void normalise_f64(int32_t n, const double* v, double* out, hipStream_t s) {
  DVec<double> sums(2), c(n);
  sum_f64(v, n, sums.p, s);
  sub_scalar_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, v, sums.p, c.p);
  PCAMG_LAUNCHED();
  dot_f64(c.p, c.p, n, sums.p + 1, s);
  fill_f64(sums.p, 0.0, 1, s);
  centre_scale_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, c.p, sums.p, out);
  PCAMG_LAUNCHED();
}

static void net_forward(const float* th, const pcamg_graph* g, const double* e2, NetPass& P, uint16_t* wt[NL],
                        uint16_t* wn[NL], hipStream_t s) {
  const int32_t n = g->n;
  P.n = n;
  P.rows = pad_rows(n);
  DVec<double> d(n), logd(n), u(n), au(n), l(n), al(n), sums(1);
  degree_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->weight, d.p, logd.p);
  PCAMG_LAUNCHED();
  normalise_f64(n, e2, u.p, s);
  sum_f64(logd.p, n, sums.p, s);
  sub_scalar_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, logd.p, sums.p, l.p);
  PCAMG_LAUNCHED();
  ahat_f64_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, g->weight, d.p, u.p, au.p);
  PCAMG_LAUNCHED();
  ahat_f64_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, g->weight, d.p, l.p, al.p);
  PCAMG_LAUNCHED();
  P.F.resize(4 * (size_t)n);
  features_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, u.p, au.p, l.p, al.p, P.F.p);
  PCAMG_LAUNCHED();
  P.a.resize(std::max<int32_t>(g->nnz, 1));
  P.at.resize(std::max<int32_t>(g->nnz, 1));
  ahat_vals_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, g->weight, d.p, P.a.p, P.at.p);
  PCAMG_LAUNCHED();
  for (int k = 0; k <= NL; ++k) {
    P.h[k].resize(P.rows * HID);
    fill_f32(P.h[k].p, 0.0f, P.rows * HID, s);
  }
  layer0_kernel<<<grid_for((size_t)n * HID, 256), 256, 0, s>>>(n, P.F.p, th, P.h[0].p);
  PCAMG_LAUNCHED();
  for (int k = 0; k < NL; ++k) {
    P.z[k].resize(P.rows * ZD);
    fill_u32(reinterpret_cast<uint32_t*>(P.z[k].p), 0u, P.rows * ZD / 2, s);
    message_kernel<<<grid_for(n, 4), 256, 0, s>>>(n, g->row_ptr, g->col_idx, P.a.p, P.h[k].p, P.z[k].p);
    PCAMG_LAUNCHED();
    const float* bias = th + OFF_L1 + k * LAYER_SZ + ZD * HID;
    mfma_rows_kernel<ZD, HID><<<grid_for(P.rows / 16, 4), 256, 0, s>>>(n, P.z[k].p, wt[k], bias, P.h[k + 1].p, 0);
    PCAMG_LAUNCHED();
  }
  P.y.resize(n);
  output_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, P.h[NL].p, th, P.F.p, P.y.p);
  PCAMG_LAUNCHED();
}

}  // namespace pcamg

using namespace pcamg;

struct pcamg_net {
  DVec<float> th, m, v, grad;
  DVec<uint16_t> wt[NL], wn[NL];
  int64_t step = 0;
  bool bf_ready = false;
};

namespace pcamg {

static void refresh_bf16(pcamg_net* net, hipStream_t s) {
  for (int k = 0; k < NL; ++k) {
    weights_bf16_kernel<<<grid_for(ZD * HID, 256), 256, 0, s>>>(net->th.p + OFF_L1 + k * LAYER_SZ, net->wt[k].p,
                                                                 net->wn[k].p);
    PCAMG_LAUNCHED();
  }
  net->bf_ready = true;
}

int32_t net_num_params() { return NPAR; }

// Parameters, Adam moments and gradient start at zero; the network refuses
// forward, backward and optimiser calls until net_set_params or net_init has
// given it parameters.
void net_create(pcamg_net** out) {
  auto net = std::make_unique<pcamg_net>();
  net->th.resize(NPAR);
  net->m.resize(NPAR);
  net->v.resize(NPAR);
  net->grad.resize(NPAR);
  for (int k = 0; k < NL; ++k) {
    net->wt[k].resize(ZD * HID);
    net->wn[k].resize(ZD * HID);
  }
  for (DVec<float>* a : {&net->th, &net->m, &net->v, &net->grad}) PCAMG_HIP(hipMemset(a->p, 0, a->bytes()));
  PCAMG_HIP(hipDeviceSynchronize());
  *out = net.release();
}

void net_init(pcamg_net* net, uint64_t seed, hipStream_t s) {
  const double lim0 = std::sqrt(6.0 / (NF + HID)), limh = std::sqrt(6.0 / (ZD + HID));
  init_params_kernel<<<grid_for(NPAR, 256), 256, 0, s>>>(seed, lim0, limh, net->th.p);
  PCAMG_LAUNCHED();
  fill_f32(net->m.p, 0.0f, NPAR, s);
  fill_f32(net->v.p, 0.0f, NPAR, s);
  fill_f32(net->grad.p, 0.0f, NPAR, s);
  net->step = 0;
  refresh_bf16(net, s);
  PCAMG_HIP(hipStreamSynchronize(s));
}

void net_destroy(pcamg_net* net) { delete net; }

void net_set_params(pcamg_net* net, const float* host, hipStream_t s) {
  copy_h2d(net->th.p, host, NPAR, s);
  fill_f32(net->m.p, 0.0f, NPAR, s);
  fill_f32(net->v.p, 0.0f, NPAR, s);
  fill_f32(net->grad.p, 0.0f, NPAR, s);
  net->step = 0;
  refresh_bf16(net, s);
  PCAMG_HIP(hipStreamSynchronize(s));
}

void net_get_params(pcamg_net* net, float* host, hipStream_t s) {
  PCAMG_HIP(hipMemcpyAsync(host, net->th.p, NPAR * sizeof(float), hipMemcpyDeviceToHost, s));
  PCAMG_HIP(hipStreamSynchronize(s));
}

void net_forward_f32(pcamg_net* net, const pcamg_graph* g, const double* e2, float* y, hipStream_t s) {
  require(net->bf_ready, PCAMG_EINVAL, "network parameters not set");
  NetPass P;
  uint16_t* wt[NL];
  uint16_t* wn[NL];
  for (int k = 0; k < NL; ++k) wt[k] = net->wt[k].p, wn[k] = net->wn[k].p;
  net_forward(net->th.p, g, e2, P, wt, wn, s);
  copy_d2d(y, P.y.p, g->n, s);
  PCAMG_HIP(hipStreamSynchronize(s));
}

void net_forward_f64(pcamg_net* net, const pcamg_graph* g, const double* e2, double* e, hipStream_t s) {
  DVec<float> y(g->n);
  net_forward_f32(net, g, e2, y.p, s);
  widen_kernel<<<grid_for(g->n, 256), 256, 0, s>>>(g->n, y.p, e);
  PCAMG_LAUNCHED();
}

double net_loss_grad(pcamg_net* net, const pcamg_graph* g, const double* e2, const double* target, float* grad_host,
                     hipStream_t s) {
  require(net->bf_ready, PCAMG_EINVAL, "network parameters not set");
  const int32_t n = g->n;
  NetPass P;
  uint16_t* wt[NL];
  uint16_t* wn[NL];
  for (int k = 0; k < NL; ++k) wt[k] = net->wt[k].p, wn[k] = net->wn[k].p;
  const float* th = net->th.p;
  float* G = net->grad.p;
  net_forward(th, g, e2, P, wt, wn, s);
  const size_t rows = P.rows;
  const int32_t chunks = (int32_t)(rows / ROWS_PER_CHUNK);
  // loss and dy
  DVec<double> t(n), r(n), lsum(1);
  normalise_f64(n, target, t.p, s);
  DVec<float> dy(rows);
  fill_f32(dy.p, 0.0f, rows, s);
  loss_grad_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, P.y.p, t.p, r.p, dy.p);
  PCAMG_LAUNCHED();
  dot_f64(r.p, r.p, n, lsum.p, s);
  // output layer: g_wo = h3^T dy, g_bo = sum dy
  DVec<float> part((size_t)chunks * std::max(ZD * HID, NF * HID));
  colsum_kernel<<<chunks, HID, 0, s>>>(n, P.h[NL].p, dy.p, part.p);
  PCAMG_LAUNCHED();
  sum_parts_kernel<<<1, HID, 0, s>>>(chunks, HID, part.p, G + OFF_WO);
  PCAMG_LAUNCHED();
  vsum_kernel<<<grid_for(chunks, 64), 64, 0, s>>>(n, chunks, dy.p, part.p);
  PCAMG_LAUNCHED();
  sum_parts_kernel<<<1, 1, 0, s>>>(chunks, 1, part.p, G + OFF_BO);
  PCAMG_LAUNCHED();
  DVec<float> dP(rows * HID), dz(rows * ZD);
  DVec<uint16_t> dPb(rows * HID);
  fill_f32(dP.p, 0.0f, rows * HID, s);
  fill_u32(reinterpret_cast<uint32_t*>(dPb.p), 0u, rows * HID / 2, s);
  out_back_kernel<<<grid_for((size_t)n * HID, 256), 256, 0, s>>>(n, dy.p, th, P.h[NL].p, dP.p, dPb.p);
  PCAMG_LAUNCHED();
  for (int k = NL - 1; k >= 0; --k) {
    float* gW = G + OFF_L1 + k * LAYER_SZ;
    // weight gradient: Z_k^T dP (split over node chunks)
    mfma_wgrad_kernel<<<chunks, 256, 0, s>>>(P.z[k].p, dPb.p, part.p);
    PCAMG_LAUNCHED();
    sum_parts_kernel<<<grid_for(ZD * HID, 256), 256, 0, s>>>(chunks, ZD * HID, part.p, gW);
    PCAMG_LAUNCHED();
    // bias gradient: column sums of dP
    colsum_kernel<<<chunks, HID, 0, s>>>(n, dP.p, nullptr, part.p);
    PCAMG_LAUNCHED();
    sum_parts_kernel<<<1, HID, 0, s>>>(chunks, HID, part.p, gW + ZD * HID);
    PCAMG_LAUNCHED();
    // dz = dP W_k^T, then dh_{k} -> dP of the layer below
    mfma_rows_kernel<HID, ZD><<<grid_for(rows / 16, 4), 256, 0, s>>>(n, dPb.p, wn[k], nullptr, dz.p, 1);
    PCAMG_LAUNCHED();
    msg_back_kernel<<<grid_for(n, 4), 256, 0, s>>>(n, g->row_ptr, g->col_idx, P.at.p, dz.p,
                                                    P.h[k].p, dP.p, dPb.p);
    PCAMG_LAUNCHED();
  }
  // first layer
  w0grad_kernel<<<chunks, 256, 0, s>>>(n, P.F.p, dP.p, part.p);
  PCAMG_LAUNCHED();
  sum_parts_kernel<<<1, 256, 0, s>>>(chunks, NF * HID, part.p, G + OFF_W0);
  PCAMG_LAUNCHED();
  colsum_kernel<<<chunks, HID, 0, s>>>(n, dP.p, nullptr, part.p);
  PCAMG_LAUNCHED();
  sum_parts_kernel<<<1, HID, 0, s>>>(chunks, HID, part.p, G + OFF_B0);
  PCAMG_LAUNCHED();
  if (grad_host) {
    PCAMG_HIP(hipMemcpyAsync(grad_host, G, NPAR * sizeof(float), hipMemcpyDeviceToHost, s));
  }
  const double L = 0.5 * read_scalar(lsum.p, s) / n;
  return L;
}

void net_adam(pcamg_net* net, float lr, hipStream_t s) {
  require(net->bf_ready, PCAMG_EINVAL, "network parameters not set");
  net->step += 1;
  const float c1 = 1.0f - powf(0.9f, (float)net->step);
  const float c2 = 1.0f - powf(0.999f, (float)net->step);
  adam_kernel<<<grid_for(NPAR, 256), 256, 0, s>>>(NPAR, net->th.p, net->m.p, net->v.p, net->grad.p, lr, c1, c2);
  PCAMG_LAUNCHED();
  refresh_bf16(net, s);
}

}  // namespace pcamg
