// Row sums of a CSR matrix against a vector, s = fma(a_k, x[c_k], s) over the
// row's entries in stored order.  This order is fixed because smoothed and
// restricted values must match the FP64 reference bit for bit; what these
// routines change is only how the operands reach the chain:
//
//  * row_chain1: one thread per row.  Entries are taken in batches of eight
//    whose column indices and values are loaded independently, then the
//    eight gathered x values, then eight chained fmas -- two memory round
//    trips per batch instead of two per entry.  The last, partial batch
//    loads unconditionally too (past the end: the row's last entry again,
//    never added): loads under a condition would each wait for their value
//    before the next one issues.
//  * row_chain_g<G>: G adjacent lanes of a wavefront per row (G divides 64).
//    Lane q loads entries q, q+G, ... of the row (coalesced), U chunks at a
//    time; every lane of the group then runs the same chain with the operands
//    broadcast lane by lane (DPP quad moves for G = 4, shuffles otherwise), so
//    the group holds the row sum in all its lanes.  Every lane of the
//    wavefront must call it with uniform control flow, rows beyond the range
//    with len = 0.  Loads past a row's end re-read its last entry (or, for an
//    empty row, entry k0): they are unconditional, so a chunk's loads issue
//    together instead of one masked load at a time, and never enter the
//    chain.  The arrays need one readable slot at index nnz (a zero pad).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcamg {

// pointer into global memory, for pointers the compiler cannot trace to a
// kernel argument (loads become global_load instead of flat_load)
#define PCAMG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const PCAMG_GLOBAL T* gptr(const T* p) {
  return (const PCAMG_GLOBAL T*)p;
}

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each
// with its own L2.  This maps the launch's workgroups to tiles so that each XCD
// takes a contiguous range of tiles (XCD x: tiles x*q + min(x, r) + [0, q + (x < r)),
// q = nb / 8, r = nb % 8), which keeps the vector gathers of neighbouring rows
// in one L2.  A bijection on [0, nb) for every nb.
__device__ __forceinline__ uint32_t xcd_block() {
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// The index, value and vector pointers are template parameters so callers can
// pass pointers qualified with an address space (global or LDS) and get the
// matching load instructions.
template <typename T, typename PI, typename PA, typename PX>
__device__ __forceinline__ T row_chain1(int32_t k0, int32_t k1, PI ci, PA av, PX x, T s) {
  constexpr int U = 8;
  int32_t k = k0;
  for (; k + U <= k1; k += U) {
    int32_t c[U];
    T a[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = ci[k + u];
      a[u] = av[k + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(a[u], v[u], s);
  }
  const int32_t rem = k1 - k;
  if (rem > 0) {
    int32_t c[U];
    T a[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // past the end: the last entry again, not added
      c[u] = ci[k + min(u, rem - 1)];
      a[u] = av[k + min(u, rem - 1)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < rem) s = fma(a[u], v[u], s);
  }
  return s;
}

// Row of a sliced-ELL matrix (slices of 64 rows, entry j of a row at
// base + 64 j): the same batches of eight and the same fma order as
// row_chain1, so the row sum is identical; a wavefront's load of entry j of
// its 64 rows is one contiguous segment.
template <typename T, typename PI, typename PA, typename PX>
__device__ __forceinline__ T sell_chain(int32_t base, int32_t len, PI ci, PA av, PX x, T s) {
  constexpr int U = 8;
  int32_t j = 0;
  for (; j + U <= len; j += U) {
    int32_t c[U];
    T a[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = ci[base + 64 * (j + u)];
      a[u] = av[base + 64 * (j + u)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s = fma(a[u], v[u], s);
  }
  const int32_t rem = len - j;
  if (rem > 0) {
    int32_t c[U];
    T a[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {  // past the end: the last entry again, not added
      c[u] = ci[base + 64 * (j + min(u, rem - 1))];
      a[u] = av[base + 64 * (j + min(u, rem - 1))];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < rem) s = fma(a[u], v[u], s);
  }
  return s;
}

// Largest len over the wavefront, as a wave-uniform value.
__device__ __forceinline__ int32_t wave_max_len(int32_t len) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
  return __builtin_amdgcn_readfirstlane(len);
}

// Broadcast lane t of each quad (4 adjacent lanes) to the whole quad: DPP
// quad_perm [t,t,t,t], a VALU lane move.
template <int t>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), t * 0x55, 0xF, 0xF, false));
}
template <int t>
__device__ __forceinline__ double quad_bcast(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, t * 0x55, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), t * 0x55, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Lane t's value as a wave-uniform (scalar) value: v_readlane, no LDS
// permute.
__device__ __forceinline__ float lane_value(float v, int t) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}
__device__ __forceinline__ double lane_value(double v, int t) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, t);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), t);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

template <typename T, int G, typename PI, typename PA, typename PX>
__device__ __forceinline__ T row_chain_g(int32_t k0, int32_t len, PI ci, PA av, PX x, T s) {
  static_assert(G > 1 && G <= 64 && (64 % G) == 0, "group size");
  constexpr int U = G == 4 ? 8 : 4;
  const int q = (int)(threadIdx.x & (G - 1));
  const int32_t span = wave_max_len(len);
  const int32_t klast = len > 0 ? len - 1 : 0;
  for (int32_t base = 0; base < span; base += U * G) {
    T a[U], v[U];
    int32_t c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t kk = min(base + u * G + q, klast);
      c[u] = ci[k0 + kk];
      a[u] = av[k0 + kk];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = base + u * G;
      if (e >= span) break;  // wave-uniform
      if constexpr (G == 4) {
        const T a0 = quad_bcast<0>(a[u]), v0 = quad_bcast<0>(v[u]);
        const T a1 = quad_bcast<1>(a[u]), v1 = quad_bcast<1>(v[u]);
        const T a2 = quad_bcast<2>(a[u]), v2 = quad_bcast<2>(v[u]);
        const T a3 = quad_bcast<3>(a[u]), v3 = quad_bcast<3>(v[u]);
        if (e + 0 < len) s = fma(a0, v0, s);
        if (e + 1 < len) s = fma(a1, v1, s);
        if (e + 2 < len) s = fma(a2, v2, s);
        if (e + 3 < len) s = fma(a3, v3, s);
      } else if constexpr (G == 64) {  // one row per wavefront: scalar broadcasts
#pragma unroll
        for (int t = 0; t < 64; ++t) {
          const T at = lane_value(a[u], t);
          const T vt = lane_value(v[u], t);
          if (e + t < len) s = fma(at, vt, s);
        }
      } else {
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const T at = __shfl(a[u], t, G);
          const T vt = __shfl(v[u], t, G);
          if (e + t < len) s = fma(at, vt, s);
        }
      }
    }
  }
  return s;
}

}  // namespace pcamg
