// Solve-phase layout: every level is stored with its rows grouped by colour
// (stable: ascending natural id within a colour), so one Gauss-Seidel pass per
// colour streams a contiguous block of rows.  Row entries keep their natural
// column order, so every fma chain runs in the same order as in natural
// numbering and results are identical bit for bit.
#include "internal.hpp"

namespace pcamg {

__global__ void coff_kernel(int32_t n, int32_t ncol, const uint32_t* __restrict__ keys, int32_t* __restrict__ coff,
                            int32_t* __restrict__ bad) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t k = keys[p];
  if (k >= (uint32_t)ncol) {
    atomicOr(bad, 1);
    return;
  }
  if (p == 0 || keys[p - 1] != k) coff[k] = p;
  if (p == n - 1) coff[k + 1] = n;
}

__global__ void iperm_kernel(int32_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ iperm) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) iperm[perm[p]] = p;
}

// perm[p] = natural id at position p, iperm its inverse, coff[c] = first row of
// colour c.  Keys must be 0..ncol-1 with every value present.
void build_perm(int32_t n, const int32_t* colour, int32_t ncol, int32_t* perm, int32_t* iperm,
                std::vector<int32_t>& coff, hipStream_t s) {
  require(n > 0 && ncol >= 1, PCAMG_EINVAL, "build_perm: empty input");
  DVec<uint32_t> ks(n), vs(n), ko(n);
  copy_d2d(ks.p, (const uint32_t*)colour, n, s);
  iota_i32((int32_t*)vs.p, n, s);
  int bits = 1;
  while ((1ll << bits) < ncol) ++bits;
  // a key >= ncol may sort out of place on the low bits but is rejected below
  radix_sort_u32_u32(ks.p, vs.p, ko.p, (uint32_t*)perm, n, bits, s);
  DVec<int32_t> co(ncol + 1), bad(1);
  fill_i32(co.p, -1, ncol + 1, s);
  fill_i32(bad.p, 0, 1, s);
  coff_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, ncol, ko.p, co.p, bad.p);
  PCAMG_LAUNCHED();
  require(read_scalar(bad.p, s) == 0, PCAMG_EINVAL, "key (colour or aggregate id) out of range");
  iperm_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, iperm);
  PCAMG_LAUNCHED();
  coff = to_host(co.p, ncol + 1, s);
  bool ok = coff[0] == 0 && coff[ncol] == n;
  for (int32_t c = 0; c < ncol && ok; ++c) ok = coff[c] >= 0 && coff[c] <= coff[c + 1];
  require(ok, PCAMG_EINVAL, "keys must take every value 0..ncol-1");
}

__global__ void long_key_kernel(int32_t n, const int32_t* __restrict__ colour, const int32_t* __restrict__ rp,
                                int32_t long_min, uint32_t* __restrict__ key) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) key[v] = 2u * (uint32_t)colour[v] + (rp[v + 1] - rp[v] >= long_min ? 0u : 1u);
}

// first position of every key present (start[k] = -1 for keys absent)
__global__ void key_start_kernel(int32_t n, int32_t nkeys, const uint32_t* __restrict__ keys,
                                 int32_t* __restrict__ start, int32_t* __restrict__ bad) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t k = keys[p];
  if (k >= (uint32_t)nkeys) {
    atomicOr(bad, 1);
    return;
  }
  if (p == 0 || keys[p - 1] != k) start[k] = p;
}

void build_perm_long(int32_t n, const int32_t* colour, int32_t ncol, const int32_t* rp, int32_t long_min,
                     int32_t* perm, int32_t* iperm, std::vector<int32_t>& coff, std::vector<int32_t>& lend,
                     hipStream_t s) {
  require(n > 0 && ncol >= 1 && long_min > 0, PCAMG_EINVAL, "build_perm_long: bad input");
  const int32_t nkeys = 2 * ncol;
  DVec<uint32_t> ks(n), vs(n), ko(n);
  long_key_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, colour, rp, long_min, ks.p);
  PCAMG_LAUNCHED();
  iota_i32((int32_t*)vs.p, n, s);
  int bits = 1;
  while ((1ll << bits) < nkeys) ++bits;
  radix_sort_u32_u32(ks.p, vs.p, ko.p, (uint32_t*)perm, n, bits, s);
  DVec<int32_t> st(nkeys), bad(1);
  fill_i32(st.p, -1, nkeys, s);
  fill_i32(bad.p, 0, 1, s);
  key_start_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, nkeys, ko.p, st.p, bad.p);
  PCAMG_LAUNCHED();
  require(read_scalar(bad.p, s) == 0, PCAMG_EINVAL, "colour out of range");
  iperm_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, iperm);
  PCAMG_LAUNCHED();
  std::vector<int32_t> start = to_host(st.p, nkeys, s);
  // absent keys start where the next present one does
  int32_t next = n;
  for (int32_t k = nkeys - 1; k >= 0; --k) {
    if (start[k] < 0) start[k] = next;
    next = start[k];
  }
  coff.assign(ncol + 1, n);
  lend.assign(ncol, n);
  for (int32_t c = 0; c < ncol; ++c) {
    coff[c] = start[2 * c];
    lend[c] = start[2 * c + 1];
  }
  bool ok = coff[0] == 0;
  for (int32_t c = 0; c < ncol && ok; ++c) ok = coff[c] <= lend[c] && lend[c] <= coff[c + 1] && coff[c] < coff[c + 1];
  require(ok, PCAMG_EINVAL, "colours must take every value 0..ncol-1");
}

__global__ void perm_deg_kernel(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ rp,
                                int32_t* __restrict__ deg) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) deg[p] = rp[perm[p] + 1] - rp[perm[p]];
}

// Row p of the permuted matrix is row perm[p] with its columns renumbered;
// rows of more than PERM_LONG entries are copied by perm_rows_long_kernel.
constexpr int32_t PERM_LONG = 256;

__global__ void perm_rows_kernel(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ iperm,
                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ av, const int32_t* __restrict__ rpp,
                                 int32_t* __restrict__ cip, double* __restrict__ avp, float* __restrict__ avp32) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = perm[p];
  if (rp[i + 1] - rp[i] > PERM_LONG) return;
  int32_t o = rpp[p];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k, ++o) {
    cip[o] = iperm[ci[k]];
    avp[o] = av[k];
    avp32[o] = (float)av[k];
  }
}

__global__ void __launch_bounds__(256)
    perm_rows_long_kernel(const int32_t* __restrict__ pos, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ iperm, const int32_t* __restrict__ rp,
                          const int32_t* __restrict__ ci, const double* __restrict__ av,
                          const int32_t* __restrict__ rpp, int32_t* __restrict__ cip, double* __restrict__ avp,
                          float* __restrict__ avp32) {
  const int32_t p = pos[blockIdx.x];
  const int32_t i = perm[p];
  const int32_t k0 = rp[i], len = rp[i + 1] - k0, o = rpp[p];
  for (int32_t j = (int32_t)threadIdx.x; j < len; j += 256) {
    cip[o + j] = iperm[ci[k0 + j]];
    const double a = av[k0 + j];
    avp[o + j] = a;
    avp32[o + j] = (float)a;
  }
}

__global__ void perm_diag_kernel(int32_t n, const int32_t* __restrict__ perm, const double* __restrict__ d,
                                 const double* __restrict__ dinv, double* __restrict__ dp, double* __restrict__ dinvp,
                                 float* __restrict__ dp32, float* __restrict__ dinvp32) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = perm[p];
  dp[p] = d[i];
  dinvp[p] = dinv[i];
  dp32[p] = (float)d[i];
  dinvp32[p] = (float)dinv[i];
}

void permute_csr(int32_t n, const int32_t* perm, const int32_t* iperm, const int32_t* rp, const int32_t* ci,
                 const double* av, const double* d, const double* dinv, int32_t* rpp, int32_t* cip, double* avp,
                 float* avp32, double* dp, double* dinvp, float* dp32, float* dinvp32, hipStream_t s) {
  if (n <= 0) return;
  DVec<int32_t> deg(n);
  perm_deg_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, rp, deg.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(deg.p, rpp, n, rpp + n, s);
  perm_rows_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, iperm, rp, ci, av, rpp, cip, avp, avp32);
  PCAMG_LAUNCHED();
  DVec<int32_t> lpos;
  const int32_t nl = rows_longer_than(n, rp, perm, PERM_LONG, lpos, s);
  if (nl > 0) {
    perm_rows_long_kernel<<<nl, 256, 0, s>>>(lpos.p, perm, iperm, rp, ci, av, rpp, cip, avp, avp32);
    PCAMG_LAUNCHED();
  }
  perm_diag_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, d, dinv, dp, dinvp, dp32, dinvp32);
  PCAMG_LAUNCHED();
}

__global__ void perm_agg_kernel(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ agg,
                                const int32_t* __restrict__ ipermc, const double* __restrict__ pval,
                                int32_t* __restrict__ aggp, double* __restrict__ pvalp, float* __restrict__ pvalp32) {
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = perm[p];
  aggp[p] = ipermc ? ipermc[agg[i]] : agg[i];
  if (pval) {
    pvalp[p] = pval[i];
    pvalp32[p] = (float)pval[i];
  }
}

__global__ void perm_msz_kernel(int32_t nc, const int32_t* __restrict__ permc, const int32_t* __restrict__ moff,
                                int32_t* __restrict__ sz) {
  int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int32_t I = permc ? permc[q] : q;
  sz[q] = moff[I + 1] - moff[I];
}

__global__ void perm_mem_kernel(int32_t nc, const int32_t* __restrict__ permc, const int32_t* __restrict__ moff,
                                const int32_t* __restrict__ mem, const int32_t* __restrict__ iperm,
                                const int32_t* __restrict__ moffp, int32_t* __restrict__ memp) {
  int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int32_t I = permc ? permc[q] : q;
  int32_t o = moffp[q];
  for (int32_t t = moff[I]; t < moff[I + 1]; ++t, ++o) memp[o] = iperm[mem[t]];
}

// Transfer of level l in permuted numbering: fine positions -> coarse
// positions; members of each coarse position keep ascending natural order.
void permute_transfer(int32_t n, const int32_t* perm, const int32_t* iperm, int32_t nc, const int32_t* permc,
                      const int32_t* ipermc, const int32_t* agg, const double* pval, const int32_t* moff,
                      const int32_t* mem, int32_t* aggp, double* pvalp, float* pvalp32, int32_t* moffp,
                      int32_t* memp, hipStream_t s) {
  perm_agg_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, perm, agg, ipermc, pval, aggp, pvalp, pvalp32);
  PCAMG_LAUNCHED();
  DVec<int32_t> sz(nc);
  perm_msz_kernel<<<grid_for(nc, 256), 256, 0, s>>>(nc, permc, moff, sz.p);
  PCAMG_LAUNCHED();
  scan_exclusive_i32(sz.p, moffp, nc, moffp + nc, s);
  perm_mem_kernel<<<grid_for(nc, 256), 256, 0, s>>>(nc, permc, moff, mem, iperm, moffp, memp);
  PCAMG_LAUNCHED();
}

}  // namespace pcamg
