// Solver state: levels in the colour-permuted solve layout, hierarchies, and
// the context behind the C ABI.
#pragma once

#include <array>
#include <memory>

#include "internal.hpp"

namespace pcamg {

// A level operator in the solve layout (rows grouped by colour).
struct LevelMatrix {
  int32_t n = 0, nnz = 0, ncol = 0;
  std::vector<int32_t> coff;  // host, ncol + 1
  DVec<int32_t> rp, ci;
  DVec<double> av, d, dinv;
  DVec<float> av32, d32, dinv32;
  DVec<int32_t> perm, iperm;  // position -> natural id, natural id -> position
};

// Transfer from a level to the next one (permuted numbering on both sides).
struct Transfer {
  int32_t nc = 0;
  DVec<int32_t> agg;           // [n] fine position -> coarse position
  DVec<double> pval;           // [n] or empty (boolean P)
  DVec<float> pval32;
  DVec<int32_t> moff, mem;     // [nc+1], [n]: members in ascending natural order
};

// Setup arrays of a level (natural numbering), kept only for inspection.
struct SetupLevel {
  int32_t n = 0, nnz = 0, ncol = 0, nnz_g = 0;
  DVec<int32_t> rp, ci, colour, grp, gci, nb, path_id, pos, agg;
  DVec<double> av, d, dinv, gv, gkey, pval;
};

struct Level {
  std::shared_ptr<LevelMatrix> A;
  Transfer T;
  DVec<double> x, b, r;        // work vectors (x, b unused on level 0)
  DVec<float> x32, b32, r32;
  std::array<int64_t, 16> info{};
};

struct Hierarchy {
  std::vector<Level> lv;
  // coarsest dense factor (natural order of the coarsest level)
  int32_t cn = 0, cm = 0;
  bool grounded = false, fallback = false;
  DVec<double> cL, cD;
  double op_complexity = 0.0;
  std::vector<SetupLevel> setup;  // if keep_setup
  AggStats st0;
  int32_t cover_rounds = 0;
};

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    PCAMG_HIP(hipEventCreate(&a));
    PCAMG_HIP(hipEventCreate(&b));
    PCAMG_HIP(hipEventRecord(a, s));
  }
  double ms() {
    PCAMG_HIP(hipEventRecord(b, s));
    PCAMG_HIP(hipEventSynchronize(b));
    float t = 0;
    PCAMG_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace pcamg

struct pcamg_ctx {
  hipStream_t s = nullptr;
  pcamg_params P{};
  int32_t n = 0, nnz = 0;
  // finest level, natural numbering
  pcamg::DVec<int32_t> rp, ci, colour;
  pcamg::DVec<double> av, d, dinv;
  int32_t ncol = 0;
  std::shared_ptr<pcamg::LevelMatrix> M0;  // finest level in the solve layout (shared by all hierarchies)
  // A^2 pattern of the finest level (depends on the graph only)
  bool a2_ready = false;
  int32_t nnz2 = 0, m2 = 0;
  pcamg::DVec<int32_t> rp2, ci2;
  // hierarchies (Alg. 5 P_hist)
  std::vector<std::unique_ptr<pcamg::Hierarchy>> hist;
  int32_t starts_used = 0;     // start vectors drawn from the seed stream
  pcamg::DVec<double> rhs;     // natural order
  bool have_rhs = false;
  double t_build_ms = 0.0;
};

namespace pcamg {
void ctx_init(pcamg_ctx* c, const pcamg_graph* g, const pcamg_params* p);
void ctx_validate(pcamg_ctx* c);
// Builds a hierarchy from a smooth error in natural order (device).
std::unique_ptr<Hierarchy> build_hierarchy(pcamg_ctx* c, const double* e_nat);
// Relax A e = 0 with `sweeps` symmetric sweeps, natural-order device vector in place.
void relax_homogeneous(pcamg_ctx* c, double* e_nat, int sweeps);
void initial_error(pcamg_ctx* c, int32_t r, double* e_nat);
// Cycles on the solve layout (level-0 vectors in permuted order).
void cycle64(pcamg_ctx* c, Hierarchy& H, int l, const double* b, double* x, int gamma);
void cycle32(pcamg_ctx* c, Hierarchy& H, int l, const float* b, float* x);
// Alg. 2 on permuted vectors.
void approx_error(pcamg_ctx* c, int Re, const double* r, double* e, int* wcycles, int* vcycles);
void bench_smoother(pcamg_ctx* c, int prec, int sweeps, double* ms, int64_t* launches, double* bytes);
void solve(pcamg_ctx* c, double* x_nat, pcamg_stats* st);
}  // namespace pcamg
