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
  int32_t lanes = 1;          // lanes per row in the smoother and residual kernels
  std::vector<int32_t> coff;  // host, ncol + 1
  DVec<int32_t> rp, ci;
  DVec<double> av, d, dinv;
  DVec<float> av32, d32, dinv32;
  DVec<int32_t> perm, iperm;  // position -> natural id, natural id -> position
  // sliced-ELL copy for the launched passes of short-row levels (woff empty:
  // none); rp still gives the row lengths
  DVec<int32_t> woff, sci;
  DVec<double> sav;
  DVec<float> sav32;
  bool sell() const { return woff.p != nullptr; }
  // rows of at least long_min entries (0: none), first within their colour:
  // lend[c] = end of colour c's long rows; long_rows = all of them
  int32_t long_min = 0, nlong = 0;
  std::vector<int32_t> lend;
  DVec<int32_t> long_rows;
  // padded-row FP32 copy for the FP32 passes of lane-group levels (ell_w = 0: none)
  int32_t ell_w = 0;
  DVec<int32_t> eci;
  DVec<float> eav32;
  // many colours of a few rows each: a whole sweep in one single-workgroup
  // launch (colour offsets and long-row ends on the device)
  bool block_sweep = false;
  DVec<int32_t> coff_d, lend_d;
};

// Gauss-Seidel pass over colour k and residual (b == nullptr: product) of a
// level matrix, on its sliced-ELL copy when it has one.
// chain: every row by the single fma chain in stored order (the relaxation
// before a build), long rows included (a wavefront of 64 lanes each).
void smooth_colour(const LevelMatrix& A, int k, const double* b, double* x, hipStream_t s, bool chain = false);
void smooth_colour(const LevelMatrix& A, int k, const float* b, float* x, hipStream_t s, bool chain = false);
void level_residual(const LevelMatrix& A, const double* b, const double* x, double* r, hipStream_t s);
void level_residual(const LevelMatrix& A, const float* b, const float* x, float* r, hipStream_t s);

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

// Level descriptor for the single-workgroup tail kernel (device memory).  The
// vectors (x, b, r) of the smaller tail levels, the dense solve's accumulator
// and, when it fits, the coarsest factor live in the workgroup's LDS for the
// duration of a launch (o64 / o32: element offsets in the LDS pool seen as
// double / float); the larger tail levels keep theirs in global memory.
constexpr int TAIL_MAX_LEVELS = 40;
constexpr int LDLT_MAX = 4096;
constexpr int TAIL_LDS_BYTES = 128 * 1024;
constexpr int TAIL_COFF_MAX = 2048;
struct TailLevel {
  int32_t n, ncol, lds, ocoff, lanes;  // lanes per row: 1 or 16
  int32_t nnz;
  int32_t o64[3], o32[3];  // x, b, r in LDS (lds = 1)
  const int32_t *coff, *rp, *ci, *agg, *moff, *mem;
  const double *av, *d, *dinv, *pval;
  const float *av32, *d32, *dinv32, *pval32;
  double *x, *b, *r;       // in global memory (lds = 0)
  float *x32, *b32, *r32;
};
struct TailDesc {
  int32_t nlev;  // tail levels including the coarsest
  int32_t cn, cm, grounded;
  int32_t oacc64, oacc32;  // accumulator offsets (doubles) in the two layouts
  int32_t oL64, oL32;      // factor L offsets (doubles), -1 = read from global memory
  int32_t ncoff;
  const double *L, *D;
  TailLevel lv[TAIL_MAX_LEVELS];
};

struct Hierarchy {
  std::vector<Level> lv;
  // tail: levels tail_start.. run in one workgroup launch
  int tail_start = -1;
  DVec<TailDesc> tail_desc;
  // W-cycles: the level whose two sub-cycles the level above applies as one
  // dense operator (column-major, built on first use); 0: the whole cycle
  // of a small graph as one operator, applied as x += C (b - A x)
  int dense_start = -1;
  DVec<double> C64, dpart64;
  DVec<float> C32, dpart32;
  // V-cycles: the level whose cycle the level above applies as one dense
  // operator (column-major, built on first use); 0: as dense_start
  int dense_v_start = -1;
  DVec<double> CV64, dvpart64;
  DVec<float> CV32, dvpart32;
  std::vector<DVec<int32_t>> coff_dev;
  // captured top-level cycles (fixed input/output buffers)
  hipGraphExec_t g64v = nullptr, g64w = nullptr, g32v = nullptr, g32w = nullptr;
  DVec<double> gb, gx;
  DVec<float> gb32, gx32;
  ~Hierarchy() {
    if (g64v) (void)hipGraphExecDestroy(g64v);
    if (g64w) (void)hipGraphExecDestroy(g64w);
    if (g32v) (void)hipGraphExecDestroy(g32v);
    if (g32w) (void)hipGraphExecDestroy(g32w);
  }
  // coarsest dense factor (natural order of the coarsest level)
  int32_t cn = 0, cm = 0;
  bool grounded = false, fallback = false;
  DVec<double> cL, cD;
  double op_complexity = 0.0;
  std::vector<SetupLevel> setup;  // if keep_setup
  DVec<double> source;             // if keep_setup: the build's vector before the sweeps (natural order)
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
  hipStream_t capture_stream = nullptr;  // private stream used only to capture cycle graphs
  ~pcamg_ctx() {
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
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
  // learned proposals (pcamg_setup_learned): the caller's network (not owned)
  // and the graph weights its features need
  pcamg_net* net = nullptr;
  pcamg::DVec<double> w;
  double t_build_ms = 0.0;
};

namespace pcamg {
void ctx_init(pcamg_ctx* c, const pcamg_graph* g, const pcamg_params* p);
void ctx_validate(pcamg_ctx* c);
// Builds a hierarchy from a smooth error in natural order (device).
std::unique_ptr<Hierarchy> build_hierarchy(pcamg_ctx* c, const double* e_nat);
// The UA-AMG hierarchy of MWM aggregation (init = PCAMG_INIT_MWM).
std::unique_ptr<Hierarchy> build_hierarchy_mwm(pcamg_ctx* c);
// Relax A e = 0 with `sweeps` symmetric sweeps, natural-order device vector in place.
void relax_homogeneous(pcamg_ctx* c, double* e_nat, int sweeps);
void initial_error(pcamg_ctx* c, int32_t r, double* e_nat, int32_t sweeps = -1);  // sweeps < 0: relax_sweeps

// learned smooth-error network (learned.hip)
int32_t net_num_params();
void net_create(pcamg_net** out);
void net_destroy(pcamg_net* net);
void net_set_params(pcamg_net* net, const float* host, hipStream_t s);
void net_init(pcamg_net* net, uint64_t seed, hipStream_t s);
void net_get_params(pcamg_net* net, float* host, hipStream_t s);
void net_forward_f32(pcamg_net* net, const pcamg_graph* g, const double* e2, float* y, hipStream_t s);
void net_forward_f64(pcamg_net* net, const pcamg_graph* g, const double* e2, double* e, hipStream_t s);
double net_loss_grad(pcamg_net* net, const pcamg_graph* g, const double* e2, const double* target, float* grad_host,
                     hipStream_t s);
void net_adam(pcamg_net* net, float lr, hipStream_t s);
// Cycles on the solve layout (level-0 vectors in permuted order).
void cycle64(pcamg_ctx* c, Hierarchy& H, int l, const double* b, double* x, int gamma, int skip = 0);
void cycle32(pcamg_ctx* c, Hierarchy& H, int l, const float* b, float* x, int gamma, int skip = 0);
// Whole cycles on level-0 vectors (solve layout), replayed from captured graphs.
void run_cycle64(pcamg_ctx* c, Hierarchy& H, const double* b, double* x, int gamma);
void run_cycle32(pcamg_ctx* c, Hierarchy& H, const float* b, float* x, int gamma);
void tail_cycle64(const Hierarchy& H, const double* b, double* x, int gamma, hipStream_t s);
void tail_cycle32(const Hierarchy& H, const float* b, float* x, int gamma, hipStream_t s);

// dense.hip: the dense operator of `calls` (1, or gamma) calls of level d's
// cycle (gamma = 1: V, 2: W) from x = 0, built level by level from the
// coarsest up (GEMMs for the products with dense operators); column-major
// into C (n_d^2).
bool dense_bottom_up_fits(const Hierarchy& H, int d);
template <typename T>
void dense_bottom_up(Hierarchy& H, int d, int gamma, T* C, hipStream_t s, int calls);

// y = C b, or y += C b with add
template <typename T>
void dense_apply(int32_t n, const T* C, const T* b, T* part, T* y, hipStream_t s, bool add = false);
int32_t dense_chunks(int32_t n);
// Alg. 2 on permuted vectors.
void approx_error(pcamg_ctx* c, int Re, const double* r, double* e, int* wcycles, int* vcycles, int* vcycles32);
void bench_smoother(pcamg_ctx* c, int prec, int sweeps, double* ms, int64_t* launches, double* bytes);
void bench_level(pcamg_ctx* c, int kind, int prec, int reps, int64_t flush_bytes, double* ms, int64_t* launches,
                 double* bytes);
double bench_copy(int64_t nbytes, int reps, hipStream_t s);
// reps products P = Q R (p x q times q x r, row-major) by the dense operators'
// MFMA GEMM in FP64 or FP32 (prec), timed with HIP events; milliseconds
double bench_gemm(int32_t p, int32_t q, int32_t r, int prec, int reps, hipStream_t s);
void solve(pcamg_ctx* c, double* x_nat, pcamg_stats* st);
}  // namespace pcamg
