// Host orchestration: hierarchy construction (Alg. 4), multigrid cycles, the
// error approximation (Alg. 2) and the adaptive loop (Alg. 5, plus the FCG
// variant).  All arithmetic runs in the kernels of this library; the host only
// sequences launches and reads back scalars (sizes, norms, step lengths).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "solver.hpp"

namespace pcamg {

namespace {

// Lanes per row for the smoother and residual kernels: one thread per row for
// short rows, cooperating lane groups for the long rows of coarse operators,
// where the launch is latency-bound and a row's entries should arrive in one
// or two round trips (measured on the 3D grid hierarchies).
int32_t pick_lanes(int32_t n, int32_t nnz, int32_t forced) {
  if (forced) return forced;
  const double avg = n > 0 ? (double)nnz / n : 0.0;
  return avg <= 10.0 ? 1 : avg <= 24.0 ? 4 : 16;
}

// Levels at most this size run in the single-workgroup tail or are latency
// bound: no sliced-ELL copy.
constexpr int32_t SELL_MIN_N = 4096;
// A hierarchy built from the network's proposal whose first measured
// convergence factor exceeds this gives the next re-setup back to the plain
// relaxation (the network stays only while the convergence it delivers holds).
constexpr double LEARNED_FALLBACK_CONVR = 0.9;
// Levels at most this size are not timed by the lanes autotuner (they run in
// the tail kernel by default).
constexpr int32_t TUNE_MIN_N = 2048;
// Rows per colour below which a level of up to twice v_dense_max_n rows
// still joins the V-cycle's dense operator.
constexpr int32_t V_DENSE_ROWS_PER_COLOUR = 16;
// Largest top_dense_max_n: graphs of at most this many vertices may run each
// cycle type as one dense operator of the whole cycle (n^2 entries per type
// and precision).
constexpr int32_t TOP_DENSE_MAX_N = 2048;

// A level of at least block_sweep_min_colours colours (a parameter), with at
// most this many rows per colour on average, runs its sweeps in one
// single-workgroup launch.
constexpr int32_t BLOCK_SWEEP_ROWS_PER_COLOUR = 64;

// Autotuned lanes per row (row_lanes = -1).  Candidates: one thread per row
// (on the sliced-ELL copy when the level has one), 4 and 16 lanes per row.
// Each runs one symmetric FP32 sweep of the level as a warm-up and two timed
// with HIP events on the level's stream; the fastest is kept.  Every candidate
// sums each row in the same order, so the choice changes the time only.
// Decisions are cached for the life of the process by level shape: size in
// quarter octaves, mean row length in halves, number of colours.
struct LaneShape {
  int32_t logn4, mean2, ncol;
  bool operator<(const LaneShape& o) const {
    return logn4 != o.logn4 ? logn4 < o.logn4 : mean2 != o.mean2 ? mean2 < o.mean2 : ncol < o.ncol;
  }
};
std::mutex g_lane_mu;
std::map<LaneShape, int32_t> g_lane_cache;

int32_t tune_lanes(const LevelMatrix& M, hipStream_t s) {
  const LaneShape key{(int32_t)std::lround(4.0 * std::log2((double)M.n)),
                      (int32_t)std::lround(2.0 * (double)M.nnz / M.n), M.ncol};
  {
    std::lock_guard<std::mutex> lk(g_lane_mu);
    auto it = g_lane_cache.find(key);
    if (it != g_lane_cache.end()) return it->second;
  }
  DVec<float> b(M.n), x(M.n);
  fill_f32(b.p, 1.0f, M.n, s);
  fill_f32(x.p, 0.0f, M.n, s);
  auto pass = [&](int k, int lanes) {
    if (lanes == 1 && M.sell())
      gs_colour_sell<float>(M.coff[k], M.coff[k + 1], M.rp.p, M.woff.p, M.sci.p, M.sav32.p, M.dinv32.p, b.p, x.p, s);
    else  // the long rows (if any) take their own kernel whatever the lanes
      gs_colour<float>(M.long_min > 0 ? M.lend[k] : M.coff[k], M.coff[k + 1], M.rp.p, M.ci.p, M.av32.p,
                       M.dinv32.p, b.p, x.p, s, lanes);
  };
  auto sweep = [&](int lanes) {
    for (int k = 0; k < M.ncol; ++k) pass(k, lanes);
    for (int k = M.ncol - 1; k >= 0; --k) pass(k, lanes);
  };
  int32_t best = 1;
  double best_ms = 0.0;
  for (int lanes : {1, 4, 16}) {
    sweep(lanes);
    Timer t(s);
    sweep(lanes);
    sweep(lanes);
    const double ms = t.ms();
    if (lanes == 1 || ms < best_ms) {
      best = lanes;
      best_ms = ms;
    }
  }
  std::lock_guard<std::mutex> lk(g_lane_mu);
  g_lane_cache.emplace(key, best);
  return best;
}

std::shared_ptr<LevelMatrix> make_level_matrix(int32_t n, int32_t nnz, const int32_t* rp, const int32_t* ci,
                                               const double* av, const double* d, const double* dinv,
                                               const int32_t* colour, int32_t ncol, int32_t row_lanes,
                                               int32_t long_min, int32_t block_min_colours, hipStream_t s) {
  auto M = std::make_shared<LevelMatrix>();
  M->n = n;
  M->nnz = nnz;
  const bool tune = row_lanes < 0 && n > TUNE_MIN_N && ncol >= 1;
  M->lanes = pick_lanes(n, nnz, row_lanes < 0 ? 0 : row_lanes);
  M->perm.resize(n);
  M->iperm.resize(n);
  // levels with long rows (and launched passes: the single-workgroup tail
  // keeps its own loops) put them first in each colour
  if (colour && long_min > 0 && n > TUNE_MIN_N && max_row_len(n, rp, s) >= long_min) {
    build_perm_long(n, colour, ncol, rp, long_min, M->perm.p, M->iperm.p, M->coff, M->lend, s);
    M->ncol = ncol;
    M->long_min = long_min;
    std::vector<int32_t> rows;
    for (int32_t c = 0; c < ncol; ++c)
      for (int32_t r = M->coff[c]; r < M->lend[c]; ++r) rows.push_back(r);
    M->nlong = (int32_t)rows.size();
    M->long_rows.resize(rows.size());
    copy_h2d(M->long_rows.p, rows.data(), rows.size(), s);
    PCAMG_HIP(hipStreamSynchronize(s));  // rows is a host temporary
  } else if (colour) {
    build_perm(n, colour, ncol, M->perm.p, M->iperm.p, M->coff, s);
    M->ncol = ncol;
  } else {
    iota_i32(M->perm.p, n, s);
    iota_i32(M->iperm.p, n, s);
    M->coff = {0, n};
    M->ncol = 1;
  }
  M->rp.resize(n + 1);
  // one zero pad slot at nnz: the lane-group chains load past a row's end
  M->ci.resize((size_t)nnz + 1);
  M->av.resize((size_t)nnz + 1);
  M->av32.resize((size_t)nnz + 1);
  fill_i32(M->ci.p + nnz, 0, 1, s);
  fill_f64(M->av.p + nnz, 0.0, 1, s);
  fill_f32(M->av32.p + nnz, 0.0f, 1, s);
  M->d.resize(n);
  M->dinv.resize(n);
  M->d32.resize(n);
  M->dinv32.resize(n);
  permute_csr(n, M->perm.p, M->iperm.p, rp, ci, av, d, dinv, M->rp.p, M->ci.p, M->av.p, M->av32.p, M->d.p,
              M->dinv.p, M->d32.p, M->dinv32.p, s);
  // short rows on a level large enough for launched passes: sliced-ELL copy
  // (the autotuner tries it on every level it times)
  if ((M->lanes == 1 || tune) && n > SELL_MIN_N && M->long_min == 0)
    sell_build(n, nnz, M->rp.p, M->ci.p, M->av.p, M->av32.p, M->woff, M->sci, M->sav, M->sav32, s);
  if (tune) {
    M->lanes = tune_lanes(*M, s);
    if (M->lanes != 1 && M->sell()) {
      M->woff.resize(0);
      M->sci.resize(0);
      M->sav.resize(0);
      M->sav32.resize(0);
    }
  }
  // launched lane-group levels without long rows: padded-row FP32 copy
  if (n > TUNE_MIN_N && M->long_min == 0 && !M->sell() && (M->lanes == 4 || M->lanes == 16))
    ell_build(n, M->lanes, M->rp.p, M->ci.p, M->av32.p, M->ell_w, M->eci, M->eav32, s);
  // many colours with a few rows each (near-dense coarse levels of power-law
  // graphs: hundreds of colours): a sweep runs in one single-workgroup launch
  // instead of one or two launches per colour
  if (colour && !M->sell() && block_min_colours > 0 && M->ncol >= block_min_colours &&
      (int64_t)n <= (int64_t)BLOCK_SWEEP_ROWS_PER_COLOUR * M->ncol) {
    M->block_sweep = true;
    M->coff_d.resize(M->ncol + 1);
    M->lend_d.resize(M->ncol);
    std::vector<int32_t> lend = M->long_min > 0 ? M->lend : std::vector<int32_t>(M->coff.begin(), M->coff.end() - 1);
    copy_h2d(M->coff_d.p, M->coff.data(), M->ncol + 1, s);
    copy_h2d(M->lend_d.p, lend.data(), M->ncol, s);
    PCAMG_HIP(hipStreamSynchronize(s));  // lend is a host temporary
  }
  return M;
}

// One level of the setup in natural numbering.
struct NatLevel {
  int32_t n = 0, nnz = 0, ncol = 0, nnz_g = 0;
  const int32_t *rp = nullptr, *ci = nullptr, *colour = nullptr, *grp = nullptr, *gci = nullptr, *nb = nullptr;
  const double *av = nullptr, *d = nullptr, *dinv = nullptr, *gv = nullptr, *gkey = nullptr;
  DVec<int32_t> o_rp, o_ci, o_colour, o_grp, o_gci, o_nb;
  DVec<double> o_av, o_d, o_dinv, o_gv;
  // transfer
  int32_t nc = 0;
  DVec<int32_t> agg, moff, mem, pid, pos, plen;
  DVec<double> pval;
  AggStats st;
};

void sync(hipStream_t s) { PCAMG_HIP(hipStreamSynchronize(s)); }

}  // namespace

void smooth_colour(const LevelMatrix& A, int k, const double* b, double* x, hipStream_t s, bool chain) {
  if (A.sell()) {
    gs_colour_sell<double>(A.coff[k], A.coff[k + 1], A.rp.p, A.woff.p, A.sci.p, A.sav.p, A.dinv.p, b, x, s);
  } else if (A.long_min > 0) {  // long rows first: a workgroup each, or one wavefront's chain
    if (chain)
      gs_colour_chain_long<double>(A.coff[k], A.lend[k], A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s);
    else {  // both parts in one launch
      gs_colour_fused<double>(A.coff[k], A.lend[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s, A.lanes);
      return;
    }
    gs_colour<double>(A.lend[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s, A.lanes);
  } else {
    gs_colour<double>(A.coff[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s, A.lanes);
  }
}

void smooth_colour(const LevelMatrix& A, int k, const float* b, float* x, hipStream_t s, bool chain) {
  if (A.sell()) {
    gs_colour_sell<float>(A.coff[k], A.coff[k + 1], A.rp.p, A.woff.p, A.sci.p, A.sav32.p, A.dinv32.p, b, x, s);
  } else if (A.ell_w > 0) {
    gs_colour_ell(A.coff[k], A.coff[k + 1], A.ell_w, A.lanes, A.rp.p, A.eci.p, A.eav32.p, A.dinv32.p, b, x, s);
  } else if (A.long_min > 0) {  // long rows first: a workgroup each, or one wavefront's chain
    if (chain)
      gs_colour_chain_long<float>(A.coff[k], A.lend[k], A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x, s);
    else {  // both parts in one launch
      gs_colour_fused<float>(A.coff[k], A.lend[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x, s, A.lanes);
      return;
    }
    gs_colour<float>(A.lend[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x, s, A.lanes);
  } else {
    gs_colour<float>(A.coff[k], A.coff[k + 1], A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x, s, A.lanes);
  }
}

void level_residual(const LevelMatrix& A, const double* b, const double* x, double* r, hipStream_t s) {
  if (A.sell()) {
    residual_sell<double>(A.n, A.rp.p, A.woff.p, A.sci.p, A.sav.p, A.d.p, b, x, r, s);
  } else {
    residual<double>(A.n, A.rp.p, A.ci.p, A.av.p, A.d.p, b, x, r, s, A.lanes, A.long_min);
    residual_long<double>(A.nlong, A.long_rows.p, A.rp.p, A.ci.p, A.av.p, A.d.p, b, x, r, s);
  }
}

void level_residual(const LevelMatrix& A, const float* b, const float* x, float* r, hipStream_t s) {
  if (A.sell()) {
    residual_sell<float>(A.n, A.rp.p, A.woff.p, A.sci.p, A.sav32.p, A.d32.p, b, x, r, s);
  } else {
    residual<float>(A.n, A.rp.p, A.ci.p, A.av32.p, A.d32.p, b, x, r, s, A.lanes, A.long_min);
    residual_long<float>(A.nlong, A.long_rows.p, A.rp.p, A.ci.p, A.av32.p, A.d32.p, b, x, r, s);
  }
}

// One multicoloured Gauss-Seidel sweep of a level inside a cycle: colours
// skip..C-1 (forward) or C-1..0 (backward).
void smooth_sweep(const LevelMatrix& A, bool forward, int skip, const double* b, double* x, hipStream_t s) {
  if (A.block_sweep) {
    if (forward) gs_sweep_block<double>(skip, A.ncol, 1, A.coff_d.p, A.lend_d.p, A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s);
    else gs_sweep_block<double>(A.ncol - 1, -1, -1, A.coff_d.p, A.lend_d.p, A.rp.p, A.ci.p, A.av.p, A.dinv.p, b, x, s);
    return;
  }
  if (forward)
    for (int k = skip; k < A.ncol; ++k) smooth_colour(A, k, b, x, s);
  else
    for (int k = A.ncol - 1; k >= 0; --k) smooth_colour(A, k, b, x, s);
}

void smooth_sweep(const LevelMatrix& A, bool forward, int skip, const float* b, float* x, hipStream_t s) {
  if (A.block_sweep) {
    if (forward)
      gs_sweep_block<float>(skip, A.ncol, 1, A.coff_d.p, A.lend_d.p, A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x, s);
    else
      gs_sweep_block<float>(A.ncol - 1, -1, -1, A.coff_d.p, A.lend_d.p, A.rp.p, A.ci.p, A.av32.p, A.dinv32.p, b, x,
                            s);
    return;
  }
  if (forward)
    for (int k = skip; k < A.ncol; ++k) smooth_colour(A, k, b, x, s);
  else
    for (int k = A.ncol - 1; k >= 0; --k) smooth_colour(A, k, b, x, s);
}

void ctx_init(pcamg_ctx* c, const pcamg_graph* g, const pcamg_params* p) {
  hipStream_t s = c->s;
  c->P = *p;
  c->n = g->n;
  c->nnz = g->nnz;
  const int32_t n = g->n, nnz = g->nnz;
  c->rp.resize(n + 1);
  c->ci.resize(nnz);
  c->av.resize(nnz);
  c->d.resize(n);
  c->dinv.resize(n);
  c->colour.resize(n);
  copy_d2d(c->rp.p, g->row_ptr, n + 1, s);
  copy_d2d(c->ci.p, g->col_idx, nnz, s);
  laplacian(n, c->rp.p, g->weight, c->av.p, c->d.p, c->dinv.p, nnz, s);
  c->ncol = colour_level(n, c->rp.p, c->ci.p, c->P.colour_seed, 0, c->colour.p, s);
  c->M0 = make_level_matrix(n, nnz, c->rp.p, c->ci.p, c->av.p, c->d.p, c->dinv.p, c->colour.p, c->ncol,
                            c->P.row_lanes, c->P.long_row_min, c->P.block_sweep_min_colours, s);
  sync(s);
}

// Descriptor of the sub-hierarchy from level `start` to the coarsest for the
// single-workgroup kernels.  LDS takes the vectors of the coarsest and of as
// many levels above it as fit (FP64 layout, the larger one); the levels above
// those keep theirs in global memory.  False if the coarsest does not fit.
static bool make_tail_desc(Hierarchy& H, int start, TailDesc& D, hipStream_t s) {
  const int nl = (int)H.lv.size();
  const int64_t budget = TAIL_LDS_BYTES / 8;  // doubles
  // accumulator of cn doubles (the grounded solve sets its last entry), factor
  const int64_t fixed = (int64_t)H.cn + (H.cm <= 64 ? (int64_t)H.cm * H.cm : 0);
  if (3 * (int64_t)H.cn + fixed > budget) return false;
  std::memset(&D, 0, sizeof(D));
  D.nlev = nl - start;
  D.cn = H.cn;
  D.cm = H.cm;
  D.grounded = H.grounded ? 1 : 0;
  D.L = H.cL.p;
  D.D = H.cD.p;
  int first_lds = nl - 1;
  int64_t used = 3 * (int64_t)H.cn + fixed;
  while (first_lds > start && used + 3 * (int64_t)H.lv[first_lds - 1].A->n <= budget) {
    --first_lds;
    used += 3 * (int64_t)H.lv[first_lds].A->n;
  }
  int32_t o64 = 0, o32 = 0, oco = 0;
  for (int l = start; l < nl; ++l) {
    Level& V = H.lv[l];
    const LevelMatrix& A = *V.A;
    TailLevel& T = D.lv[l - start];
    T.n = A.n;
    T.nnz = A.nnz;
    T.ncol = A.ncol;
    T.lds = l >= first_lds ? 1 : 0;
    // one workgroup: one thread per row measured fastest for rows of up to
    // ~50 entries (grid hierarchies); the near-dense coarse rows of
    // power-law graphs take 16 lanes per row
    T.lanes = (double)A.nnz > 48.0 * std::max(A.n, 1) ? 16 : 1;
    if (T.lds) {
      for (int j = 0; j < 3; ++j) {
        T.o64[j] = o64 + j * A.n;
        T.o32[j] = o32 + j * A.n;
      }
      o64 += 3 * A.n;
      o32 += 3 * A.n;
    }
    if (l + 1 < nl) {
      T.ocoff = oco;
      oco += A.ncol + 1;
      if (!H.coff_dev[l].p) {
        H.coff_dev[l].resize(A.ncol + 1);
        copy_h2d(H.coff_dev[l].p, A.coff.data(), A.ncol + 1, s);
      }
      T.coff = H.coff_dev[l].p;
    }
    T.rp = A.rp.p;
    T.ci = A.ci.p;
    T.av = A.av.p;
    T.d = A.d.p;
    T.dinv = A.dinv.p;
    T.av32 = A.av32.p;
    T.d32 = A.d32.p;
    T.dinv32 = A.dinv32.p;
    T.agg = V.T.agg.p;
    T.moff = V.T.moff.p;
    T.mem = V.T.mem.p;
    T.pval = V.T.pval.p;
    T.pval32 = V.T.pval32.p;
    T.x = V.x.p;
    T.b = V.b.p;
    T.r = V.r.p;
    T.x32 = V.x32.p;
    T.b32 = V.b32.p;
    T.r32 = V.r32.p;
  }
  D.ncoff = oco;
  D.oacc64 = o64;
  D.oacc32 = (o32 + 1) / 2;
  const bool lds_L = H.cm <= 64;
  D.oL64 = lds_L ? D.oacc64 + H.cn : -1;
  D.oL32 = lds_L ? D.oacc32 + H.cn : -1;
  return true;
}

static std::unique_ptr<Hierarchy> assemble_hierarchy(pcamg_ctx* c, std::unique_ptr<Hierarchy> H,
                                                     std::vector<NatLevel>& nat, bool laplacian_op);

std::unique_ptr<Hierarchy> build_hierarchy(pcamg_ctx* c, const double* e_nat) {
  hipStream_t s = c->s;
  const pcamg_params& P = c->P;
  const int32_t n = c->n;
  auto H = std::make_unique<Hierarchy>();
  // Step 2: the A^2 pattern depends on the graph only -- built once per context
  if (!c->a2_ready) {
    c->rp2.resize(n + 1);
    int64_t nnz2 = a2_count(n, c->rp.p, c->ci.p, P.a2_hub_cap, c->rp2.p, s);
    c->ci2.resize(std::max<int64_t>(nnz2, 1));
    a2_fill(n, c->rp.p, c->ci.p, P.a2_hub_cap, c->rp2.p, c->ci2.p, s);
    c->nnz2 = (int32_t)nnz2;
    c->m2 = (int32_t)(nnz2 / 2);
    c->a2_ready = true;
  }
  std::vector<NatLevel> nat(1);
  DVec<double> gv0(std::max(c->nnz2, 1)), gkey0(std::max(c->nnz2, 1));
  DVec<int32_t> nb0(2 * (size_t)n);
  {
    // reweighting, sort (Alg. 1 Step 3) and path cover (Alg. 1) on the finest level
    const int32_t m2 = std::max(c->m2, 1);
    DVec<int32_t> eu(m2), ev(m2);
    DVec<uint64_t> ekey(m2), ksorted(m2);
    const int32_t m = a2_keys(n, c->rp2.p, c->ci2.p, e_nat, gkey0.p, gv0.p, eu.p, ev.p, ekey.p, s);
    DVec<uint32_t> idx(m2), order(m2);
    iota_i32((int32_t*)idx.p, m, s);
    radix_sort_u64_u32(ekey.p, idx.p, ksorted.p, order.p, m, s);
    DVec<int32_t> su(m2), sv(m2);
    sorted_endpoints(m, order.p, eu.p, ev.p, su.p, sv.p, s);
    H->cover_rounds = path_cover(n, m, su.p, sv.p, nb0.p, s);
  }
  {
    NatLevel& L0 = nat[0];
    L0.n = n;
    L0.nnz = c->nnz;
    L0.rp = c->rp.p;
    L0.ci = c->ci.p;
    L0.av = c->av.p;
    L0.d = c->d.p;
    L0.dinv = c->dinv.p;
    L0.colour = c->colour.p;
    L0.ncol = c->ncol;
    L0.grp = c->rp2.p;
    L0.gci = c->ci2.p;
    L0.gv = gv0.p;
    L0.gkey = gkey0.p;
    L0.nnz_g = c->nnz2;
    L0.nb = nb0.p;
  }
  // level loop (Alg. 4, Steps 5-9)
  for (int l = 0;; ++l) {
    NatLevel& L = nat[l];
    if (L.n <= P.coarse_max || l + 1 >= P.max_levels) break;
    L.pid.resize(L.n);
    L.pos.resize(L.n);
    L.plen.resize(L.n);
    orient_paths(L.n, L.nb, L.pid.p, L.pos.p, L.plen.p, s);
    L.agg.resize(L.n);
    L.moff.resize(L.n + 1);
    L.mem.resize(L.n);
    const int32_t nc = aggregate_level(L.n, L.grp, L.gci, L.gv, L.gkey, L.nb, L.pid.p, L.pos.p, L.plen.p, L.agg.p,
                                       L.moff.p, L.mem.p, L.st, s, P.case3);
    // stall (n_c > 0.9 n): this level becomes the coarsest if the dense solve
    // can take it; a larger level keeps coarsening while it still shrinks
    if (nc > 0.9 * L.n && (L.n <= LDLT_MAX || nc >= L.n)) {
      L.agg.release();
      L.moff.release();
      L.mem.release();
      break;
    }
    L.nc = nc;
    if (l == 0 && P.p1_mode == PCAMG_P1_SMOOTH) {
      L.pval.resize(L.n);
      L.st.p1_fallback = smooth_pval(L.n, e_nat, nc, L.moff.p, L.mem.p, L.pval.p, s);
    }
    NatLevel C;
    C.n = nc;
    C.o_rp.resize(nc + 1);
    GalerkinCache gc;
    int64_t nnzc = galerkin_count(L.n, L.rp, L.ci, nc, L.moff.p, L.mem.p, L.agg.p, C.o_rp.p, false, s, &gc);
    C.nnz = (int32_t)nnzc;
    C.o_ci.resize(std::max<int64_t>(nnzc, 1));
    C.o_av.resize(std::max<int64_t>(nnzc, 1));
    C.o_d.resize(nc);
    C.o_dinv.resize(nc);
    galerkin_fill(L.n, L.rp, L.ci, L.av, L.d, nc, L.moff.p, L.mem.p, L.agg.p, L.pval.p, C.o_rp.p, C.o_ci.p,
                  C.o_av.p, C.o_d.p, C.o_dinv.p, false, s, &gc);
    C.o_grp.resize(nc + 1);
    int64_t nnzg = galerkin_count(L.n, L.grp, L.gci, nc, L.moff.p, L.mem.p, L.agg.p, C.o_grp.p, true, s, &gc);
    C.nnz_g = (int32_t)nnzg;
    C.o_gci.resize(std::max<int64_t>(nnzg, 1));
    C.o_gv.resize(std::max<int64_t>(nnzg, 1));
    galerkin_fill(L.n, L.grp, L.gci, L.gv, nullptr, nc, L.moff.p, L.mem.p, L.agg.p, nullptr, C.o_grp.p, C.o_gci.p,
                  C.o_gv.p, nullptr, nullptr, true, s, &gc);
    C.o_nb.resize(2 * (size_t)nc);
    shorten_paths(L.n, L.nb, L.pid.p, L.pos.p, nc, L.agg.p, C.o_nb.p, s);
    C.o_colour.resize(nc);
    C.ncol = colour_level(nc, C.o_rp.p, C.o_ci.p, P.colour_seed, l + 1, C.o_colour.p, s);
    C.rp = C.o_rp.p;
    C.ci = C.o_ci.p;
    C.av = C.o_av.p;
    C.d = C.o_d.p;
    C.dinv = C.o_dinv.p;
    C.grp = C.o_grp.p;
    C.gci = C.o_gci.p;
    C.gv = C.o_gv.p;
    C.nb = C.o_nb.p;
    C.colour = C.o_colour.p;
    nat.push_back(std::move(C));
  }
  // the coarsest operator is a Laplacian when every prolongation is boolean
  // (boolean mode, or no coarsening at all)
  return assemble_hierarchy(c, std::move(H), nat, P.p1_mode == PCAMG_P1_CONST || nat.size() == 1);
}

// UA-AMG hierarchy by MWM aggregation on every level (the MWM_setup of
// Alg. 5/6 Step 2, Sec. 2.1): boolean prolongations and Galerkin products.
std::unique_ptr<Hierarchy> build_hierarchy_mwm(pcamg_ctx* c) {
  hipStream_t s = c->s;
  const pcamg_params& P = c->P;
  auto H = std::make_unique<Hierarchy>();
  std::vector<NatLevel> nat(1);
  {
    NatLevel& L0 = nat[0];
    L0.n = c->n;
    L0.nnz = c->nnz;
    L0.rp = c->rp.p;
    L0.ci = c->ci.p;
    L0.av = c->av.p;
    L0.d = c->d.p;
    L0.dinv = c->dinv.p;
    L0.colour = c->colour.p;
    L0.ncol = c->ncol;
  }
  for (int l = 0;; ++l) {
    NatLevel& L = nat[l];
    if (L.n <= P.coarse_max || l + 1 >= P.max_levels) break;
    L.agg.resize(L.n);
    L.moff.resize(L.n + 1);
    L.mem.resize(L.n);
    const int32_t nc = mwm_aggregate_level(L.n, L.rp, L.ci, L.av, L.agg.p, L.moff.p, L.mem.p, L.st, s);
    if (nc > 0.9 * L.n && (L.n <= LDLT_MAX || nc >= L.n)) {
      L.agg.release();
      L.moff.release();
      L.mem.release();
      break;
    }
    L.nc = nc;
    NatLevel C;
    C.n = nc;
    C.o_rp.resize(nc + 1);
    GalerkinCache gc;
    int64_t nnzc = galerkin_count(L.n, L.rp, L.ci, nc, L.moff.p, L.mem.p, L.agg.p, C.o_rp.p, false, s, &gc);
    C.nnz = (int32_t)nnzc;
    C.o_ci.resize(std::max<int64_t>(nnzc, 1));
    C.o_av.resize(std::max<int64_t>(nnzc, 1));
    C.o_d.resize(nc);
    C.o_dinv.resize(nc);
    galerkin_fill(L.n, L.rp, L.ci, L.av, L.d, nc, L.moff.p, L.mem.p, L.agg.p, nullptr, C.o_rp.p, C.o_ci.p,
                  C.o_av.p, C.o_d.p, C.o_dinv.p, false, s, &gc);
    C.o_colour.resize(nc);
    C.ncol = colour_level(nc, C.o_rp.p, C.o_ci.p, P.colour_seed, l + 1, C.o_colour.p, s);
    C.rp = C.o_rp.p;
    C.ci = C.o_ci.p;
    C.av = C.o_av.p;
    C.d = C.o_d.p;
    C.dinv = C.o_dinv.p;
    C.colour = C.o_colour.p;
    nat.push_back(std::move(C));
  }
  return assemble_hierarchy(c, std::move(H), nat, true);
}

// Solve layout, transfers, coarsest factor, statistics and cycle descriptors
// of a hierarchy whose levels were built in natural numbering.
static std::unique_ptr<Hierarchy> assemble_hierarchy(pcamg_ctx* c, std::unique_ptr<Hierarchy> H,
                                                     std::vector<NatLevel>& nat, bool laplacian_op) {
  hipStream_t s = c->s;
  const pcamg_params& P = c->P;
  const int nl = (int)nat.size();
  NatLevel& Lc = nat.back();
  require(Lc.n <= 4096, PCAMG_EUNSUPPORTED, "coarsest level larger than 4096 vertices");

  // solve layout
  H->lv.resize(nl);
  for (int l = 0; l < nl; ++l) {
    NatLevel& L = nat[l];
    Level& V = H->lv[l];
    if (l == 0) V.A = c->M0;
    else if (l + 1 < nl)
      V.A = make_level_matrix(L.n, L.nnz, L.rp, L.ci, L.av, L.d, L.dinv, L.colour, L.ncol, P.row_lanes,
                              P.long_row_min, P.block_sweep_min_colours, s);
    else
      V.A = make_level_matrix(L.n, L.nnz, L.rp, L.ci, L.av, L.d, L.dinv, nullptr, 1, P.row_lanes, 0, 0, s);
    V.x.resize(L.n);
    V.b.resize(L.n);
    V.r.resize(L.n);
    V.x32.resize(L.n);
    V.b32.resize(L.n);
    V.r32.resize(L.n);
  }
  for (int l = 0; l + 1 < nl; ++l) {
    NatLevel& L = nat[l];
    Level& V = H->lv[l];
    const LevelMatrix& Af = *V.A;
    const LevelMatrix& Ac = *H->lv[l + 1].A;
    const bool coarsest_next = l + 2 == nl;
    V.T.nc = L.nc;
    V.T.agg.resize(L.n);
    V.T.moff.resize(L.nc + 1);
    V.T.mem.resize(L.n);
    if (L.pval.p) {
      V.T.pval.resize(L.n);
      V.T.pval32.resize(L.n);
    }
    permute_transfer(L.n, Af.perm.p, Af.iperm.p, L.nc, coarsest_next ? nullptr : Ac.perm.p,
                     coarsest_next ? nullptr : Ac.iperm.p, L.agg.p, L.pval.p, L.moff.p, L.mem.p, V.T.agg.p,
                     V.T.pval.p, V.T.pval32.p, V.T.moff.p, V.T.mem.p, s);
  }
  // coarsest level: dense LDL^T; grounded iff the operator is a Laplacian
  {
    bool grounded = P.coarse_solve == PCAMG_COARSE_GROUNDED ? true
                    : P.coarse_solve == PCAMG_COARSE_FULL   ? false
                                                            : laplacian_op;
    const int32_t cn = Lc.n;
    DVec<double> Ad((size_t)cn * cn);
    dense_from_csr(cn, Lc.rp, Lc.ci, Lc.av, Lc.d, Ad.p, s);
    H->cn = cn;
    H->cL.resize((size_t)cn * cn);
    H->cD.resize(cn);
    bool ok = false;
    if (!grounded) {
      H->cm = cn;
      ok = ldlt_factor(cn, cn, Ad.p, H->cL.p, H->cD.p, s);
      if (!ok) H->fallback = true;
    }
    if (!ok) {
      grounded = true;
      H->cm = cn - 1;
      ok = ldlt_factor(cn, cn - 1, Ad.p, H->cL.p, H->cD.p, s);
      require(ok, PCAMG_EBREAKDOWN, "coarsest level: non-positive pivot in grounded LDL^T");
    }
    H->grounded = grounded;
  }
  // statistics
  double tot = 0.0;
  for (int l = 0; l < nl; ++l) tot += (double)nat[l].nnz + nat[l].n;
  H->op_complexity = tot / ((double)nat[0].nnz + nat[0].n);
  for (int l = 0; l < nl; ++l) {
    NatLevel& L = nat[l];
    int64_t npaths = 0, npv = 0;
    if (L.pid.p) {
      auto pid = to_host(L.pid.p, L.n, s);
      for (int32_t v = 0; v < L.n; ++v) {
        npaths += pid[v] == v;
        npv += pid[v] >= 0;
      }
    }
    H->lv[l].info = {L.n, L.nnz, L.ncol, L.nc, L.nnz_g, npaths, L.st.n_unagg, L.st.case1, L.st.case2,
                     L.st.case3, L.st.middle, L.st.singleton, L.st.p1_fallback, H->grounded ? 1 : 0,
                     H->fallback ? 1 : 0, npv};
  }
  H->st0 = nat[0].st;
  // tail: the levels of at most tail_max_n vertices and the coarsest run in one
  // workgroup launch (tail_desc).  W-cycles apply the two sub-cycles of the
  // first level of at most dense_max_n vertices as one dense operator.
  {
    const int32_t tail_n = c->P.tail_max_n > 0 ? c->P.tail_max_n : 0;
    auto first_small = [&](int32_t limit) {
      int ts = nl - 1;
      int64_t nco = 0;
      while (limit > 0 && ts > 0 && H->lv[ts - 1].A->n <= limit && nl - (ts - 1) <= TAIL_MAX_LEVELS &&
             nco + H->lv[ts - 1].A->ncol + 1 <= TAIL_COFF_MAX) {
        --ts;
        nco += H->lv[ts].A->ncol + 1;
      }
      return ts;
    };
    H->coff_dev.resize(nl);
    TailDesc D;
    int ts = first_small(tail_n);
    H->tail_start = (tail_n > 0 && !(ts == 0 && nl == 1) && make_tail_desc(*H, ts, D, s)) ? ts : -1;
    if (H->tail_start >= 0) {
      H->tail_desc.resize(1);
      copy_h2d(H->tail_desc.p, &D, 1, s);
      sync(s);  // D is a host temporary
    }
    // the dense operators start at the first level of at most their size
    // limit (no tail descriptor limits), not below the tail's first level:
    // the dense product is applied from a level launched step by step
    auto first_at_most = [&](int32_t limit) {
      int l = nl - 1;
      while (l > 0 && H->lv[l - 1].A->n <= limit) --l;
      return l;
    };
    int ds = first_at_most(std::max<int32_t>(c->P.dense_max_n, 1));
    if (H->tail_start >= 0) ds = std::min(ds, H->tail_start);
    if (ds >= 1 && nl - ds >= 2) H->dense_start = ds;
    // V-cycles: the same from the first level of at most v_dense_max_n
    if (c->P.v_dense_max_n > 0) {
      int dv = first_at_most(c->P.v_dense_max_n);
      // near-dense levels of up to twice the limit join (more than one colour
      // per V_DENSE_ROWS_PER_COLOUR rows: a launch per colour of a few hub
      // rows each in every sweep, while their dense build is cheap)
      while (dv > 1 && H->lv[dv - 1].A->n <= 2 * (int64_t)c->P.v_dense_max_n &&
             (int64_t)H->lv[dv - 1].A->ncol * V_DENSE_ROWS_PER_COLOUR > H->lv[dv - 1].A->n)
        --dv;
      if (H->tail_start >= 0) dv = std::min(dv, H->tail_start);
      if (dv >= 1 && nl - dv >= 2) H->dense_v_start = dv;
    }
    // a graph of at most top_dense_max_n vertices: each cycle type as one
    // dense operator of the whole cycle (instead of the single-workgroup
    // tail, whose colour passes run one after another in one workgroup)
    const int32_t n0 = H->lv[0].A->n;
    if (nl >= 2 && n0 <= std::min(c->P.top_dense_max_n, TOP_DENSE_MAX_N) && dense_bottom_up_fits(*H, 0)) {
      if (c->P.v_dense_max_n > 0 && n0 <= c->P.v_dense_max_n) H->dense_v_start = 0;
      if (c->P.w_dense != 0 && n0 <= c->P.dense_max_n) H->dense_start = 0;
    }
  }
  if (P.keep_setup) {
    H->setup.resize(nl);
    for (int l = 0; l < nl; ++l) {
      NatLevel& L = nat[l];
      SetupLevel& S = H->setup[l];
      S.n = L.n;
      S.nnz = L.nnz;
      S.ncol = L.ncol;
      S.nnz_g = L.nnz_g;
      auto cp_i = [&](DVec<int32_t>& dst, const int32_t* src, size_t cnt) {
        if (!src) return;
        dst.resize(std::max<size_t>(cnt, 1));
        copy_d2d(dst.p, src, cnt, s);
      };
      auto cp_d = [&](DVec<double>& dst, const double* src, size_t cnt) {
        if (!src) return;
        dst.resize(std::max<size_t>(cnt, 1));
        copy_d2d(dst.p, src, cnt, s);
      };
      cp_i(S.rp, L.rp, L.n + 1);
      cp_i(S.ci, L.ci, L.nnz);
      cp_i(S.colour, L.colour, L.n);
      cp_i(S.grp, L.grp, L.n + 1);
      cp_i(S.gci, L.gci, L.nnz_g);
      cp_i(S.nb, L.nb, 2 * (size_t)L.n);
      cp_i(S.path_id, L.pid.p, L.n);
      cp_i(S.pos, L.pos.p, L.n);
      cp_i(S.agg, L.agg.p, L.n);
      cp_d(S.av, L.av, L.nnz);
      cp_d(S.d, L.d, L.n);
      cp_d(S.dinv, L.dinv, L.n);
      cp_d(S.gv, L.gv, L.nnz_g);
      if (l == 0) cp_d(S.gkey, L.gkey, L.nnz_g);
      cp_d(S.pval, L.pval.p, L.n);
    }
  }
  sync(s);
  return H;
}

// ---------------------------------------------------------------------------
// Cycles (Alg. 5 V_cycle, Alg. 2 W_cycle), solve layout.
// ---------------------------------------------------------------------------
// The whole cycle of level 0 as one dense operator (small graphs; built when
// the cycle of this type is first run).  A cycle is an affine map of its
// start vector whose fixed points are the exact solutions, so from any x it
// gives x + C (b - A x), C being its map of b from x = 0.
namespace {
template <typename T>
bool top_dense(const Hierarchy& H, int gamma, const T* cv, const T* cw) {
  return gamma == 1 ? H.dense_v_start == 0 && cv != nullptr : gamma == 2 && H.dense_start == 0 && cw != nullptr;
}
}  // namespace

void cycle64(pcamg_ctx* c, Hierarchy& H, int l, const double* b, double* x, int gamma, int skip) {
  hipStream_t s = c->s;
  const int nl = (int)H.lv.size();
  if (l == 0 && top_dense(H, gamma, H.CV64.p, H.C64.p)) {  // a small graph's whole cycle: x += C (b - A x)
    Level& L = H.lv[0];
    level_residual(*L.A, b, x, L.r.p, s);
    dense_apply<double>(L.A->n, gamma == 2 ? H.C64.p : H.CV64.p, L.r.p, gamma == 2 ? H.dpart64.p : H.dvpart64.p, x,
                        s, true);
    return;
  }
  if (l == H.tail_start && !(l == 0 && nl == 1)) {
    tail_cycle64(H, b, x, gamma, s);
    return;
  }
  if (l + 1 == nl) {
    if (l == 0) {  // no coarsening: the dense factor is in natural order, level 0 is colour-permuted
      Level& L = H.lv[0];
      scatter_f64(b, L.A->perm.p, L.b.p, H.cn, s);
      ldlt_solve(H.cn, H.cm, H.grounded, H.cL.p, H.cD.p, L.b.p, L.x.p, s);
      gather_f64(L.x.p, L.A->perm.p, x, H.cn, s);
      return;
    }
    ldlt_solve(H.cn, H.cm, H.grounded, H.cL.p, H.cD.p, b, x, s);
    return;
  }
  Level& L = H.lv[l];
  const LevelMatrix& A = *L.A;
  smooth_sweep(A, true, skip, b, x, s);
  Level& N = H.lv[l + 1];
  const LevelMatrix& AN = *N.A;
  const int calls = (gamma > 1 && l + 2 < nl) ? gamma : 1;
  const bool dense_v = gamma == 1 && l + 1 == H.dense_v_start && H.CV64.p;
  const bool dense = (calls == 2 && l + 1 == H.dense_start && H.C64.p) || dense_v;
  // the child's x: written by the dense product or the coarsest solve, zero
  // for the tail, else zero with its first colour pass done here
  const bool launched_child = !dense && l + 2 < nl && l + 1 != H.tail_start;
  const int mode = dense || l + 2 == nl ? 0 : launched_child ? 2 : 1;
  level_residual(A, b, x, L.r.p, s);
  restrict_members<double>(L.T.nc, L.T.moff.p, L.T.mem.p, L.T.pval.p, L.r.p, N.b.p, s, N.x.p, AN.dinv.p,
                        AN.coff.size() > 1 ? AN.coff[1] : 0, mode);
  if (dense_v) {  // the V-cycle below at once
    dense_apply<double>(AN.n, H.CV64.p, N.b.p, H.dvpart64.p, N.x.p, s);
  } else if (dense) {  // both sub-cycles below at once
    dense_apply<double>(AN.n, H.C64.p, N.b.p, H.dpart64.p, N.x.p, s);
  } else {
    for (int q = 0; q < calls; ++q) cycle64(c, H, l + 1, N.b.p, N.x.p, gamma, q == 0 && mode == 2 ? 1 : 0);
  }
  prolong_add<double>(A.n, L.T.agg.p, L.T.pval.p, N.x.p, x, s);
  smooth_sweep(A, false, 0, b, x, s);
}

void cycle32(pcamg_ctx* c, Hierarchy& H, int l, const float* b, float* x, int gamma, int skip) {
  hipStream_t s = c->s;
  const int nl = (int)H.lv.size();
  if (l == 0 && top_dense(H, gamma, H.CV32.p, H.C32.p)) {  // a small graph's whole cycle: x += C (b - A x)
    Level& L = H.lv[0];
    level_residual(*L.A, b, x, L.r32.p, s);
    dense_apply<float>(L.A->n, gamma == 2 ? H.C32.p : H.CV32.p, L.r32.p, gamma == 2 ? H.dpart32.p : H.dvpart32.p,
                       x, s, true);
    return;
  }
  if (l == H.tail_start && !(l == 0 && nl == 1)) {
    tail_cycle32(H, b, x, gamma, s);
    return;
  }
  if (l + 1 == nl) {
    if (l == 0) {  // no coarsening: natural-order factor, colour-permuted vectors
      Level& L = H.lv[0];
      scatter_f32(b, L.A->perm.p, L.b32.p, H.cn, s);
      ldlt_solve32(H.cn, H.cm, H.grounded, H.cL.p, H.cD.p, L.b32.p, L.x32.p, s);
      gather_f32(L.x32.p, L.A->perm.p, x, H.cn, s);
      return;
    }
    ldlt_solve32(H.cn, H.cm, H.grounded, H.cL.p, H.cD.p, b, x, s);
    return;
  }
  Level& L = H.lv[l];
  const LevelMatrix& A = *L.A;
  smooth_sweep(A, true, skip, b, x, s);
  Level& N = H.lv[l + 1];
  const LevelMatrix& AN = *N.A;
  const int calls = (gamma > 1 && l + 2 < nl) ? gamma : 1;
  const bool dense_v = gamma == 1 && l + 1 == H.dense_v_start && H.CV32.p;
  const bool dense = (calls == 2 && l + 1 == H.dense_start && H.C32.p) || dense_v;
  // the child's x: written by the dense product or the coarsest solve, zero
  // for the tail, else zero with its first colour pass done here
  const bool launched_child = !dense && l + 2 < nl && l + 1 != H.tail_start;
  const int mode = dense || l + 2 == nl ? 0 : launched_child ? 2 : 1;
  level_residual(A, b, x, L.r32.p, s);
  restrict_members<float>(L.T.nc, L.T.moff.p, L.T.mem.p, L.T.pval32.p, L.r32.p, N.b32.p, s, N.x32.p, AN.dinv32.p,
                        AN.coff.size() > 1 ? AN.coff[1] : 0, mode);
  if (dense_v) {  // the V-cycle below at once
    dense_apply<float>(AN.n, H.CV32.p, N.b32.p, H.dvpart32.p, N.x32.p, s);
  } else if (dense) {  // both sub-cycles below at once
    dense_apply<float>(AN.n, H.C32.p, N.b32.p, H.dpart32.p, N.x32.p, s);
  } else {
    for (int q = 0; q < calls; ++q) cycle32(c, H, l + 1, N.b32.p, N.x32.p, gamma, q == 0 && mode == 2 ? 1 : 0);
  }
  prolong_add<float>(A.n, L.T.agg.p, L.T.pval32.p, N.x32.p, x, s);
  smooth_sweep(A, false, 0, b, x, s);
}

// ---------------------------------------------------------------------------
// Whole cycles from captured graphs.  A cycle's launch sequence is fixed for a
// hierarchy, so it is captured once (per precision and cycle type) on fixed
// input/output buffers and replayed; inputs are copied in and results out.
// ---------------------------------------------------------------------------
namespace {
// Records the launches of body() into a graph.  Capture is not allowed on the
// legacy null stream, so the launches are redirected to the context's private
// capture stream (nothing executes during capture); the graph is then replayed
// on the caller's stream.
template <typename F>
hipGraphExec_t capture(pcamg_ctx* c, F&& body) {
  if (!c->capture_stream) PCAMG_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  hipStream_t user = c->s;
  hipGraph_t g = nullptr;
  PCAMG_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  c->s = c->capture_stream;
  try {
    body();
  } catch (...) {
    c->s = user;
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(c->capture_stream, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    throw;
  }
  c->s = user;
  PCAMG_HIP(hipStreamEndCapture(c->capture_stream, &g));
  hipGraphExec_t e = nullptr;
  hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  PCAMG_HIP(err);
  return e;
}
}  // namespace

// The dense operators of the two W sub-cycles of level dense_start
// (gamma = 2) and of the V-cycle of level dense_v_start (gamma = 1), built
// once per hierarchy and precision on first use.
template <typename T>
struct DenseOf;
template <>
struct DenseOf<double> {
  static DVec<double>& C(Hierarchy& H, int gamma) { return gamma == 2 ? H.C64 : H.CV64; }
  static DVec<double>& part(Hierarchy& H, int gamma) { return gamma == 2 ? H.dpart64 : H.dvpart64; }
};
template <>
struct DenseOf<float> {
  static DVec<float>& C(Hierarchy& H, int gamma) { return gamma == 2 ? H.C32 : H.CV32; }
  static DVec<float>& part(Hierarchy& H, int gamma) { return gamma == 2 ? H.dpart32 : H.dvpart32; }
};

template <typename T>
void ensure_dense(pcamg_ctx* c, Hierarchy& H, int gamma) {
  const int nl = (int)H.lv.size();
  const int d = gamma == 2 ? H.dense_start : H.dense_v_start;
  const bool on = gamma == 2 ? c->P.w_dense != 0 : c->P.v_dense_max_n > 0;
  // without a dense operator the cycle recurses (levels too large for the build)
  if (!on || d < 0 || nl - d < 2 || !dense_bottom_up_fits(H, d)) return;
  DVec<T>& C = DenseOf<T>::C(H, gamma);
  if (C.p) return;
  const int32_t nd = H.lv[d].A->n;
  C.resize((size_t)nd * nd);
  DenseOf<T>::part(H, gamma).resize((size_t)dense_chunks(nd) * nd);
  // level 0: one call of the whole cycle; below: the calls of the level above
  dense_bottom_up<T>(H, d, gamma, C.p, c->s, d == 0 ? 1 : gamma);
}

void run_cycle64(pcamg_ctx* c, Hierarchy& H, const double* b, double* x, int gamma) {
  hipStream_t s = c->s;
  ensure_dense<double>(c, H, gamma > 1 ? 2 : 1);
  const int32_t n = c->n;
  if (!c->P.use_graphs) {
    cycle64(c, H, 0, b, x, gamma);
    return;
  }
  if (!H.gb.p) {
    H.gb.resize(n);
    H.gx.resize(n);
  }
  hipGraphExec_t& g = gamma > 1 ? H.g64w : H.g64v;
  if (!g) g = capture(c, [&] { cycle64(c, H, 0, H.gb.p, H.gx.p, gamma); });
  copy_d2d(H.gb.p, b, n, s);
  copy_d2d(H.gx.p, x, n, s);
  PCAMG_HIP(hipGraphLaunch(g, s));
  copy_d2d(x, H.gx.p, n, s);
}

void run_cycle32(pcamg_ctx* c, Hierarchy& H, const float* b, float* x, int gamma) {
  hipStream_t s = c->s;
  ensure_dense<float>(c, H, gamma > 1 ? 2 : 1);
  const int32_t n = c->n;
  if (!c->P.use_graphs) {
    cycle32(c, H, 0, b, x, gamma);
    return;
  }
  if (!H.gb32.p) {
    H.gb32.resize(n);
    H.gx32.resize(n);
  }
  hipGraphExec_t& g = gamma > 1 ? H.g32w : H.g32v;
  if (!g) g = capture(c, [&] { cycle32(c, H, 0, H.gb32.p, H.gx32.p, gamma); });
  copy_d2d(H.gb32.p, b, n, s);
  copy_d2d(H.gx32.p, x, n, s);
  PCAMG_HIP(hipGraphLaunch(g, s));
  copy_d2d(x, H.gx32.p, n, s);
}

// ---------------------------------------------------------------------------
// Smooth errors
// ---------------------------------------------------------------------------
namespace {
void relax_perm(pcamg_ctx* c, double* e_perm, const double* zero, int sweeps) {
  const LevelMatrix& A = *c->M0;
  for (int q = 0; q < sweeps; ++q) {
    for (int k = 0; k < A.ncol; ++k)
      smooth_colour(A, k, zero, e_perm, c->s, true);
    for (int k = A.ncol - 1; k >= 0; --k)
      smooth_colour(A, k, zero, e_perm, c->s, true);
  }
}
}  // namespace

void relax_homogeneous(pcamg_ctx* c, double* e_nat, int sweeps) {
  const int32_t n = c->n;
  DVec<double> ep(n), zero(n);
  fill_f64(zero.p, 0.0, n, c->s);
  gather_f64(e_nat, c->M0->perm.p, ep.p, n, c->s);
  relax_perm(c, ep.p, zero.p, sweeps);
  scatter_f64(ep.p, c->M0->perm.p, e_nat, n, c->s);
}

void initial_error(pcamg_ctx* c, int32_t r, double* e_nat, int32_t sweeps) {
  xi_fill(c->P.seed, r, nullptr, e_nat, c->n, c->s);
  relax_homogeneous(c, e_nat, sweeps < 0 ? c->P.relax_sweeps : sweeps);
}

// ---------------------------------------------------------------------------
// Error approximation (Alg. 2), permuted vectors: PCG on A e = r from e = 0;
// preconditioner = W-cycle of the latest hierarchy while Re <= numW, else the
// symmetric composite B_1 .. B_Re, B_Re .. B_1 of V-cycles; preconditioned
// vectors and the result made orthogonal to 1.
// ---------------------------------------------------------------------------
void approx_error(pcamg_ctx* c, int Re, const double* r, double* e, int* wcycles, int* vcycles, int* vcycles32) {
  hipStream_t s = c->s;
  const int32_t n = c->n;
  const pcamg_params& P = c->P;
  const LevelMatrix& A = *c->M0;
  const bool wcyc = Re <= P.numW;
  const int steps = wcyc ? P.iterW : P.iterV;
  DVec<double> rr(n), z(n), p(n), q(n), scal(2);
  const bool f32 = P.cycle_prec == PCAMG_PREC_F32;
  DVec<float> v32(f32 ? n : 0), z32(f32 ? n : 0);
  auto dot = [&](const double* a, const double* b) {
    dot_f64(a, b, n, scal.p, s);
    return read_scalar(scal.p, s);
  };
  // FP32 setting: the preconditioning cycles run in FP32, input rounded once,
  // result widened once
  auto prec = [&](const double* v, double* zz) {
    fill_f64(zz, 0.0, n, s);
    if (f32) {
      cast_f64_f32(v, v32.p, n, s);
      fill_f32(z32.p, 0.0f, n, s);
      if (wcyc) {
        run_cycle32(c, *c->hist[Re - 1], v32.p, z32.p, 2);
        if (wcycles) *wcycles += 1;
      } else {
        for (int j = 0; j < Re; ++j) run_cycle32(c, *c->hist[j], v32.p, z32.p, 1);
        for (int j = Re - 1; j >= 0; --j) run_cycle32(c, *c->hist[j], v32.p, z32.p, 1);
        if (vcycles32) *vcycles32 += 2 * Re;
      }
      cast_f32_f64(z32.p, zz, n, s);
    } else if (wcyc) {
      run_cycle64(c, *c->hist[Re - 1], v, zz, 2);
      if (wcycles) *wcycles += 1;
    } else {
      for (int j = 0; j < Re; ++j) run_cycle64(c, *c->hist[j], v, zz, 1);
      for (int j = Re - 1; j >= 0; --j) run_cycle64(c, *c->hist[j], v, zz, 1);
      if (vcycles) *vcycles += 2 * Re;
    }
    sum_f64(zz, n, scal.p + 1, s);
    sub_mean_f64(zz, scal.p + 1, n, s);
  };
  fill_f64(e, 0.0, n, s);
  copy_d2d(rr.p, r, n, s);
  prec(rr.p, z.p);
  copy_d2d(p.p, z.p, n, s);
  double rz = dot(rr.p, z.p);
  for (int t = 0; t < steps; ++t) {
    level_residual(A, nullptr, p.p, q.p, s);
    const double pq = dot(p.p, q.p);
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    axpy_f64(alpha, p.p, e, n, s);
    if (t + 1 == steps) break;
    axpy_f64(-alpha, q.p, rr.p, n, s);
    prec(rr.p, z.p);
    const double rz2 = dot(rr.p, z.p);
    const double beta = rz2 / rz;
    DVec<double> bd(1);
    copy_h2d(bd.p, &beta, 1, s);
    xpby_dev_f64(z.p, bd.p, p.p, n, s);
    sync(s);  // `beta` is a host temporary
    rz = rz2;
  }
  sum_f64(e, n, scal.p + 1, s);
  sub_mean_f64(e, scal.p + 1, n, s);
}

// ---------------------------------------------------------------------------
// Adaptive solve (Alg. 5): standalone V-cycles or FCG(1) with a V-cycle
// preconditioner (FP64 or FP32), in the solve layout of the finest level.
// ---------------------------------------------------------------------------
void solve(pcamg_ctx* c, double* x_nat, pcamg_stats* st) {
  hipStream_t s = c->s;
  const pcamg_params& P = c->P;
  const int32_t n = c->n;
  const LevelMatrix& A = *c->M0;
  require(c->have_rhs, PCAMG_EINVAL, "no right-hand side");
  require(!c->hist.empty(), PCAMG_EINVAL, "no hierarchy");
  Timer total(s);
  double t_rebuild = 0.0, t_approx = 0.0, t_build = 0.0;
  int vc64 = 0, vc32 = 0, wc = 0;
  DVec<double> b(n), x(n), r(n), scal(4);
  gather_f64(c->rhs.p, A.perm.p, b.p, n, s);
  gather_f64(x_nat, A.perm.p, x.p, n, s);
  auto dot = [&](const double* a, const double* bb) {
    dot_f64(a, bb, n, scal.p, s);
    return read_scalar(scal.p, s);
  };
  auto remove_mean = [&](double* v) {
    sum_f64(v, n, scal.p + 1, s);
    sub_mean_f64(v, scal.p + 1, n, s);
  };
  auto res_of = [&](const double* xx, double* rr) { level_residual(A, b.p, xx, rr, s); };
  std::vector<double> hist{1.0};
  std::vector<double> conv, conv_all;
  int rebuilds = 0, k = 0, status = PCAMG_OK;
  double oc_sum = 0.0;
  for (auto& h : c->hist) oc_sum += h->op_complexity;
  int nh = (int)c->hist.size();
  res_of(x.p, r.p);
  const double nr0 = std::sqrt(dot(r.p, r.p));
  double nr = nr0, nr_prev = nr0;
  auto triggered = [&]() {
    if (rebuilds >= P.max_rebuilds) return false;
    if (P.rebuild_rule == 1) return conv.back() > P.theta;
    double mean = 0.0;
    for (double q : conv) mean = mean + q;
    mean = mean / (double)conv.size();
    return mean > P.theta;
  };
  // re-setup (Alg. 5, Steps 13-16); corr is the correction for x (0 for the relaxation source)
  int learned_builds = 0, fallback_builds = 0;
  bool last_learned = c->net != nullptr;  // the first hierarchy came from the network
  double first_convr = 0.0;               // first ConvR measured with the current hierarchy
  auto rebuild = [&](const double* res, double* corr) {
    Timer tr(s);
    first_convr = conv.empty() ? 0.0 : conv.front();
    const int Re = (int)c->hist.size();
    DVec<double> eb(n), enat(n), zero(n);
    if (P.rebuild_source == PCAMG_REBUILD_ERROR_APPROX) {
      int nw = 0, nv = 0, nv32 = 0;
      Timer ta(s);
      approx_error(c, Re, res, corr, &nw, &nv, &nv32);
      t_approx += ta.ms();
      wc += nw;
      vc64 += nv;
      vc32 += nv32;
      copy_d2d(eb.p, corr, n, s);
    } else if (P.rebuild_source == PCAMG_REBUILD_ITERATE) {
      // Alg. 6: the current iterate itself (its normalisation is a scaling,
      // which neither the key order nor the renormalised P_1 sees)
      copy_d2d(eb.p, x.p, n, s);
      fill_f64(corr, 0.0, n, s);
    } else {
      xi_fill(P.seed, Re, A.perm.p, eb.p, n, s);
      fill_f64(zero.p, 0.0, n, s);
      for (int q = 0; q < P.rebuild_vcycles; ++q) run_cycle64(c, *c->hist.back(), zero.p, eb.p, 1);
      vc64 += P.rebuild_vcycles;
      fill_f64(corr, 0.0, n, s);
    }
    fill_f64(zero.p, 0.0, n, s);
    DVec<double> src;
    if (P.keep_setup) {  // the build's source vector before any sweep, for inspection
      src.resize(n);
      scatter_f64(eb.p, A.perm.p, src.p, n, s);
    }
    // learned proposals: the network maps the source relaxed by first_sweeps
    // (default 2) to the build's smooth error; a learned hierarchy whose first
    // measured ConvR exceeded LEARNED_FALLBACK_CONVR hands the next build back
    // to the plain relaxation
    const bool use_net = c->net && P.rebuild_source != PCAMG_REBUILD_ITERATE &&
                         !(last_learned && first_convr > LEARNED_FALLBACK_CONVR);
    if (use_net) {
      relax_perm(c, eb.p, zero.p, P.first_sweeps >= 0 ? P.first_sweeps : 2);
      DVec<double> e2(n);
      scatter_f64(eb.p, A.perm.p, e2.p, n, s);
      const pcamg_graph g{n, c->nnz, c->rp.p, c->ci.p, c->w.p};
      net_forward_f64(c->net, &g, e2.p, enat.p, s);
      ++learned_builds;
    } else {
      if (P.rebuild_source != PCAMG_REBUILD_ITERATE) relax_perm(c, eb.p, zero.p, P.relax_sweeps);
      scatter_f64(eb.p, A.perm.p, enat.p, n, s);
      if (c->net) ++fallback_builds;
    }
    last_learned = use_net;
    Timer tb(s);
    c->hist.push_back(build_hierarchy(c, enat.p));
    if (src.p) c->hist.back()->source = std::move(src);
    t_build += tb.ms();
    oc_sum += c->hist.back()->op_complexity;
    ++nh;
    ++rebuilds;
    conv.clear();
    t_rebuild += tr.ms();
  };
  if (nr0 > 0.0) {
    if (P.outer == PCAMG_OUTER_VCYCLE) {
      DVec<double> corr(n);
      while (k < P.max_iter) {
        run_cycle64(c, *c->hist.back(), b.p, x.p, 1);
        ++vc64;
        remove_mean(x.p);
        res_of(x.p, r.p);
        nr = std::sqrt(dot(r.p, r.p));
        ++k;
        const double cr = nr / nr_prev;
        conv.push_back(cr);
        conv_all.push_back(cr);
        nr_prev = nr;
        hist.push_back(nr / nr0);
        if (!std::isfinite(nr)) { status = PCAMG_ENAN; break; }
        if (nr / nr0 <= P.tol) break;
        if (triggered()) {
          rebuild(r.p, corr.p);
          if (P.rebuild_source == PCAMG_REBUILD_ERROR_APPROX) {
            axpy_f64(1.0, corr.p, x.p, n, s);
            res_of(x.p, r.p);
            nr_prev = std::sqrt(dot(r.p, r.p));
          }
        }
      }
    } else {
      DVec<double> z(n), p(n), q(n), rn(n), zn(n), corr(n), x32buf(1);
      DVec<float> r32(n), z32(n);
      auto precond = [&](const double* rr, double* zz) {
        Hierarchy& H = *c->hist.back();
        if (P.cycle_prec == PCAMG_PREC_F32) {
          cast_f64_f32(rr, r32.p, n, s);
          fill_f32(z32.p, 0.0f, n, s);
          run_cycle32(c, H, r32.p, z32.p, 1);
          cast_f32_f64(z32.p, zz, n, s);
          ++vc32;
        } else {
          fill_f64(zz, 0.0, n, s);
          run_cycle64(c, H, rr, zz, 1);
          ++vc64;
        }
        remove_mean(zz);
      };
      precond(r.p, z.p);
      copy_d2d(p.p, z.p, n, s);
      double rz = dot(r.p, z.p);
      while (k < P.max_iter) {
        level_residual(A, nullptr, p.p, q.p, s);
        const double pq = dot(p.p, q.p);
        if (!(pq > 0.0)) { status = PCAMG_EBREAKDOWN; break; }
        const double alpha = rz / pq;
        axpy_f64(alpha, p.p, x.p, n, s);
        copy_d2d(rn.p, r.p, n, s);
        axpy_f64(-alpha, q.p, rn.p, n, s);
        nr = std::sqrt(dot(rn.p, rn.p));
        ++k;
        const double cr = nr / nr_prev;
        conv.push_back(cr);
        conv_all.push_back(cr);
        nr_prev = nr;
        hist.push_back(nr / nr0);
        if (!std::isfinite(nr)) { status = PCAMG_ENAN; break; }
        if (nr / nr0 <= P.tol) { copy_d2d(r.p, rn.p, n, s); break; }
        bool restart = false;
        if (triggered()) {
          rebuild(rn.p, corr.p);
          if (P.rebuild_source == PCAMG_REBUILD_ERROR_APPROX) {
            axpy_f64(1.0, corr.p, x.p, n, s);
            res_of(x.p, rn.p);
            nr_prev = std::sqrt(dot(rn.p, rn.p));
          }
          restart = true;
        }
        precond(rn.p, zn.p);
        if (restart) {
          copy_d2d(p.p, zn.p, n, s);
        } else {
          zsub_dot_f64(zn.p, rn.p, r.p, n, scal.p + 2, s);
          const double num = read_scalar(scal.p + 2, s);
          const double beta = num / rz;
          DVec<double> bd(1);
          copy_h2d(bd.p, &beta, 1, s);
          xpby_dev_f64(zn.p, bd.p, p.p, n, s);
          sync(s);
        }
        rz = dot(rn.p, zn.p);
        std::swap(r, rn);
        std::swap(z, zn);
      }
      remove_mean(x.p);
    }
  }
  if (status == PCAMG_OK && nr0 > 0.0 && nr / nr0 > P.tol) status = PCAMG_ENOCONV;
  // true residual
  res_of(x.p, r.p);
  const double true_rel = nr0 > 0.0 ? std::sqrt(dot(r.p, r.p)) / nr0 : 0.0;
  scatter_f64(x.p, A.perm.p, x_nat, n, s);
  sync(s);
  if (st) {
    st->iterations = k;
    st->rebuilds = rebuilds;
    st->levels = (int32_t)c->hist.back()->lv.size();
    st->status = status;
    st->relres = nr0 > 0.0 ? nr / nr0 : 0.0;
    st->true_relres = true_rel;
    st->rho_geo = k > 0 ? std::pow(st->relres, 1.0 / k) : 0.0;
    const int m10 = std::min<int>(10, (int)conv_all.size());
    double s10 = 0.0;
    for (int t = (int)conv_all.size() - m10; t < (int)conv_all.size(); ++t) s10 = s10 + conv_all[t];
    st->convr_last10 = m10 ? s10 / m10 : 0.0;
    st->op_complexity = oc_sum / nh;
    st->t_solve_ms = total.ms();
    st->t_rebuild_ms = t_rebuild;
    st->t_approx_ms = t_approx;
    st->t_build_ms = t_build;
    st->t_setup_ms = c->t_build_ms;
    st->vcycles64 = vc64;
    st->vcycles32 = vc32;
    st->wcycles = wc;
    st->learned_builds = learned_builds;
    st->fallback_builds = fallback_builds;
    st->hist_len = 0;
    if (st->relres_hist && st->hist_cap > 0) {
      const int h = std::min<int>(st->hist_cap, (int)hist.size());
      for (int t = 0; t < h; ++t) st->relres_hist[t] = hist[t];
      st->hist_len = h;
    }
  }
  if (status != PCAMG_OK) throw Error(status, std::string(pcamg_status_str(status)) + " after " + std::to_string(k) +
                                                  " iterations");
}

// Smoother timing on the finest level of the current hierarchy.
void bench_smoother(pcamg_ctx* c, int prec, int sweeps, double* ms, int64_t* launches, double* bytes) {
  hipStream_t s = c->s;
  const LevelMatrix& A = *c->M0;
  const int32_t n = A.n;
  const size_t vs = prec == PCAMG_PREC_F32 ? 4 : 8;
  std::vector<int32_t> rp = to_host(A.rp.p, n + 1, s);
  double per_sweep = 0.0;
  for (int k = 0; k < A.ncol; ++k) {
    const double rows = A.coff[k + 1] - A.coff[k];
    const double nz = rp[A.coff[k + 1]] - rp[A.coff[k]];
    per_sweep += (vs + 4.0) * nz + 4.0 * (rows + 1.0) + 4.0 * vs * rows;
  }
  DVec<double> b(n), x(n);
  DVec<float> b32(n), x32(n);
  xi_fill(c->P.seed, 7, nullptr, b.p, n, s);
  xi_fill(c->P.seed, 8, nullptr, x.p, n, s);
  cast_f64_f32(b.p, b32.p, n, s);
  cast_f64_f32(x.p, x32.p, n, s);
  auto sweep = [&]() {
    for (int k = 0; k < A.ncol; ++k) {
      if (prec == PCAMG_PREC_F32)
        smooth_colour(A, k, b32.p, x32.p, s);
      else
        smooth_colour(A, k, b.p, x.p, s);
    }
    for (int k = A.ncol - 1; k >= 0; --k) {
      if (prec == PCAMG_PREC_F32)
        smooth_colour(A, k, b32.p, x32.p, s);
      else
        smooth_colour(A, k, b.p, x.p, s);
    }
  };
  sweep();  // warm-up
  Timer t(s);
  for (int q = 0; q < sweeps; ++q) sweep();
  *ms = t.ms();
  *launches = (int64_t)sweeps * 2 * A.ncol;
  *bytes = per_sweep * 2.0 * sweeps;
}

// ---------------------------------------------------------------------------
// Roofline measurement on the finest level.  Each repetition first reads a
// scratch buffer of flush_bytes (so the 256 MB last-level cache holds clean
// lines of that buffer and none of the level's data; reading rather than
// writing leaves no dirty lines whose write-back would land in the timed
// pass), then times one forward Gauss-Seidel sweep (kind 0: colours 0..C-1,
// the kernels and launch configuration of the cycles) or one residual
// r = b - A x (kind 1) between HIP events on the context's stream.
// Algorithmic bytes per repetition: matrix values and columns, row pointers,
// and per row four vector entries (GS: x written, x read once, b, dinv;
// residual: x, b, d, r); re-gathered x of neighbouring rows is not counted.
// ---------------------------------------------------------------------------
namespace {
__global__ void fill4_kernel(float4* __restrict__ a, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = make_float4(v, v, v, v);
}
// Reads every element once; one partial sum per block keeps the loads live.
__global__ void __launch_bounds__(256) read_kernel(const float4* __restrict__ a, size_t n, float* __restrict__ part) {
  float acc = 0.0f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = a[i];
    acc += v.x + v.y + v.z + v.w;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}
// Streaming copy: each thread moves four float4 per step, 256 consecutive
// float4 per wavefront access (fully coalesced), grid-stride over the buffer.
__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  const size_t step = (size_t)gridDim.x * blockDim.x * 4;
  for (size_t base = (size_t)blockIdx.x * blockDim.x * 4 + threadIdx.x; base < n; base += step) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = base + (size_t)u * blockDim.x;
      if (i < n) v[u] = a[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = base + (size_t)u * blockDim.x;
      if (i < n) b[i] = v[u];
    }
  }
}
constexpr unsigned READ_BLOCKS = 4096;
}  // namespace

void bench_level(pcamg_ctx* c, int kind, int prec, int reps, int64_t flush_bytes, double* ms, int64_t* launches,
                 double* bytes) {
  hipStream_t s = c->s;
  const LevelMatrix& A = *c->M0;
  const int32_t n = A.n;
  const double vs = prec == PCAMG_PREC_F32 ? 4.0 : 8.0;
  const double per = (vs + 4.0) * A.nnz + 4.0 * (n + 1.0) + 4.0 * vs * n;
  DVec<double> b(n), x(n), r(n);
  DVec<float> b32(n), x32(n), r32(n);
  xi_fill(c->P.seed, 7, nullptr, b.p, n, s);
  xi_fill(c->P.seed, 8, nullptr, x.p, n, s);
  cast_f64_f32(b.p, b32.p, n, s);
  cast_f64_f32(x.p, x32.p, n, s);
  const size_t nf = flush_bytes > 0 ? (size_t)flush_bytes / sizeof(float4) : 0;
  DVec<float4> fl(nf);
  DVec<float> part(nf ? 4 * READ_BLOCKS : 0);
  if (nf) {
    fill4_kernel<<<1024, 256, 0, s>>>(fl.p, nf, 1.0f);
    PCAMG_LAUNCHED();
  }
  hipEvent_t e0, e1;
  PCAMG_HIP(hipEventCreate(&e0));
  PCAMG_HIP(hipEventCreate(&e1));
  int64_t nl = 0;
  auto body = [&]() {
    if (kind == 0) {
      for (int k = 0; k < A.ncol; ++k) {
        if (prec == PCAMG_PREC_F32) smooth_colour(A, k, b32.p, x32.p, s);
        else smooth_colour(A, k, b.p, x.p, s);
        // launches made: one per non-empty colour (long and other rows in one
        // launch), two when both are present and the rows take single lanes
        const int32_t r0 = A.coff[k], r1 = A.coff[k + 1];
        const int32_t rl = A.long_min > 0 && !A.sell() ? A.lend[k] : r0;
        const bool split = A.long_min > 0 && !A.sell() && !(prec == PCAMG_PREC_F32 && A.ell_w > 0) && rl > r0 &&
                           rl < r1 && A.lanes < 4;
        nl += r1 > r0 ? (split ? 2 : 1) : 0;
      }
    } else {
      if (prec == PCAMG_PREC_F32) level_residual(A, b32.p, x32.p, r32.p, s);
      else level_residual(A, b.p, x.p, r.p, s);
      nl += A.sell() ? 1 : (A.n > 0) + (A.nlong > 0);
    }
  };
  double total = 0.0;
  try {
    body();  // warm-up
    nl = 0;
    for (int q = 0; q < reps; ++q) {
      if (nf) {
        read_kernel<<<READ_BLOCKS, 256, 0, s>>>(fl.p, nf, part.p);
        PCAMG_LAUNCHED();
      }
      PCAMG_HIP(hipEventRecord(e0, s));
      body();
      PCAMG_HIP(hipEventRecord(e1, s));
      PCAMG_HIP(hipEventSynchronize(e1));
      float t = 0.0f;
      PCAMG_HIP(hipEventElapsedTime(&t, e0, e1));
      total += t;
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = total;
  *launches = nl;
  *bytes = per * reps;
}

double bench_copy(int64_t nbytes, int reps, hipStream_t s) {
  const size_t n = (size_t)nbytes / sizeof(float4);
  DVec<float4> a(n), b(n);
  fill4_kernel<<<1024, 256, 0, s>>>(a.p, n, 1.0f);
  PCAMG_LAUNCHED();
  const unsigned blocks = (unsigned)std::min<size_t>(8192, std::max<size_t>(1, (n + 1023) / 1024));
  copy_kernel<<<blocks, 256, 0, s>>>(a.p, b.p, n);  // warm-up
  PCAMG_LAUNCHED();
  Timer t(s);
  for (int q = 0; q < reps; ++q) {
    copy_kernel<<<blocks, 256, 0, s>>>(a.p, b.p, n);
    PCAMG_LAUNCHED();
  }
  return t.ms();
}

}  // namespace pcamg
