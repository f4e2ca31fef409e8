// C ABI of the library (declared in include/pcamg.h).  Every entry point
// catches exceptions and returns a status; the message is kept per thread.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <vector>

#include "solver.hpp"

using namespace pcamg;

namespace {
thread_local std::string g_last_error;

template <typename F>
pcamg_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return PCAMG_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PCAMG_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PCAMG_EINVAL;
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// the same, with the thread's allocations tagged to stream s
template <typename F>
pcamg_status guarded_s(hipStream_t s, F&& f) {
  StreamScope scope(s);
  return guarded(std::forward<F>(f));
}

// ---------------------------------------------------------------------------
// Graph validation (the paper's preprocessing, Sec. 4.3): no self loops,
// strictly ascending columns, positive finite symmetric weights, connected.
// ---------------------------------------------------------------------------
// Checks of entry k of row i.
__device__ __forceinline__ void validate_entry(int32_t n, int32_t i, int32_t k, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const double* __restrict__ w,
                                               int32_t* __restrict__ flags) {
  const int32_t j = ci[k];
  if (j < 0 || j >= n) {
    atomicOr(&flags[0], 1);
    return;
  }
  if (j == i) atomicOr(&flags[0], 2);
  if (k > rp[i] && ci[k - 1] >= j) atomicOr(&flags[0], 4);
  const double x = w[k];
  if (!(x > 0.0) || !isfinite(x)) atomicOr(&flags[0], 8);
  // symmetric partner
  int32_t lo = rp[j], hi = rp[j + 1];
  bool found = false;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (ci[mid] == i) { found = true; lo = mid; break; }
    if (ci[mid] < i) lo = mid + 1;
    else hi = mid;
  }
  if (!found || __double_as_longlong(w[lo]) != __double_as_longlong(x)) atomicOr(&flags[0], 16);
}

// Rows of more than VALIDATE_LONG entries (hubs) are checked by a workgroup each.
constexpr int32_t VALIDATE_LONG = 256;

__global__ void validate_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const double* __restrict__ w, int32_t* __restrict__ flags) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || rp[i + 1] - rp[i] > VALIDATE_LONG) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) validate_entry(n, i, k, rp, ci, w, flags);
}

__global__ void __launch_bounds__(256)
    validate_long_kernel(int32_t n, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ ci, const double* __restrict__ w, int32_t* __restrict__ flags) {
  const int32_t i = rows[blockIdx.x];
  for (int32_t k = rp[i] + (int32_t)threadIdx.x; k < rp[i + 1]; k += 256) validate_entry(n, i, k, rp, ci, w, flags);
}

__global__ void rp_check_kernel(int32_t n, int32_t nnz, const int32_t* __restrict__ rp, int32_t* __restrict__ flags) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == 0 && rp[0] != 0) atomicOr(&flags[0], 32);
  if (i == n && rp[n] != nnz) atomicOr(&flags[0], 32);
  if (i < n && rp[i + 1] < rp[i]) atomicOr(&flags[0], 32);
}

__device__ __forceinline__ void cc_hook_entry(int32_t v, int32_t u, int32_t* __restrict__ label,
                                              int32_t* __restrict__ changed) {
  int32_t a = __atomic_load_n(&label[v], __ATOMIC_RELAXED);
  int32_t b = __atomic_load_n(&label[u], __ATOMIC_RELAXED);
  if (a != b) {
    atomicMin(&label[max(a, b)], min(a, b));
    atomicMin(&label[v], min(a, b));
    *changed = 1;
  }
}

__global__ void cc_hook_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               int32_t* __restrict__ label, int32_t* __restrict__ changed) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || rp[v + 1] - rp[v] > VALIDATE_LONG) return;
  for (int32_t k = rp[v]; k < rp[v + 1]; ++k) cc_hook_entry(v, ci[k], label, changed);
}

__global__ void __launch_bounds__(256)
    cc_hook_long_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                        const int32_t* __restrict__ ci, int32_t* __restrict__ label, int32_t* __restrict__ changed) {
  const int32_t v = rows[blockIdx.x];
  for (int32_t k = rp[v] + (int32_t)threadIdx.x; k < rp[v + 1]; k += 256) cc_hook_entry(v, ci[k], label, changed);
}

__global__ void cc_compress_kernel(int32_t n, int32_t* __restrict__ label) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t l = label[v];
  for (int it = 0; it < 64; ++it) {
    int32_t ll = __atomic_load_n(&label[l], __ATOMIC_RELAXED);
    if (ll == l) break;
    l = ll;
  }
  label[v] = l;
}

__global__ void cc_nonzero_kernel(int32_t n, const int32_t* __restrict__ label, int32_t* __restrict__ flags) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && label[v] != 0) atomicOr(&flags[0], 64);
}

void validate_graph(const pcamg_graph* g, hipStream_t s) {
  require(g && g->n > 0 && g->nnz >= 0 && g->row_ptr && (g->nnz == 0 || (g->col_idx && g->weight)), PCAMG_EINVAL,
          "graph: null pointer or bad size");
  const int32_t n = g->n;
  DVec<int32_t> flags(1), label(n), changed(1);
  fill_i32(flags.p, 0, 1, s);
  rp_check_kernel<<<grid_for(n + 1, 256), 256, 0, s>>>(n, g->nnz, g->row_ptr, flags.p);
  PCAMG_LAUNCHED();
  int32_t f = read_scalar(flags.p, s);
  require(!(f & 32), PCAMG_EINVAL, "graph: row pointers not monotone or not ending at nnz");
  validate_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, g->weight, flags.p);
  PCAMG_LAUNCHED();
  DVec<int32_t> lrows;
  const int32_t nl = rows_longer_than(n, g->row_ptr, nullptr, VALIDATE_LONG, lrows, s);
  if (nl > 0) {
    validate_long_kernel<<<nl, 256, 0, s>>>(n, lrows.p, g->row_ptr, g->col_idx, g->weight, flags.p);
    PCAMG_LAUNCHED();
  }
  f = read_scalar(flags.p, s);
  require(!(f & 1), PCAMG_EINVAL, "graph: column index out of range");
  require(!(f & 2), PCAMG_ESELFLOOP, "graph: self loop");
  require(!(f & 4), PCAMG_EDUPEDGE, "graph: columns not strictly ascending (duplicate edge?)");
  require(!(f & 8), PCAMG_EWEIGHT, "graph: weight not positive and finite");
  require(!(f & 16), PCAMG_ENOTSYM, "graph: pattern or weights not symmetric");
  iota_i32(label.p, n, s);
  for (int32_t round = 0; round <= n; ++round) {
    fill_i32(changed.p, 0, 1, s);
    cc_hook_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, label.p, changed.p);
    PCAMG_LAUNCHED();
    if (nl > 0) {
      cc_hook_long_kernel<<<nl, 256, 0, s>>>(lrows.p, g->row_ptr, g->col_idx, label.p, changed.p);
      PCAMG_LAUNCHED();
    }
    cc_compress_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, label.p);
    PCAMG_LAUNCHED();
    if (!read_scalar(changed.p, s)) break;
  }
  cc_nonzero_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, label.p, flags.p);
  PCAMG_LAUNCHED();
  f = read_scalar(flags.p, s);
  require(!(f & 64), PCAMG_EDISCONNECTED, "graph: not connected (extract the largest component)");
}

__global__ void abs_kernel(const double* a, double* b, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = fabs(a[i]);
}

void validate_rhs(const double* b, int32_t n, hipStream_t s) {
  DVec<double> t(n), sums(2);
  abs_kernel<<<grid_for(n, 256), 256, 0, s>>>(b, t.p, n);
  PCAMG_LAUNCHED();
  sum_f64(b, n, sums.p, s);
  sum_f64(t.p, n, sums.p + 1, s);
  auto h = to_host(sums.p, 2, s);
  require(std::isfinite(h[0]) && std::isfinite(h[1]), PCAMG_ERHS, "rhs not finite");
  require(std::fabs(h[0]) <= 1e-12 * h[1], PCAMG_ERHS, "rhs does not sum to zero (graph Laplacians are singular)");
}

// Arrays indexed by stored entry may be null only for a pattern with no
// stored entries: the count rp[n] is read from the device when one is null.
void require_entries(int32_t n, const int32_t* rp, std::initializer_list<const void*> arrays, hipStream_t s) {
  bool all = true;
  for (const void* a : arrays) all = all && a != nullptr;
  if (all) return;
  const int32_t nnz = n > 0 ? read_scalar(rp + n, s) : 0;
  require(nnz == 0, PCAMG_EINVAL, "null entry array for a pattern with stored entries");
}

Hierarchy& hier(pcamg_ctx* c, int32_t h) {
  require(c && h >= 0 && h < (int32_t)c->hist.size(), PCAMG_EINVAL, "hierarchy index out of range");
  return *c->hist[h];
}

}  // namespace

extern "C" {

const char* pcamg_status_str(pcamg_status s) {
  switch (s) {
    case PCAMG_OK: return "ok";
    case PCAMG_EINVAL: return "invalid argument";
    case PCAMG_ENOTSYM: return "graph not symmetric";
    case PCAMG_ESELFLOOP: return "self loop";
    case PCAMG_EDUPEDGE: return "duplicate edge";
    case PCAMG_EWEIGHT: return "bad weight";
    case PCAMG_EDISCONNECTED: return "graph not connected";
    case PCAMG_ERHS: return "rhs not zero-sum";
    case PCAMG_ENOMEM: return "out of memory";
    case PCAMG_EHIP: return "HIP error";
    case PCAMG_ENOCONV: return "no convergence within max_iter";
    case PCAMG_EBREAKDOWN: return "breakdown";
    case PCAMG_ENAN: return "NaN or Inf";
    case PCAMG_EUNSUPPORTED: return "unsupported input";
    default: return "unknown status";
  }
}

const char* pcamg_last_error(void) { return g_last_error.c_str(); }

pcamg_status pcamg_params_default(pcamg_params* p) {
  if (!p) return PCAMG_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-8;
  p->theta = 0.4;
  p->max_iter = 2500;
  p->outer = PCAMG_OUTER_VCYCLE;
  p->cycle_prec = PCAMG_PREC_F64;
  p->coarse_max = 64;
  p->relax_sweeps = 3;
  p->rebuild_vcycles = 2;
  p->rebuild_source = PCAMG_REBUILD_ERROR_APPROX;
  p->p1_mode = PCAMG_P1_SMOOTH;
  p->coarse_solve = PCAMG_COARSE_AUTO;
  p->a2_hub_cap = 0;
  p->max_rebuilds = 50;
  p->max_levels = 64;
  p->numW = 2;
  p->iterW = 7;
  p->iterV = 4;
  p->rebuild_rule = 0;
  p->keep_setup = 0;
  p->validate = 1;
  p->tail_max_n = 2048;
  p->use_graphs = 1;
  p->row_lanes = 0;
  p->w_dense = 1;
  p->first_sweeps = -1;
  p->dense_max_n = 12288;
  p->long_row_min = 256;
  p->v_dense_max_n = 4096;
  p->seed = 0x5EED;
  p->colour_seed = 0xC010;
  p->case3 = 0;
  p->block_sweep_min_colours = 0;
  p->init = PCAMG_INIT_RELAX;
  p->top_dense_max_n = 0;
  return PCAMG_OK;
}

namespace {
// Shared by pcamg_setup and pcamg_setup_learned: context, right-hand side, and
// the first hierarchy from e_first (natural order), or from the relaxed start
// vector when e_first is null.
void setup_impl(const pcamg_graph* g, const double* rhs, const pcamg_params* p, void* stream, pcamg_ctx** out,
                pcamg_net* net) {
  require(g && p && out, PCAMG_EINVAL, "null argument");
  *out = nullptr;
  require(p->row_lanes == -1 || p->row_lanes == 0 || p->row_lanes == 1 || p->row_lanes == 4 || p->row_lanes == 16 ||
              p->row_lanes == 64,
          PCAMG_EINVAL, "row_lanes must be -1, 0, 1, 4, 16 or 64");
  require(p->first_sweeps >= -1 && p->first_sweeps <= 1000, PCAMG_EINVAL, "first_sweeps out of range");
  require(p->long_row_min >= 0, PCAMG_EINVAL, "long_row_min must be >= 0");
  require(p->v_dense_max_n >= 0, PCAMG_EINVAL, "v_dense_max_n must be >= 0");
  require(p->case3 == 0 || p->case3 == 1, PCAMG_EINVAL, "case3 must be 0 or 1");
  require(p->block_sweep_min_colours >= 0, PCAMG_EINVAL, "block_sweep_min_colours must be >= 0");
  require(p->top_dense_max_n >= 0 && p->top_dense_max_n <= 2048, PCAMG_EINVAL,
          "top_dense_max_n must be in [0, 2048]");
  require(p->init == PCAMG_INIT_RELAX || p->init == PCAMG_INIT_MWM, PCAMG_EINVAL, "unknown init");
  require(p->rebuild_source >= PCAMG_REBUILD_ERROR_APPROX && p->rebuild_source <= PCAMG_REBUILD_ITERATE,
          PCAMG_EINVAL, "unknown rebuild_source");
  require(!(net && p->init == PCAMG_INIT_MWM), PCAMG_EINVAL, "the learned setup builds its own first hierarchy");
  hipStream_t s = as_stream(stream);
  if (p->validate) validate_graph(g, s);
  require(g->n >= 1, PCAMG_EINVAL, "empty graph");
  auto c = std::make_unique<pcamg_ctx>();
  c->s = s;
  ctx_init(c.get(), g, p);
  if (rhs) {
    validate_rhs(rhs, g->n, s);
    c->rhs.resize(g->n);
    copy_d2d(c->rhs.p, rhs, g->n, s);
    c->have_rhs = true;
  }
  Timer t(s);
  DVec<double> e(g->n);
  if (p->init == PCAMG_INIT_MWM) {  // MWM_setup (Alg. 5/6 Step 2): no smooth error
    c->hist.push_back(build_hierarchy_mwm(c.get()));
    c->t_build_ms = t.ms();
    *out = c.release();
    return;
  }
  DVec<double> src;
  if (p->keep_setup) {  // the first build's source: the start vector before any sweep
    src.resize(g->n);
    xi_fill(p->seed, 0, nullptr, src.p, g->n, s);
  }
  if (net) {  // the network's proposal from first_sweeps (default 2) sweeps
    c->net = net;
    c->w.resize(std::max(g->nnz, 1));
    copy_d2d(c->w.p, g->weight, g->nnz, s);
    DVec<double> e2(g->n);
    initial_error(c.get(), 0, e2.p, p->first_sweeps >= 0 ? p->first_sweeps : 2);
    net_forward_f64(net, g, e2.p, e.p, s);
  } else {
    initial_error(c.get(), 0, e.p, p->first_sweeps);
  }
  c->hist.push_back(build_hierarchy(c.get(), e.p));
  if (src.p) c->hist.back()->source = std::move(src);
  c->t_build_ms = t.ms();
  *out = c.release();
}
}  // namespace

pcamg_status pcamg_setup(const pcamg_graph* g, const double* rhs, const pcamg_params* p, void* stream,
                         pcamg_ctx** out) {
  return guarded_s(as_stream(stream), [&] { setup_impl(g, rhs, p, stream, out, nullptr); });
}

pcamg_status pcamg_setup_learned(const pcamg_graph* g, const double* rhs, const pcamg_params* p, pcamg_net* net,
                                 void* stream, pcamg_ctx** out) {
  return guarded_s(as_stream(stream), [&] {
    require(net, PCAMG_EINVAL, "null network");
    setup_impl(g, rhs, p, stream, out, net);
  });
}

pcamg_status pcamg_start_vector(const pcamg_graph* g, const pcamg_params* p, int32_t sweeps, double* e,
                                void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(g && p && e && sweeps >= 0, PCAMG_EINVAL, "bad argument");
    hipStream_t s = as_stream(stream);
    if (p->validate) validate_graph(g, s);
    require(g->n >= 1, PCAMG_EINVAL, "empty graph");
    pcamg_ctx c;
    c.s = s;
    ctx_init(&c, g, p);
    initial_error(&c, 0, e, sweeps);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

pcamg_status pcamg_relax_vector(const pcamg_graph* g, const pcamg_params* p, int32_t sweeps, const double* e_in,
                                double* e_out, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(g && p && e_in && e_out && sweeps >= 0, PCAMG_EINVAL, "bad argument");
    hipStream_t s = as_stream(stream);
    if (p->validate) validate_graph(g, s);
    require(g->n >= 1, PCAMG_EINVAL, "empty graph");
    pcamg_ctx c;
    c.s = s;
    ctx_init(&c, g, p);
    if (e_out != e_in) copy_d2d(e_out, e_in, g->n, s);
    relax_homogeneous(&c, e_out, sweeps);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

int32_t pcamg_net_num_params(void) { return net_num_params(); }

pcamg_status pcamg_net_create(pcamg_net** out) {
  return guarded([&] {
    require(out, PCAMG_EINVAL, "null argument");
    net_create(out);
  });
}

void pcamg_net_destroy(pcamg_net* net) {
  if (net) net_destroy(net);
}

pcamg_status pcamg_net_set_params(pcamg_net* net, const float* theta, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net && theta, PCAMG_EINVAL, "null argument");
    net_set_params(net, theta, as_stream(stream));
  });
}

pcamg_status pcamg_net_init(pcamg_net* net, uint64_t seed, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net, PCAMG_EINVAL, "null argument");
    net_init(net, seed, as_stream(stream));
  });
}

pcamg_status pcamg_net_get_params(pcamg_net* net, float* theta, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net && theta, PCAMG_EINVAL, "null argument");
    net_get_params(net, theta, as_stream(stream));
  });
}

pcamg_status pcamg_net_forward(pcamg_net* net, const pcamg_graph* g, const double* e2, float* y, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net && g && e2 && y && g->n >= 1, PCAMG_EINVAL, "bad argument");
    net_forward_f32(net, g, e2, y, as_stream(stream));
  });
}

pcamg_status pcamg_net_loss_grad(pcamg_net* net, const pcamg_graph* g, const double* e2, const double* target,
                                 double* loss, float* grad, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net && g && e2 && target && g->n >= 1, PCAMG_EINVAL, "bad argument");
    const double L = net_loss_grad(net, g, e2, target, grad, as_stream(stream));
    if (loss) *loss = L;
  });
}

pcamg_status pcamg_net_adam_step(pcamg_net* net, float lr, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(net && lr > 0.0f, PCAMG_EINVAL, "bad argument");
    net_adam(net, lr, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_set_rhs(pcamg_ctx* c, const double* rhs) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && rhs, PCAMG_EINVAL, "null argument");
    validate_rhs(rhs, c->n, c->s);
    c->rhs.resize(c->n);
    copy_d2d(c->rhs.p, rhs, c->n, c->s);
    c->have_rhs = true;
  });
}

pcamg_status pcamg_solve(pcamg_ctx* c, double* x, pcamg_stats* st) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && x, PCAMG_EINVAL, "null argument");
    pcamg::solve(c, x, st);
  });
}

pcamg_status pcamg_rebuild(pcamg_ctx* c, const double* e) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c, PCAMG_EINVAL, "null context");
    DVec<double> eb(c->n);
    if (e) {
      copy_d2d(eb.p, e, c->n, c->s);
      relax_homogeneous(c, eb.p, c->P.relax_sweeps);
    } else {
      initial_error(c, (int32_t)c->hist.size(), eb.p);
    }
    c->hist.push_back(build_hierarchy(c, eb.p));
  });
}

void pcamg_destroy(pcamg_ctx* c) {
  if (!c) return;
  try {
    hipStream_t s = c->s;
    (void)hipStreamSynchronize(s);
    {
      StreamScope scope(s);
      delete c;
    }
    dev_cache_idle(s);  // everything enqueued on s has completed
  } catch (...) {
  }
}

// ---------------------------------------------------------------------------
// Batches of independent graphs: the graphs, largest first, each set up and
// solved on a stream of the call's own exactly as the single-graph entry points
// do.  One worker only, on the calling thread: a pool of host threads sharing
// the device ended once in a host segmentation fault whose cause is not
// shown, so several workers are refused.
// ---------------------------------------------------------------------------
pcamg_status pcamg_batch_solve(const pcamg_graph* graphs, const double* const* rhs, double* const* x, int32_t count,
                               const pcamg_params* p, int32_t workers, pcamg_stats* stats) {
  return guarded([&] {
    require(p && count >= 0, PCAMG_EINVAL, "bad argument");
    require(workers == 1, PCAMG_EINVAL,
            "batch workers must be 1 (several host threads are switched off: a host crash there is unexplained)");
    if (count == 0) return;
    require(graphs && rhs && x, PCAMG_EINVAL, "null argument");
    std::vector<int32_t> order(count);
    for (int32_t g = 0; g < count; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return (int64_t)graphs[a].nnz + graphs[a].n > (int64_t)graphs[b].nnz + graphs[b].n;
    });
    std::vector<pcamg_status> status(count, PCAMG_OK);
    std::vector<std::string> msg(count);
    hipStream_t s = nullptr;
    PCAMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (const int32_t g : order) {  // the graphs one after another on the calling thread
      pcamg_ctx* c = nullptr;
      pcamg_status r = pcamg_setup(&graphs[g], rhs[g], p, s, &c);
      pcamg_stats local{};
      pcamg_stats* so = stats ? &stats[g] : &local;
      if (r == PCAMG_OK) {
        r = pcamg_solve(c, x[g], so);
      } else if (stats) {
        pcamg_stats keep = stats[g];
        std::memset(so, 0, sizeof(*so));
        so->relres_hist = keep.relres_hist;
        so->hist_cap = keep.hist_cap;
      }
      so->status = r;
      if (r != PCAMG_OK) msg[g] = pcamg_last_error();
      status[g] = r;
      pcamg_destroy(c);
    }
    (void)hipStreamSynchronize(s);
    dev_cache_idle(s);
    (void)hipStreamDestroy(s);
    for (int32_t g = 0; g < count; ++g)
      if (status[g] != PCAMG_OK) throw Error(status[g], "graph " + std::to_string(g) + ": " + msg[g]);
  });
}

pcamg_status pcamg_num_hierarchies(pcamg_ctx* c, int32_t* count) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && count, PCAMG_EINVAL, "null argument");
    *count = (int32_t)c->hist.size();
  });
}

pcamg_status pcamg_num_levels(pcamg_ctx* c, int32_t h, int32_t* levels) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(levels, PCAMG_EINVAL, "null argument");
    *levels = (int32_t)hier(c, h).lv.size();
  });
}

pcamg_status pcamg_level_info(pcamg_ctx* c, int32_t h, int32_t level, int64_t* info) {
  return guarded_s(c ? c->s : nullptr, [&] {
    Hierarchy& H = hier(c, h);
    require(info && level >= 0 && level < (int32_t)H.lv.size(), PCAMG_EINVAL, "level out of range");
    std::memcpy(info, H.lv[level].info.data(), 16 * sizeof(int64_t));
  });
}

pcamg_status pcamg_level_get(pcamg_ctx* c, int32_t h, int32_t level, const char* name, void* out) {
  return guarded_s(c ? c->s : nullptr, [&] {
    Hierarchy& H = hier(c, h);
    require(out && name && level >= 0 && level < (int32_t)H.lv.size(), PCAMG_EINVAL, "bad argument");
    require(!H.setup.empty(), PCAMG_EINVAL, "level arrays need keep_setup = 1");
    SetupLevel& S = H.setup[level];
    const std::string nm(name);
    if (nm == "source") {
      require(level == 0 && H.source.p != nullptr, PCAMG_EINVAL, "no source vector for this hierarchy");
      PCAMG_HIP(hipMemcpyAsync(out, H.source.p, (size_t)c->n * sizeof(double), hipMemcpyDeviceToHost, c->s));
      PCAMG_HIP(hipStreamSynchronize(c->s));
      return;
    }
    auto gi = [&](const DVec<int32_t>& v, size_t cnt) {
      require(v.p != nullptr, PCAMG_EINVAL, "array '" + nm + "' not present on this level");
      if (cnt) PCAMG_HIP(hipMemcpyAsync(out, v.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, c->s));
    };
    auto gd = [&](const DVec<double>& v, size_t cnt) {
      require(v.p != nullptr, PCAMG_EINVAL, "array '" + nm + "' not present on this level");
      if (cnt) PCAMG_HIP(hipMemcpyAsync(out, v.p, cnt * sizeof(double), hipMemcpyDeviceToHost, c->s));
    };
    if (nm == "colour") gi(S.colour, S.n);
    else if (nm == "agg") gi(S.agg, S.n);
    else if (nm == "A_rp") gi(S.rp, S.n + 1);
    else if (nm == "A_ci") gi(S.ci, S.nnz);
    else if (nm == "path_id") gi(S.path_id, S.n);
    else if (nm == "pos") gi(S.pos, S.n);
    else if (nm == "nb") gi(S.nb, 2 * (size_t)S.n);
    else if (nm == "G_rp") gi(S.grp, S.n + 1);
    else if (nm == "G_ci") gi(S.gci, S.nnz_g);
    else if (nm == "A_v") gd(S.av, S.nnz);
    else if (nm == "d") gd(S.d, S.n);
    else if (nm == "dinv") gd(S.dinv, S.n);
    else if (nm == "pval") gd(S.pval, S.n);
    else if (nm == "G_v") gd(S.gv, S.nnz_g);
    else if (nm == "gkey") gd(S.gkey, S.nnz_g);
    else throw Error(PCAMG_EINVAL, "unknown array name '" + nm + "'");
    PCAMG_HIP(hipStreamSynchronize(c->s));
  });
}

pcamg_status pcamg_cycle(pcamg_ctx* c, int32_t h, const double* b, double* x, int32_t gamma) {
  return guarded_s(c ? c->s : nullptr, [&] {
    Hierarchy& H = hier(c, h);
    require(b && x && gamma >= 1 && gamma <= 2, PCAMG_EINVAL, "bad argument");
    const int32_t n = c->n;
    DVec<double> bp(n), xp(n);
    gather_f64(b, c->M0->perm.p, bp.p, n, c->s);
    gather_f64(x, c->M0->perm.p, xp.p, n, c->s);
    run_cycle64(c, H, bp.p, xp.p, gamma);
    scatter_f64(xp.p, c->M0->perm.p, x, n, c->s);
    PCAMG_HIP(hipStreamSynchronize(c->s));
  });
}

pcamg_status pcamg_cycle32(pcamg_ctx* c, int32_t h, const float* b, float* x, int32_t gamma) {
  return guarded_s(c ? c->s : nullptr, [&] {
    Hierarchy& H = hier(c, h);
    require(b && x && gamma >= 1 && gamma <= 2, PCAMG_EINVAL, "bad argument");
    const int32_t n = c->n;
    DVec<float> bp(n), xp(n);
    gather_f32(b, c->M0->perm.p, bp.p, n, c->s);
    gather_f32(x, c->M0->perm.p, xp.p, n, c->s);
    run_cycle32(c, H, bp.p, xp.p, gamma);
    scatter_f32(xp.p, c->M0->perm.p, x, n, c->s);
    PCAMG_HIP(hipStreamSynchronize(c->s));
  });
}

pcamg_status pcamg_approx_error(pcamg_ctx* c, int32_t count, const double* r, double* e) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && r && e && count >= 1 && count <= (int32_t)c->hist.size(), PCAMG_EINVAL, "bad argument");
    const int32_t n = c->n;
    DVec<double> rp(n), ep(n);
    gather_f64(r, c->M0->perm.p, rp.p, n, c->s);
    approx_error(c, count, rp.p, ep.p, nullptr, nullptr, nullptr);
    scatter_f64(ep.p, c->M0->perm.p, e, n, c->s);
    PCAMG_HIP(hipStreamSynchronize(c->s));
  });
}

pcamg_status pcamg_bench_smoother(pcamg_ctx* c, int32_t prec, int32_t sweeps, double* ms, int64_t* launches,
                                  double* bytes) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && ms && launches && bytes && sweeps >= 1, PCAMG_EINVAL, "bad argument");
    bench_smoother(c, prec, sweeps, ms, launches, bytes);
  });
}

pcamg_status pcamg_bench_level(pcamg_ctx* c, int32_t kind, int32_t prec, int32_t reps, int64_t flush_bytes,
                               double* ms, int64_t* launches, double* bytes) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && ms && launches && bytes && reps >= 1 && (kind == 0 || kind == 1) && flush_bytes >= 0 &&
                (prec == PCAMG_PREC_F64 || prec == PCAMG_PREC_F32),
            PCAMG_EINVAL, "bad argument");
    bench_level(c, kind, prec, reps, flush_bytes, ms, launches, bytes);
  });
}

pcamg_status pcamg_bench_copy(int64_t bytes, int32_t reps, void* stream, double* ms) {
  return guarded_s(as_stream(stream), [&] {
    require(bytes >= 16 && reps >= 1 && ms, PCAMG_EINVAL, "bad argument");
    *ms = bench_copy(bytes, reps, as_stream(stream));
  });
}

pcamg_status pcamg_bench_gemm(int32_t p, int32_t q, int32_t r, int32_t prec, int32_t reps, void* stream,
                              double* ms) {
  return guarded_s(as_stream(stream), [&] {
    require(p >= 1 && q >= 1 && r >= 1 && reps >= 1 && ms, PCAMG_EINVAL, "bad argument");
    require(prec == PCAMG_PREC_F64 || prec == PCAMG_PREC_F32, PCAMG_EINVAL, "prec must be 0 (FP64) or 1 (FP32)");
    *ms = bench_gemm(p, q, r, prec, reps, as_stream(stream));
  });
}

pcamg_status pcamg_initial_error(pcamg_ctx* c, double* e) {
  return guarded_s(c ? c->s : nullptr, [&] {
    require(c && e, PCAMG_EINVAL, "null argument");
    initial_error(c, 0, e);
    PCAMG_HIP(hipStreamSynchronize(c->s));
  });
}

// ---------------------------------------------------------------------------
// Stage entry points
// ---------------------------------------------------------------------------
pcamg_status pcamg_laplacian(int32_t n, const int32_t* rp, const int32_t* ci, const double* w, double* aval,
                             double* d, double* dinv, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n >= 0 && rp && d && dinv, PCAMG_EINVAL, "null argument");
    require_entries(n, rp, {w, aval}, as_stream(stream));
    laplacian(n, rp, w, aval, d, dinv, 0, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_colour(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level,
                          int32_t* colour, int32_t* ncolours, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n >= 0 && rp && colour && ncolours, PCAMG_EINVAL, "null argument");
    require_entries(n, rp, {ci}, as_stream(stream));
    *ncolours = colour_level(n, rp, ci, seed, level, colour, as_stream(stream));
  });
}

pcamg_status pcamg_gs(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, const double* dinv,
                      const int32_t* colour, int32_t ncolours, const double* b, double* x, int32_t forward,
                      int32_t count, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && rp && dinv && colour && b && x && ncolours >= 1, PCAMG_EINVAL, "bad argument");
    hipStream_t s = as_stream(stream);
    require_entries(n, rp, {ci, aval}, s);
    DVec<int32_t> perm(n), iperm(n);
    std::vector<int32_t> coff;
    build_perm(n, colour, ncolours, perm.p, iperm.p, coff, s);
    require((int32_t)coff.size() == ncolours + 1, PCAMG_EINVAL, "colour array inconsistent with ncolours");
    for (int q = 0; q < count; ++q)
      for (int t = 0; t < ncolours; ++t) {
        const int32_t col = forward ? t : ncolours - 1 - t;
        gs_colour_rows<double>(coff[col + 1] - coff[col], perm.p + coff[col], rp, ci, aval, dinv, b, x, s);
      }
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

pcamg_status pcamg_residual(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, const double* d,
                            const double* b, const double* x, double* r, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n >= 0 && rp && d && b && x && r, PCAMG_EINVAL, "null argument");
    require_entries(n, rp, {ci, aval}, as_stream(stream));
    residual<double>(n, rp, ci, aval, d, b, x, r, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_a2_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t hub_cap, int32_t* rp2,
                            int64_t* nnz2, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && rp && rp2 && nnz2 && hub_cap >= 0, PCAMG_EINVAL, "bad argument");
    require_entries(n, rp, {ci}, as_stream(stream));
    *nnz2 = a2_count(n, rp, ci, hub_cap, rp2, as_stream(stream));
  });
}

pcamg_status pcamg_a2_fill(int32_t n, const int32_t* rp, const int32_t* ci, int32_t hub_cap, const int32_t* rp2,
                           int32_t* ci2, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && rp && rp2, PCAMG_EINVAL, "null argument");
    require_entries(n, rp, {ci}, as_stream(stream));
    require_entries(n, rp2, {ci2}, as_stream(stream));
    a2_fill(n, rp, ci, hub_cap, rp2, ci2, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_sort_edges(int32_t n, const int32_t* rp2, const int32_t* ci2, const double* e, int32_t* su,
                              int32_t* sv, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && rp2 && ci2 && e && su && sv, PCAMG_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    const int32_t nnz2 = read_scalar(rp2 + n, s);
    const int32_t m2 = std::max(nnz2 / 2, 1);
    DVec<double> gk(std::max(nnz2, 1)), gv(std::max(nnz2, 1));
    DVec<int32_t> eu(m2), ev(m2);
    DVec<uint64_t> ek(m2), ks(m2);
    DVec<uint32_t> idx(m2), order(m2);
    const int32_t m = a2_keys(n, rp2, ci2, e, gk.p, gv.p, eu.p, ev.p, ek.p, s);
    iota_i32((int32_t*)idx.p, m, s);
    radix_sort_u64_u32(ek.p, idx.p, ks.p, order.p, m, s);
    sorted_endpoints(m, order.p, eu.p, ev.p, su, sv, s);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

pcamg_status pcamg_path_cover(int32_t n, int32_t m, const int32_t* su, const int32_t* sv, int32_t* nb,
                              void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && m >= 0 && nb && (m == 0 || (su && sv)), PCAMG_EINVAL, "bad argument");
    path_cover(n, m, su, sv, nb, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_orient(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen,
                          void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && nb && path_id && pos && plen, PCAMG_EINVAL, "null argument");
    orient_paths(n, nb, path_id, pos, plen, as_stream(stream));
    PCAMG_HIP(hipStreamSynchronize(as_stream(stream)));
  });
}

pcamg_status pcamg_orient_noalloc(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen,
                                  void* stream) {
  return guarded([&] {
    require(n > 0 && nb && path_id && pos && plen, PCAMG_EINVAL, "null argument or n < 1");
    require(n <= PCAMG_ORIENT_NOALLOC_MAX_N, PCAMG_EINVAL,
            "pcamg_orient_noalloc: n = " + std::to_string(n) + " exceeds its fixed workspace (at most " +
                std::to_string(PCAMG_ORIENT_NOALLOC_MAX_N) + " vertices); use pcamg_orient");
    hipStream_t s = as_stream(stream);
    orient_paths_ws(n, nb, path_id, pos, plen, orient_noalloc_scratch(), s);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

pcamg_status pcamg_aggregate(int32_t n, const int32_t* grp, const int32_t* gci, const double* gw,
                             const double* gkey, const int32_t* nb, int32_t* agg, int32_t* nc, int32_t* stats,
                             void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && grp && nb && agg && nc, PCAMG_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    require_entries(n, grp, {gci, gw}, s);
    DVec<int32_t> pid(n), pos(n), plen(n), moff(n + 1), mem(n);
    orient_paths(n, nb, pid.p, pos.p, plen.p, s);
    AggStats st;
    *nc = aggregate_level(n, grp, gci, gw, gkey, nb, pid.p, pos.p, plen.p, agg, moff.p, mem.p, st, s);
    if (stats) {
      stats[0] = st.n_unagg;
      stats[1] = st.case1;
      stats[2] = st.case2;
      stats[3] = st.case3;
      stats[4] = st.middle;
      stats[5] = st.singleton;
    }
  });
}

pcamg_status pcamg_mwm_aggregate(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, int32_t* agg,
                                 int32_t* nc, int32_t* stats, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && rp && agg && nc, PCAMG_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    require_entries(n, rp, {ci, aval}, s);
    DVec<int32_t> moff(n + 1), mem(n);
    AggStats st;
    *nc = mwm_aggregate_level(n, rp, ci, aval, agg, moff.p, mem.p, st, s);
    if (stats) {
      stats[0] = st.n_unagg;
      stats[1] = st.case2;
      stats[2] = st.singleton;
    }
  });
}

namespace {
void members_from_agg(int32_t n, int32_t nc, const int32_t* agg, DVec<int32_t>& moff, DVec<int32_t>& mem,
                      hipStream_t s) {
  DVec<int32_t> inv(n);
  std::vector<int32_t> off;
  mem.resize(n);
  build_perm(n, agg, nc, mem.p, inv.p, off, s);
  require((int32_t)off.size() == nc + 1, PCAMG_EINVAL, "aggregate ids must cover 0..nc-1");
  moff.resize(nc + 1);
  copy_h2d(moff.p, off.data(), nc + 1, s);
  PCAMG_HIP(hipStreamSynchronize(s));
}
}  // namespace

pcamg_status pcamg_galerkin_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t nc,
                                  const int32_t* agg, int32_t* rpc, int64_t* nnzc, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && nc > 0 && rp && agg && rpc && nnzc, PCAMG_EINVAL, "bad argument");
    hipStream_t s = as_stream(stream);
    require_entries(n, rp, {ci}, s);
    DVec<int32_t> moff, mem;
    members_from_agg(n, nc, agg, moff, mem, s);
    *nnzc = galerkin_count(n, rp, ci, nc, moff.p, mem.p, agg, rpc, false, s);
  });
}

pcamg_status pcamg_galerkin_fill(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval,
                                 const double* d, int32_t nc, const int32_t* agg, const double* pval,
                                 const int32_t* rpc, int32_t* cic, double* vc, double* dc, void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && nc > 0 && rp && d && agg && rpc && dc, PCAMG_EINVAL, "bad argument");
    hipStream_t s = as_stream(stream);
    require_entries(n, rp, {ci, aval}, s);
    require_entries(nc, rpc, {cic, vc}, s);
    DVec<int32_t> moff, mem;
    members_from_agg(n, nc, agg, moff, mem, s);
    DVec<double> dinvc(nc);
    galerkin_fill(n, rp, ci, aval, d, nc, moff.p, mem.p, agg, pval, rpc, cic, vc, dc, dinvc.p, false, s);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

pcamg_status pcamg_shorten(int32_t n, const int32_t* nb, int32_t nc, const int32_t* agg, int32_t* nbc,
                           void* stream) {
  return guarded_s(as_stream(stream), [&] {
    require(n > 0 && nc > 0 && nb && agg && nbc, PCAMG_EINVAL, "null argument");
    hipStream_t s = as_stream(stream);
    DVec<int32_t> pid(n), pos(n), plen(n);
    orient_paths(n, nb, pid.p, pos.p, plen.p, s);
    shorten_paths(n, nb, pid.p, pos.p, nc, agg, nbc, s);
    PCAMG_HIP(hipStreamSynchronize(s));
  });
}

}  // extern "C"
