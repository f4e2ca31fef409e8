/*
 * pcamg.h -- C ABI of the MI355X (gfx950) path-cover adaptive AMG library.
 *
 * Method: Hu, Lin & Zikatanov, "An Adaptive Multigrid Method Based on Path
 * Cover" (arXiv 1806.07028): PC-alphaAMG for weighted graph Laplacians
 * L x = b.  Every step runs in this library's HIP kernels on the GPU.
 *
 * Conventions for every entry point:
 *  - Return a pcamg_status (0 = OK, negative = error); no exception crosses
 *    the ABI.  pcamg_last_error() gives a thread-local message for the last
 *    failure of the calling thread.
 *  - "device" pointers are HIP device memory (e.g. torch.cuda tensors' data
 *    pointers) on the current device; "host" pointers are ordinary memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued on it; functions that return sizes or statistics
 *    synchronise the stream before returning.
 *  - Graphs are symmetric CSR with int32 indices: row_ptr[n+1], col_idx[nnz]
 *    ascending within each row, no diagonal entries, no duplicates, weights
 *    w > 0 finite and w(i,j) == w(j,i) bitwise (the paper's preprocessing,
 *    Sec. 4.3: connected, no self loops, positive weights, undirected).
 *  - The caller owns every array it passes; the library copies what it keeps.
 *    Outputs are written into caller-allocated arrays of the stated sizes.
 *  - Threads: one host thread at a time drives the library.  A run with
 *    several host threads solving at once (the former multi-worker batch)
 *    ended in a host crash whose cause is not shown, so concurrent calls from
 *    several threads are not supported.
 */
#ifndef PCAMG_H
#define PCAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pcamg_status;
enum {
  PCAMG_OK = 0,
  PCAMG_EINVAL = -1,        /* bad argument (NULL, size, unknown name) */
  PCAMG_ENOTSYM = -2,       /* graph pattern or weights not symmetric */
  PCAMG_ESELFLOOP = -3,     /* diagonal entry present */
  PCAMG_EDUPEDGE = -4,      /* columns not strictly ascending */
  PCAMG_EWEIGHT = -5,       /* weight <= 0 or not finite */
  PCAMG_EDISCONNECTED = -6, /* graph has more than one component */
  PCAMG_ERHS = -7,          /* |sum b| > 1e-12 sum |b| or not finite */
  PCAMG_ENOMEM = -8,
  PCAMG_EHIP = -9,          /* HIP runtime error */
  PCAMG_ENOCONV = -10,      /* max_iter reached */
  PCAMG_EBREAKDOWN = -11,   /* p^T A p <= 0 in the Krylov iteration */
  PCAMG_ENAN = -12,         /* residual became NaN/Inf */
  PCAMG_EUNSUPPORTED = -13  /* input outside the library's limits (e.g. row too long) */
};

typedef struct pcamg_ctx pcamg_ctx;
typedef struct pcamg_net pcamg_net;  /* learned smooth-error network (extension) */

typedef struct {
  int32_t n;                /* vertices */
  int32_t nnz;              /* stored entries = 2 |E| */
  const int32_t* row_ptr;   /* device [n+1] */
  const int32_t* col_idx;   /* device [nnz] */
  const double* weight;     /* device [nnz] */
} pcamg_graph;

enum { PCAMG_OUTER_VCYCLE = 0, PCAMG_OUTER_FCG = 1 };
enum { PCAMG_PREC_F64 = 0, PCAMG_PREC_F32 = 1 };
enum { PCAMG_P1_SMOOTH = 0, PCAMG_P1_CONST = 1 };
enum { PCAMG_COARSE_AUTO = 0, PCAMG_COARSE_GROUNDED = 1, PCAMG_COARSE_FULL = 2 };
enum { PCAMG_REBUILD_ERROR_APPROX = 0, PCAMG_REBUILD_RELAX = 1, PCAMG_REBUILD_ITERATE = 2 };
enum { PCAMG_INIT_RELAX = 0, PCAMG_INIT_MWM = 1 };

typedef struct {
  double tol;              /* relative residual ||b - A x|| / ||b|| (default 1e-8, Sec. 4) */
  double theta;            /* re-setup threshold on the mean ConvR since the last re-setup (Alg. 5; 0.4) */
  int32_t max_iter;        /* 2500 (Sec. 4: "--" beyond 2500 iterations) */
  int32_t outer;           /* PCAMG_OUTER_VCYCLE (Alg. 5) or PCAMG_OUTER_FCG (V-cycle preconditioned FCG) */
  int32_t cycle_prec;      /* precision of every preconditioning cycle (outer FCG and Alg. 2's PCG):
                              PCAMG_PREC_F64 or PCAMG_PREC_F32 */
  int32_t coarse_max;      /* coarsest level size (64) */
  int32_t relax_sweeps;    /* symmetric GS sweeps on A e = 0 before each build (3) */
  int32_t rebuild_vcycles; /* V-cycles on A e = 0 (PCAMG_REBUILD_RELAX only; 2) */
  int32_t rebuild_source;  /* PCAMG_REBUILD_ERROR_APPROX (Alg. 2, default), PCAMG_REBUILD_RELAX, or
                              PCAMG_REBUILD_ITERATE (Alg. 6, b = 0: the current iterate x_{k+1} is
                              the smooth error, used without further sweeps; with rebuild_rule 1
                              and a zero right-hand side this is Alg. 6) */
  int32_t p1_mode;         /* PCAMG_P1_SMOOTH (Sec. 3.3, default) or PCAMG_P1_CONST */
  int32_t coarse_solve;    /* PCAMG_COARSE_AUTO / GROUNDED / FULL */
  int32_t a2_hub_cap;      /* 0 = exact A^2 pattern; K > 0: two-step pairs only via degree <= K */
  int32_t max_rebuilds;    /* 50 */
  int32_t max_levels;      /* 64 */
  int32_t numW, iterW, iterV; /* Alg. 2 parameters (2, 7, 4; Sec. 4) */
  int32_t rebuild_rule;    /* 0 mean ConvR since last re-setup (Alg. 5), 1 last ConvR (Alg. 6) */
  int32_t keep_setup;      /* 1 = keep per-level setup arrays for pcamg_level_get */
  int32_t validate;        /* 1 = check the graph (symmetry, weights, connectivity) in pcamg_setup */
  int32_t tail_max_n;      /* levels with at most this many vertices run as one single-workgroup
                              launch per cycle (2048; 0 = per-step launches everywhere) */
  int32_t use_graphs;      /* 1 = replay whole cycles from captured HIP graphs */
  int32_t row_lanes;       /* lanes per matrix row in the smoother/residual kernels: 0 = by the
                              level's mean row length; -1 = autotuned: each launched level
                              (more than 2048 vertices) times one sweep with 1 (sliced-ELL
                              when available), 4 and 16 lanes and keeps the fastest, cached
                              per level shape for the process; else 1, 4, 16 or 64.  Results
                              are identical for every setting */
  int32_t w_dense;         /* 1 = in W-cycles, the two sub-cycles of the first level of at most
                              dense_max_n vertices are applied as one precomputed dense operator
                              (equal up to rounding order; built level by level from the coarsest
                              on first use per hierarchy and precision, GEMMs on the matrix cores);
                              0 = recurse */
  int32_t first_sweeps;    /* symmetric sweeps before the first build: -1 = relax_sweeps; with
                              pcamg_setup_learned the sweeps of the network's input (-1: 2) */
  int32_t dense_max_n;     /* w_dense: the dense operator starts at the first level of at most this
                              many vertices below the finest (12288); levels above 65535 vertices
                              are not built (the W-cycle then recurses) */
  int32_t long_row_min;    /* rows of at least this many entries take one workgroup each in the
                              cycles' smoother and residual kernels, with a fixed summation tree
                              instead of the single chain in stored order (equal up to rounding
                              order; hubs of power-law graphs).  The relaxation of the start
                              vector before a build always keeps the chain.  0 = off (256: above
                              the longest rows of grid hierarchies) */
  int32_t v_dense_max_n;   /* V-cycles: the cycle of the first level of at most this many vertices
                              (or of at most twice as many, when it has more than one colour per
                              16 rows: the hub levels of power-law hierarchies)
                              below the finest (at or above the single-workgroup tail) is applied
                              by the level above as one precomputed dense operator (equal up to
                              rounding order; built level by level from the coarsest on first use
                              per hierarchy and precision, GEMMs on the matrix cores).  0 = recurse
                              (4096) */
  uint64_t seed;           /* start-vector stream */
  uint64_t colour_seed;    /* colouring priority stream */
  int32_t case3;           /* Alg. 3 Case 3: 0 = v leaves its aggregate only when the rest stays
                              connected (else u joins at v; aggregates may grow past three as stars
                              of diameter 2); 1 = as printed in Step 17 (v always leaves) */
  int32_t block_sweep_min_colours; /* a launched level with at least this many colours and at most 64
                              rows per colour on average runs each Gauss-Seidel sweep of the cycles
                              in one single-workgroup launch (same arithmetic, bit-identical
                              results).  0 = off (default: on the near-dense coarse levels of
                              the 4M power-law graph one workgroup's bandwidth made a sweep 2.3x
                              slower than a launch per colour) */
  int32_t init;            /* first hierarchy: PCAMG_INIT_RELAX (path cover of the relaxed start
                              vector, default) or PCAMG_INIT_MWM (UA-AMG with MWM aggregation on
                              every level, the MWM_setup of Alg. 5/6 Step 2, Sec. 2.1).  With
                              max_rebuilds = 0 and PCAMG_INIT_MWM the solve is the paper's
                              UA-AMG baseline */
  int32_t top_dense_max_n; /* a graph of at most this many vertices (at most 2048) runs each cycle
                              type as one precomputed dense operator C of the whole cycle, applied
                              from any start vector as x + C (b - A x) (equal up to rounding
                              order; built from the coarsest level up on first use per hierarchy,
                              cycle type and precision; needs w_dense for W-cycles and
                              v_dense_max_n > 0 for V-cycles).  0 = off (default: the
                              single-workgroup tail; the adaptive loop's counts then follow the
                              recursive cycle's rounding) */
} pcamg_params;

typedef struct {
  int32_t iterations, rebuilds, levels, status;
  double relres;           /* recursive residual ratio at exit */
  double true_relres;      /* ||b - A x|| / ||b|| recomputed at exit */
  double rho_geo;          /* (relres)^(1/iterations) */
  double convr_last10;     /* mean ConvR over the last 10 iterations (Sec. 4) */
  double op_complexity;    /* mean operator complexity over all hierarchies (Sec. 4) */
  double t_setup_ms;       /* first hierarchy (pcamg_setup) */
  double t_solve_ms;       /* whole pcamg_solve call */
  double t_rebuild_ms;     /* re-setups inside the solve (Alg. 2 + Alg. 4) */
  double t_approx_ms;      /* of which error approximation (Alg. 2) */
  double t_build_ms;       /* of which hierarchy builds (Alg. 4) */
  int32_t vcycles64, vcycles32, wcycles; /* cycle applications by kind */
  int32_t hist_len;        /* entries written to relres_hist */
  double* relres_hist;     /* host, optional: relres after each iteration (index 0 = 1.0) */
  int32_t hist_cap;        /* capacity of relres_hist */
  int32_t learned_builds;  /* re-setups built from the network's proposal (pcamg_setup_learned) */
  int32_t fallback_builds; /* re-setups of a learned context built from the plain relaxation */
} pcamg_stats;

const char* pcamg_status_str(pcamg_status s);
const char* pcamg_last_error(void);

/* Defaults listed above. */
pcamg_status pcamg_params_default(pcamg_params* p);

/* ------------------------------------------------------------------------
 * Solver (Alg. 5)
 * ------------------------------------------------------------------------ */

/* Validate the graph (if p->validate), build the Laplacian A = D - W
 * (Sec. 2.2), colour the finest level and build the first hierarchy (Alg. 4)
 * from a start vector relaxed by relax_sweeps symmetric GS sweeps on A e = 0.
 * rhs (device [n], nullable) must be zero-sum (PCAMG_ERHS otherwise); it can
 * be given later with pcamg_set_rhs.  On success *out owns all device memory
 * of the solver until pcamg_destroy. */
pcamg_status pcamg_setup(const pcamg_graph* g, const double* rhs, const pcamg_params* p, void* stream,
                         pcamg_ctx** out);

/* Replace the right-hand side (device [n], zero-sum). */
pcamg_status pcamg_set_rhs(pcamg_ctx* c, const double* rhs);

/* Adaptive solve (Alg. 5): V(1,1)-cycles (or FCG with a V-cycle
 * preconditioner), x made orthogonal to 1 after each step, ConvR =
 * ||r_{k+1}|| / ||r_k||, re-setup when the mean ConvR since the last re-setup
 * exceeds theta: error approximation (Alg. 2) over all hierarchies so far,
 * relaxation, new hierarchy (Alg. 4), x <- x + e.  x: device [n], input x0,
 * output x.  st: host, nullable.  Returns PCAMG_ENOCONV if tol is not
 * reached in max_iter iterations (x still holds the last iterate). */
pcamg_status pcamg_solve(pcamg_ctx* c, double* x, pcamg_stats* st);

/* Build one more hierarchy (Alg. 4) from the smooth error e (device [n],
 * natural order) after relax_sweeps symmetric sweeps on A e = 0 (e is not
 * modified); e == NULL uses the next start vector of the seed stream.  The
 * new hierarchy becomes current and joins the history. */
pcamg_status pcamg_rebuild(pcamg_ctx* c, const double* e);

void pcamg_destroy(pcamg_ctx* c);

/* Batched setup and solve of independent graphs (the batching extension;
 * per graph exactly Alg. 5 as pcamg_setup + pcamg_solve).  The calling
 * thread takes the graphs largest first on a HIP stream of its own (default
 * priority); each graph is set up, solved and released on that stream, so
 * x[g] and stats[g] equal those of the individual calls bit for bit.
 * `workers` must be 1: several host threads are switched off (PCAMG_EINVAL)
 * because one run of that path ended in a host crash with no cause shown.  graphs[count]: device CSR as for
 * pcamg_setup; rhs[g]: device [n_g] (must sum to 0); x[g]: device [n_g],
 * initial guess in, solution out; stats: host [count] or NULL (each entry's
 * relres_hist/hist_cap are used as in pcamg_solve; status holds the graph's
 * own result).  Returns PCAMG_OK if every graph converged, else the status of
 * the lowest-numbered failing graph (the others are still solved). */
pcamg_status pcamg_batch_solve(const pcamg_graph* graphs, const double* const* rhs, double* const* x, int32_t count,
                               const pcamg_params* p, int32_t workers, pcamg_stats* stats);

/* ------------------------------------------------------------------------
 * Hierarchy access (inspection and stage tests)
 * ------------------------------------------------------------------------ */

/* Number of hierarchies built so far (history, Alg. 5 P_hist). */
pcamg_status pcamg_num_hierarchies(pcamg_ctx* c, int32_t* count);
pcamg_status pcamg_num_levels(pcamg_ctx* c, int32_t h, int32_t* levels);

/* info[16] (host): n, nnz(A_l off-diagonal), ncolours, n_next, nnz(level
 * graph), paths, unaggregated after pairing, case1, case2, case3, middle,
 * singleton, p1 fallbacks, coarsest grounded, coarsest fallback, path vertices.
 * The level-graph and path counts need keep_setup. */
pcamg_status pcamg_level_info(pcamg_ctx* c, int32_t h, int32_t level, int64_t* info);

/* Copy a per-level array, natural vertex order, to host memory `out`.
 * Names (int32): "colour"[n], "agg"[n], "A_rp"[n+1], "A_ci"[nnz],
 * "path_id"[n], "pos"[n], "nb"[2n], "G_rp"[n+1], "G_ci"[nnz_G];
 * (double): "A_v"[nnz], "d"[n], "dinv"[n], "pval"[n], "G_v"[nnz_G],
 * "gkey"[nnz_G] (level 0), "source"[n] (level 0: the vector the hierarchy was
 * built from before any relaxation sweep -- the start vector for the first,
 * the error approximation or fresh start vector of a re-setup).  Setup arrays
 * (path_id, pos, nb, G_*, gkey, source) need keep_setup = 1.  Returns
 * PCAMG_EINVAL for an unknown or absent name. */
pcamg_status pcamg_level_get(pcamg_ctx* c, int32_t h, int32_t level, const char* name, void* out);

/* One multigrid cycle of hierarchy h (gamma 1 = V(1,1), 2 = W) on A x = b at
 * the finest level, natural order, device [n] vectors, in FP64. */
pcamg_status pcamg_cycle(pcamg_ctx* c, int32_t h, const double* b, double* x, int32_t gamma);

/* The same cycle in FP32 on FP32 copies of the operators (coarsest solve in
 * FP64), device [n] float vectors. */
pcamg_status pcamg_cycle32(pcamg_ctx* c, int32_t h, const float* b, float* x, int32_t gamma);

/* Error approximation (Alg. 2) with hierarchies 0..count-1 as the history
 * (Re = count): PCG steps on A e = r from e = 0, W-cycle preconditioner of the
 * latest while Re <= numW, else the symmetric composite of all V-cycles
 * (cycles in the precision cycle_prec); result made orthogonal to 1.  r, e:
 * device [n] natural order. */
pcamg_status pcamg_approx_error(pcamg_ctx* c, int32_t count, const double* r, double* e);

/* Time `sweeps` symmetric multicoloured Gauss-Seidel sweeps (the smoother of
 * every V-cycle) on the finest level of the current hierarchy, in the solve
 * layout and launch configuration used by the cycles, with HIP events on the
 * context's stream.  prec: PCAMG_PREC_F64 or PCAMG_PREC_F32.  Uses internal
 * scratch vectors only.  Outputs (host): total milliseconds, kernel launches,
 * algorithmic bytes (per row pass: matrix values and columns, row pointers,
 * x written, x read once, b, dinv). */
pcamg_status pcamg_bench_smoother(pcamg_ctx* c, int32_t prec, int32_t sweeps, double* ms, int64_t* launches,
                                  double* bytes);

/* Roofline measurement on the finest level of the context, in the solve
 * layout and launch configuration of the cycles.  Each of `reps`
 * repetitions first reads flush_bytes (0 = none) of a scratch buffer, so
 * that the last-level cache holds none of the level (and no dirty lines whose
 * write-back would fall into the timed pass), then runs between HIP
 * events on the context's stream either one forward multicoloured
 * Gauss-Seidel sweep (kind 0, colours 0..C-1) or one residual r = b - A x
 * (kind 1), in precision prec.  Outputs (host): summed event milliseconds,
 * kernel launches timed, algorithmic bytes = reps x ((s+4) nnz + 4 (n+1) +
 * 4 s n), s = 8 (FP64) or 4 (FP32): matrix values and columns, row pointers,
 * x written / read once, b, dinv (GS) or d, x, b, r (residual). */
pcamg_status pcamg_bench_level(pcamg_ctx* c, int32_t kind, int32_t prec, int32_t reps, int64_t flush_bytes,
                               double* ms, int64_t* launches, double* bytes);

/* Device-copy ceiling: `reps` copies of `bytes` (rounded down to 16) between
 * two device buffers by this library's streaming copy kernel, timed with HIP
 * events on `stream`; *ms (host) is the total.  Each copy moves 2 x bytes. */
pcamg_status pcamg_bench_copy(int64_t bytes, int32_t reps, void* stream, double* ms);

/* The matrix-core GEMM of the dense operators (the product of Alg. 2's
 * W-cycle operator construction): `reps` products P = Q R of row-major
 * p x q and q x r operands (deterministic values in [-1, 1), allocated and
 * freed here) in FP64 (prec 0) or FP32 (prec 1), timed with HIP events on
 * `stream`; *ms (host) is the total.  Each product is 2 p q r flops.
 * PCAMG_EINVAL for sizes below 1 or reps below 1. */
pcamg_status pcamg_bench_gemm(int32_t p, int32_t q, int32_t r, int32_t prec, int32_t reps, void* stream,
                              double* ms);

/* Smooth error of the first build: start vector of build 0 (SplitMix64
 * stream p->seed) and relax_sweeps symmetric sweeps on A e = 0. device [n]. */
pcamg_status pcamg_initial_error(pcamg_ctx* c, double* e);

/* ------------------------------------------------------------------------
 * Learned smooth-error proposals (extension).  The path cover orders edges by
 * |e_i - e_j| of a smooth error e (Alg. 4, Step 2; Sec. 3.2); a three-layer
 * message-passing network maps a vector relaxed by two sweeps to a smoother
 * one, in place of the first build's relaxation:
 *   u = normalise(e2) (mean 0, RMS 1), l = log d - mean(log d), Ahat = D^-1 W,
 *   F = [u, Ahat u, l, Ahat l];  h0 = relu(F W0 + b0);
 *   h_k = relu(bf16([h_{k-1} | Ahat h_{k-1}]) bf16(W_k) + b_k), k = 1..3;
 *   y = h3 wo + bo + u;  loss = 0.5 mean((y - normalise(t))^2).
 * Hidden width 64; parameters (float32, host order) W0 [4][64], b0 [64],
 * then for k = 1..3 W_k [128][64] and b_k [64], then wo [64], bo [1].  The
 * hidden-layer products and their backward products use bf16 MFMA with float32
 * accumulation; sums over nodes are ordered, so results are reproducible.
 * ------------------------------------------------------------------------ */

/* Number of float32 parameters (25,153). */
int32_t pcamg_net_num_params(void);

/* New network.  Parameters, Adam state and gradient are zero and the network
 * is not usable yet: pcamg_net_forward, pcamg_net_loss_grad,
 * pcamg_net_adam_step and pcamg_setup_learned return PCAMG_EINVAL until
 * pcamg_net_init or pcamg_net_set_params has given it parameters.  Owns
 * device memory until pcamg_net_destroy. */
pcamg_status pcamg_net_create(pcamg_net** out);
void pcamg_net_destroy(pcamg_net* net);

/* Parameters from / to host float32 [pcamg_net_num_params()]; setting them
 * also resets the Adam state. */
pcamg_status pcamg_net_set_params(pcamg_net* net, const float* theta, void* stream);
pcamg_status pcamg_net_get_params(pcamg_net* net, float* theta, void* stream);

/* Seeded initial parameters, computed on the device: flat entry k draws word
 * k + 1 of the SplitMix64 stream `seed` (u = (word >> 11) 2^-53) and takes
 * (2u - 1) lim rounded to float32, with lim = sqrt(6 / (fan_in + fan_out))
 * for W0 (4 x 64) and W1..W3 (128 x 64), 0.1 for wo and 0 for every bias
 * (Glorot-uniform weights).  Also resets the Adam state. */
pcamg_status pcamg_net_init(pcamg_net* net, uint64_t seed, void* stream);

/* Forward pass: y (device float [n]) from the graph (as for pcamg_setup) and
 * the relaxed vector e2 (device double [n], natural order). */
pcamg_status pcamg_net_forward(pcamg_net* net, const pcamg_graph* g, const double* e2, float* y, void* stream);

/* Loss against target t (device double [n]; any scale and offset) and its
 * gradient, kept in the network for pcamg_net_adam_step and copied to grad
 * (host float [num_params]) when grad is not NULL; *loss on the host. */
pcamg_status pcamg_net_loss_grad(pcamg_net* net, const pcamg_graph* g, const double* e2, const double* target,
                                 double* loss, float* grad, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * last gradient. */
pcamg_status pcamg_net_adam_step(pcamg_net* net, float lr, void* stream);

/* `sweeps` symmetric multicolour Gauss-Seidel sweeps on A e = 0 (the
 * relaxation before every build, Sec. 3.2) applied to e_in (device double
 * [n], natural order) into e_out (may alias e_in). */
pcamg_status pcamg_relax_vector(const pcamg_graph* g, const pcamg_params* p, int32_t sweeps, const double* e_in,
                                double* e_out, void* stream);

/* The start vector of the first build: SplitMix64 xi (stream p->seed, build 0)
 * relaxed by `sweeps` symmetric multicolour Gauss-Seidel sweeps on A e = 0
 * (Sec. 3.2), device double [n], natural order. */
pcamg_status pcamg_start_vector(const pcamg_graph* g, const pcamg_params* p, int32_t sweeps, double* e,
                                void* stream);

/* pcamg_setup with every hierarchy built from the network's proposal: the
 * first from the start vector, each re-setup of Alg. 5 from its source vector
 * (Alg. 2's error approximation), each relaxed by p->first_sweeps sweeps (-1:
 * 2) instead of relax_sweeps and mapped by the network to the smooth error
 * whose level sets give the path-cover keys (Alg. 4 Step 2).  The measured
 * convergence factor decides: a learned hierarchy whose first ConvR
 * exceeds 0.9 hands the next build to the plain relaxation of relax_sweeps
 * sweeps.  `net` must stay alive and unchanged until pcamg_destroy. */
pcamg_status pcamg_setup_learned(const pcamg_graph* g, const double* rhs, const pcamg_params* p, pcamg_net* net,
                                 void* stream, pcamg_ctx** out);

/* ------------------------------------------------------------------------
 * Stage entry points: single steps of the method on caller arrays (device
 * unless stated).  Used for parity tests and benchmarks.  Arrays indexed by
 * stored entry (ci, w, aval, gci, gw, ci2, cic, vc) may be NULL only when
 * their pattern has no stored entries (rp[n] = 0, read from the device when
 * one of them is NULL); any other NULL gives PCAMG_EINVAL before a launch.
 * ------------------------------------------------------------------------ */

/* Laplacian (Sec. 2.2): aval[nnz] = -w, d[n] = row sums in CSR order, dinv = 1/d. */
pcamg_status pcamg_laplacian(int32_t n, const int32_t* rp, const int32_t* ci, const double* w, double* aval,
                             double* d, double* dinv, void* stream);

/* Multicolouring used by the Gauss-Seidel smoother (Sec. 4 names the smoother
 * only as Gauss-Seidel; the ordering is this library's).  A connected
 * bipartite graph gets the red-black colouring: parity of the breadth-first
 * distance from vertex 0 (2 colours, 1 if n = 1).  Any other graph gets
 * Jones-Plassmann rounds = greedy first-fit in descending (key, id) order,
 * key = min(degree, 2^24 - 1) << 40 | (SplitMix64 word (level << 32) + v + 1
 * of stream seed) >> 24: largest degree first, random among equal degrees.  rp, ci: device CSR of a
 * symmetric pattern without self loops; colour: device int32 [n], written;
 * *ncolours: host.  PCAMG_EINVAL on null arguments or n < 0. */
pcamg_status pcamg_colour(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level,
                          int32_t* colour, int32_t* ncolours, void* stream);

/* `count` multicoloured GS passes (forward: colours 0..C-1, backward:
 * C-1..0) on A x = b with A = off-diagonal (rp, ci, aval) + diagonal dinv^-1. */
pcamg_status pcamg_gs(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, const double* dinv,
                      const int32_t* colour, int32_t ncolours, const double* b, double* x, int32_t forward,
                      int32_t count, void* stream);

/* r = b - (D + offdiag) x, sum order d_i x_i then CSR order. */
pcamg_status pcamg_residual(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, const double* d,
                            const double* b, const double* x, double* r, void* stream);

/* Off-diagonal A^2 pattern (Alg. 4, Step 2), two calls: rp2[n+1] and *nnz2
 * (host), then ci2[nnz2]. */
pcamg_status pcamg_a2_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t hub_cap, int32_t* rp2,
                            int64_t* nnz2, void* stream);
pcamg_status pcamg_a2_fill(int32_t n, const int32_t* rp, const int32_t* ci, int32_t hub_cap, const int32_t* rp2,
                           int32_t* ci2, void* stream);

/* Undirected edges (i < j) of a symmetric pattern sorted by (|e_i - e_j|
 * ascending, lexicographic edge index ascending) = heaviest reweighted edge
 * first (Alg. 4 Step 2, Alg. 1 Step 3).  The pattern's rows are sorted by
 * column with no diagonal (as pcamg_a2_fill gives them).  su, sv: device
 * int32 [nnz2/2]. */
pcamg_status pcamg_sort_edges(int32_t n, const int32_t* rp2, const int32_t* ci2, const double* e, int32_t* su,
                              int32_t* sv, void* stream);

/* Greedy path cover (Alg. 1) visiting the m edges (su[t], sv[t]) in order t.
 * nb: device int32 [2n], the cover neighbours of each vertex (-1 = none). */
pcamg_status pcamg_path_cover(int32_t n, int32_t m, const int32_t* su, const int32_t* sv, int32_t* nb,
                              void* stream);

/* Paths of a cover: start at the smaller endpoint; path_id (= start vertex),
 * pos, path length; -1/-1/0 for vertices on no path.  device int32 [n] each. */
pcamg_status pcamg_orient(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen,
                          void* stream);

/* pcamg_orient for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results, with the pointer-jumping workspace in a fixed device
 * array of the library (12 n + 1 int32 for n up to PCAMG_ORIENT_NOALLOC_MAX_N
 * = 2^19 vertices: 24 MiB per GPU, held from the first call on a GPU until the
 * process ends).  Calls no allocator.  n above the maximum returns
 * PCAMG_EINVAL without touching the GPU.  Every call on one GPU uses that
 * GPU's one workspace, so calls that overlap on one GPU (several host threads
 * or streams) race; the caller serialises them.  Synchronises `stream`. */
#define PCAMG_ORIENT_NOALLOC_MAX_N (1 << 19)
pcamg_status pcamg_orient_noalloc(int32_t n, const int32_t* nb, int32_t* path_id, int32_t* pos, int32_t* plen,
                                  void* stream);

/* Aggregation along a cover (Alg. 3): pairing along paths, isolated vertices
 * in ascending id (Cases 1-3), aggregates numbered by smallest member.  In
 * Case 3 the best neighbour v leaves its aggregate only if the rest stays
 * connected; when v is the middle of a 3-chain or the centre of a star grown
 * that way, u joins v's aggregate ("middle"), so aggregates may exceed three
 * members (stars, diameter 2; Sec. 3.3 leaves no vertex isolated).
 * Level graph (grp, gci, gw) with optional keys gkey (finest level: smaller
 * key = heavier).  agg: device [n]; *nc and stats[6] (host): unaggregated,
 * case1, case2, case3, middle (joins at the middle or centre), singleton
 * (no neighbour). */
pcamg_status pcamg_aggregate(int32_t n, const int32_t* grp, const int32_t* gci, const double* gw,
                             const double* gkey, const int32_t* nb, int32_t* agg, int32_t* nc, int32_t* stats,
                             void* stream);

/* MWM aggregation (Sec. 2.1) of one level with off-diagonal entries aval
 * (weights w_ij = -aval): edges visited heaviest first (ties by lexicographic
 * edge index) match two unaggregated ends; every vertex left over joins the
 * aggregate of its heaviest neighbour (ties to the smaller id), so aggregates
 * keep diameter <= 3; aggregates numbered by smallest member.  rp, ci, aval:
 * device CSR (aval < 0); agg: device int32 [n]; *nc and stats[3] (host):
 * left after the matching, joined, singletons.  PCAMG_EINVAL on null
 * arguments or n < 1. */
pcamg_status pcamg_mwm_aggregate(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval, int32_t* agg,
                                 int32_t* nc, int32_t* stats, void* stream);

/* Galerkin product P^T A P (Alg. 4, Step 8) for P with one value pval[k] in
 * column agg[k].  Two calls: rpc[nc+1] and *nnzc (host), then cic[nnzc],
 * vc[nnzc], dc[nc]. */
pcamg_status pcamg_galerkin_count(int32_t n, const int32_t* rp, const int32_t* ci, int32_t nc,
                                  const int32_t* agg, int32_t* rpc, int64_t* nnzc, void* stream);
pcamg_status pcamg_galerkin_fill(int32_t n, const int32_t* rp, const int32_t* ci, const double* aval,
                                 const double* d, int32_t nc, const int32_t* agg, const double* pval,
                                 const int32_t* rpc, int32_t* cic, double* vc, double* dc, void* stream);

/* Path shortening (Alg. 4, Step 7): coarse cover nbc[2 nc] from a cover and
 * an aggregation. */
pcamg_status pcamg_shorten(int32_t n, const int32_t* nb, int32_t nc, const int32_t* agg, int32_t* nbc,
                           void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PCAMG_H */
