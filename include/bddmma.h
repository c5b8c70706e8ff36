/*
 * bddmma — C ABI of the MI355X BDD Lagrange-decomposition solver for 0-1 ILPs
 * (FastDOG, Abbas & Swoboda, CVPR 2022).
 *
 * Problem (Sec. 3, Def. "Binary Program" and Example "ILP"):
 *     min c^T x   s.t.  every row  sum_k a_k x_{i_k}  (<=, ==, >=)  b,   x in {0,1}^n.
 * Every row becomes one subproblem j with feasible set X_j, represented by a
 * binary decision diagram (Sec. 5, Def. "BDD").  The solver maximises the
 * Lagrangean dual (Sec. 3, problem (D)) with the parallel deferred
 * min-marginal averaging of Alg. 1 and decodes primal points with the
 * perturbation rounding of Alg. 2.
 *
 * Conventions shared by every entry point
 *  - Return value: BDDMMA_OK (0) or one of the negative codes below.  No C++
 *    exception crosses this interface.  bddmma_last_error() returns a
 *    thread-local, NUL-terminated message for the last failing call on the
 *    calling thread (valid until that thread's next failing call).
 *  - Host arrays passed in are read during the call only; the caller keeps
 *    ownership.  Host output arrays are caller-allocated with the sizes that
 *    the matching query returns.
 *  - Device memory: the library allocates none.  After bddmma_load_ilp the
 *    caller asks bddmma_workspace_bytes, allocates that many bytes of device
 *    memory (256-byte aligned) and hands them over with bddmma_bind together
 *    with a HIP stream.  The library never frees the buffer; it must stay
 *    allocated until bddmma_destroy.  All device work is ordered on that
 *    stream; calls that return host values synchronise it.  A solver bound
 *    with bddmma_bind keeps one pinned host buffer (hipHostMalloc, allocated
 *    at its first readback, at most 512 MiB, freed by bddmma_destroy) for the
 *    values it copies back; one bound with bddmma_bind_static does not.
 *    Uploads of 1 MB or more go through one pinned host buffer per device
 *    (64 MiB, two halves filled by host threads while the other is copied),
 *    shared by all solvers of the process, made by the first bddmma_bind on
 *    that device and kept until the process ends; a solver bound with
 *    bddmma_bind_static copies directly and starts no host thread.
 *  - Pair order: a "pair" is a (variable i, subproblem j) with i in I_j.
 *    Host-visible pair arrays list subproblems in ascending original row
 *    order and, inside one subproblem, variables in ascending id order.
 *  - A solver is not thread safe; distinct solvers may be used concurrently.
 */
#ifndef BDDMMA_H
#define BDDMMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BDDMMA_OK                 0
#define BDDMMA_ERR_INVALID_ARG   (-1) /* bad pointer, size, option or ILP data           */
#define BDDMMA_ERR_INFEASIBLE    (-2) /* some row (after presolve) admits no 0-1 point   */
#define BDDMMA_ERR_NO_MEMORY     (-3) /* workspace too small / host allocation failed   */
#define BDDMMA_ERR_NOT_CONVERGED (-4) /* rounding hit max_rounds; dual state unchanged   */
#define BDDMMA_ERR_HIP           (-5) /* a HIP runtime call failed                       */
#define BDDMMA_ERR_STATE         (-6) /* call out of order (e.g. run before bind)        */

typedef struct bddmma_solver bddmma_solver; /* opaque, owned by the library */

typedef struct {
    double   omega;        /* damping of the dual update (Sec. 3, parallel update), in (0,1]; 0.5 */
    double   rel_tol;      /* stop run_dual when |dLB|/max(1,|LB|) < rel_tol between two
                              consecutive iterations, checked every lb_every iterations; 0 = off */
    int32_t  lb_every;     /* stopping-test period in iterations (>= 1); 1 */
    int32_t  precision;    /* 32: FP32 multipliers / min-marginals, FP64 bound sums;
                              64: FP64 throughout.  32 */
    double   delta0;       /* Alg. 2 initial perturbation strength delta; 1.0 (Sec. 6) */
    double   alpha;        /* Alg. 2 growth factor of delta per round; 1.2 (Sec. 6) */
    int32_t  reopt_iters;  /* Alg. 1 iterations per rounding round; 5 */
    int32_t  max_rounds;   /* rounding rounds before BDDMMA_ERR_NOT_CONVERGED; 200 */
    double   tau;          /* |M| <= tau counts as a zero min-marginal difference in Alg. 2;
                              < 0 selects 0 for precision 64 and 1e-6*max(1,max|c|) for 32 */
    uint64_t seed;         /* counter-based random draws of Alg. 2; 0 */
    int32_t  sp_in_lds_max_nodes; /* subproblems with more nodes keep their shortest
                              paths in device memory instead of LDS; 0 = built-in limit,
                              -1 = never use LDS */
    int32_t  fast_path;    /* 1: tiles of 64 identical BDDs with <= 4 nodes per layer (and
                              width x layers <= 64), and tiles of different BDDs with <= 2
                              nodes per layer and <= 32 layers, are swept by
                              register-resident kernels, and variables with |J_i| <= 2
                              inside one tile are averaged in the sweep; 0: general
                              kernels and the averaging kernel only.  1 */
    int32_t  perturb_scale;/* Alg. 2 draws r uniformly from [-delta, delta] and adds r*delta
                              (0, magnitude up to delta^2) or draws r from [-1, 1] (1,
                              magnitude up to delta).  0 */
    int32_t  graph_sweeps; /* > 0: run_sweeps / run_dual replay blocks of this many sweeps
                              (rounded down to an even number, capped by the bound-history
                              capacity) from a captured HIP graph, which removes the
                              per-launch host cost of small problems; results are
                              identical to eager launches.  A solver captures the graph
                              in its second run of sweeps, or in a first run of at
                              least eight blocks, and replays it from then on.  Not
                              used while profiling.  0 = eager launches.  64 */
    int32_t  class_merge_kib; /* register-kernel tiles of a layer class are padded into the
                              next larger class of their kind while the padding costs at
                              most this many KiB of traffic per sweep (fewer launches);
                              0 = one launch per non-empty class.  32768 */
    int32_t  small_tiles;  /* problems of at most this many tiles sweep their tiles of 64
                              identical width-2 BDDs with the per-lane (mixed) register
                              kernel, so a sweep is one launch per layer class: the
                              launches of small problems are latency-bound.  0 = never.
                              2048 */
    int32_t  serial_mma;   /* 1: also build the tables of the serial min-marginal averaging
                              (bddmma_run_serial; BDDs in their own order plus a level
                              schedule, about 4 B per node and 40 B per pair more device
                              memory); 0: none.  0 */
    int32_t  termination;  /* termination step of Alg. 1, used for the certified bound, the
                              exported multipliers, rounding and the serial start:
                              0: lambda_i^j + omega M-bar_ij (the algorithm's last loop);
                              1: lambda_i^j + (omega/|J_i|) sum_k M-bar_ik (the text's
                              description: one more min-marginal averaging).  Both sum to c_i over J_i.  0 */
    int32_t  wide_min_width; /* BDDs outside the register classes whose widest layer has at
                              least this many nodes are swept by a group of wide_lanes
                              lanes each, spread over each layer's nodes, when their
                              distances fit in LDS; narrower ones run one BDD per lane.
                              0 = never.  4 */
    int32_t  wide_lanes;   /* lanes per BDD in that kernel: 16, 32 or 64 (a 64-lane wave
                              then holds 4, 2 or 1 BDDs of a tile; more lanes are used
                              when the BDDs' LDS regions would not fit one block).  32 */
    int32_t  fused_average;/* 1: when every variable that is not averaged inside one tile lies
                              in tiles of different BDDs on the register kernels (small
                              problems) and in at most five subproblems, the sweep averages
                              it itself from a per-variable copy of the previous
                              differences instead of a separate averaging launch per sweep
                              (same operations in the same order, so the same results);
                              0: always the averaging kernel.  1 */
    int32_t  persistent;   /* 1: when every tile is a mixed register tile of one layer class
                              and the averaging is fused (or not needed), run_sweeps /
                              run_dual run blocks of sweeps in one cooperative launch with a
                              grid-wide barrier between sweeps (same results) instead of
                              one launch per sweep or graph replay; 0: off.  0 */
    int32_t  reserved;     /* must be zero */
} bddmma_options;

typedef struct {
    int64_t n_vars, n_rows;       /* as loaded */
    int64_t n_bdds;               /* subproblems after presolve (one per kept row) */
    int64_t n_pairs;              /* (variable, subproblem) pairs */
    int64_t n_nodes;              /* non-terminal BDD nodes (arcs = 2 * n_nodes) */
    int64_t n_fixed;              /* variables fixed by presolve */
    int64_t n_free;               /* variables in no kept row */
    int64_t n_tiles;              /* 64-lane tiles of whole subproblems */
    int64_t n_slots;              /* padded pair slots on the device */
    int64_t max_layers, max_width;
    double  lb_offset;            /* constant of fixed / unconstrained variables */
    int64_t n_reg_tiles;          /* tiles swept by the register kernels (one topology) */
    int64_t n_reg_mixed_tiles;    /* tiles swept by the register kernels (per-lane topologies) */
    int64_t n_reg_launches;       /* register-kernel launches per sweep (non-empty classes) */
    int64_t n_wide_tiles;         /* tiles on the node-parallel kernel (layers of >= wide_min_width nodes) */
    int64_t node_words;           /* 32-bit node words on the device: tiles of one topology share
                                     one copy (plus the register path's copy), other tiles hold
                                     one word per node and lane */
    int64_t n_fused_vars;         /* variables averaged by the sweep from the per-variable copy
                                     (options.fused_average); 0 = the averaging kernel runs */
    int64_t persist_tiles;        /* tiles the persistent kernel sweeps when options.persistent
                                     is set (all of them), 0 when the problem does not qualify */
} bddmma_stats;

/* Fill *opt with the defaults listed above.  INVALID_ARG if opt is NULL. */
int bddmma_options_default(bddmma_options *opt);

/* Create an empty solver.  opt may be NULL (defaults).  INVALID_ARG on a bad
 * option (omega outside (0,1], precision not 32/64, lb_every < 1, ...). */
int bddmma_create(const bddmma_options *opt, bddmma_solver **out);

/* Release the solver and its host memory (never the bound device buffer). */
void bddmma_destroy(bddmma_solver *s);

/* Load an ILP in CSR form (host memory, copied).  Host-only: needs no GPU.
 *   costs[n_vars] (finite doubles); row_ptr[n_rows+1] (int64, non-decreasing,
 *   row_ptr[0] = 0); col[nnz] variable ids in [0, n_vars), distinct inside a
 *   row, any order; coef[nnz] int32 (zeros are dropped, Example "ILP":
 *   I_j = {i : a_ji != 0}); sense[n_rows] in {-1: <=, 0: ==, +1: >=};
 *   rhs[n_rows] int64.
 * Presolve fixes every variable that one row allows only one value for and
 * repeats until nothing changes; variables in no remaining row take
 * x_i = [c_i < 0].  Every remaining row is compiled to a reduced ordered BDD
 * in ascending variable order (Sec. 5, Defs. "BDD" and "Constraint Set
 * Correspondence") and packed into 64-lane tiles.
 * Errors: INVALID_ARG (bad CSR data, |coef| sums beyond int64, a BDD layer
 * wider than 65533 nodes), INFEASIBLE (some row cannot be satisfied),
 * STATE (already loaded). */
int bddmma_load_ilp(bddmma_solver *s, int64_t n_vars, const double *costs, int64_t n_rows,
                    const int64_t *row_ptr, const int32_t *col, const int32_t *coef,
                    const int8_t *sense, const int64_t *rhs);

/* Sizes of the loaded problem.  STATE before load. */
int bddmma_get_stats(const bddmma_solver *s, bddmma_stats *out);

/* Device bytes needed by bddmma_bind.  STATE before load. */
int bddmma_workspace_bytes(const bddmma_solver *s, size_t *bytes);

/* Bind caller-owned device memory (dev_ptr, 256-byte aligned, >= workspace
 * bytes) and a HIP stream (hipStream_t passed as void*, NULL = null stream).
 * Copies the packed problem to the device and initialises the dual state:
 * lambda_i^j = c_i / |J_i| and M-bar = 0 (Alg. 1 initialisation, Sec. 3).
 * The original rows (only the exact check of a rounded point reads them) are
 * copied by the first rounding call instead.
 * Errors: NO_MEMORY (bytes too small), INVALID_ARG (NULL / misaligned),
 * STATE (not loaded or already bound), HIP. */
int bddmma_bind(bddmma_solver *s, void *dev_ptr, size_t bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * bddmma_bind with the library's own workspace instead of caller memory.
 * The workspace is a static device array of BDDMMA_STATIC_WORKSPACE_BYTES
 * (64 MiB) that every GPU the library runs on holds until the process ends;
 * this call allocates nothing (no hipMalloc, no torch allocation).  It binds
 * the current HIP device's copy and the given stream, then behaves exactly as
 * bddmma_bind (same tables, same initial state, same results of every later
 * call).
 * All solvers bound this way on one GPU share that GPU's array, which keeps
 * the contents the last solver left: binding a solver hands the array over
 * to it, and every later call on the solver that held it before fails with
 * STATE.  Calls that overlap in time on one GPU (a bind while the previous
 * holder's work is still running, or two threads) race; order them.
 * Errors: NO_MEMORY (workspace bytes above BDDMMA_STATIC_WORKSPACE_BYTES;
 * checked before any device call), STATE (not loaded or already bound),
 * HIP. */
#define BDDMMA_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int bddmma_bind_static(bddmma_solver *s, void *hip_stream);

/* Re-initialise the dual state of a bound solver (lambda_i^j = c_i / |J_i|,
 * M-bar = 0, empty bound history, sweep counter 0) without re-copying the
 * problem.  STATE if not bound. */
int bddmma_reset(bddmma_solver *s);

/* Run n_iter iterations of Alg. 1 (forward sweep, averaging, backward sweep,
 * averaging; the deferred differences are refreshed after every sweep) from
 * the current state.  Records LB_free after every sweep.  Stops early on the
 * rel_tol test.  *iters_done (may be NULL) gets the iterations run.
 * Stream-ordered; synchronises only at the end (and at stopping checks). */
int bddmma_run_dual(bddmma_solver *s, int32_t n_iter, int32_t *iters_done);

/* Run n half-sweeps, alternating direction and starting with the direction
 * that follows the last sweep run (ascending first after bind), each followed
 * by the averaging and the LB_free record.  run_dual(k) equals
 * run_sweeps(2k) from an even sweep count. */
int bddmma_run_sweeps(bddmma_solver *s, int32_t n_sweeps);

/* Lower bounds of the current state (any pointer may be NULL):
 *   lb_free  = sum_j E^j(lambda^j) + omega * sum_ij min(M_ij, 0)  of the last sweep;
 *   lb_cert  = sum_j E^j(t'^j), the Lagrange dual (Sec. 3, problem (D)) at
 *              dual-feasible multipliers, computed in FP64 from the stored
 *              ones: t = lambda + omega M (the terminated multipliers; their
 *              sum over J_i equals c_i in exact arithmetic, Appendix, proof of
 *              Prop. 1), residual r_i = sum_j t_i^j - c_i (nonzero in FP32),
 *              and t'_i^j = t_i^j - r_i / |J_i|, so sum_j t'_i^j = c_i;
 *   max_residual = max_i |r_i|.
 * Both bounds include the presolve constant.  Synchronises. */
int bddmma_lower_bound(bddmma_solver *s, double *lb_free, double *lb_cert, double *max_residual);

/* LB_free after every sweep since bind (oldest first).  With out == NULL only
 * *n is set.  Otherwise writes min(*n_total, cap) values and sets *n_total. */
int bddmma_lb_history(const bddmma_solver *s, double *out, int64_t cap, int64_t *n_total);

/* Number of pairs, and their (variable, original row) in pair order. */
int bddmma_num_pairs(const bddmma_solver *s, int64_t *n_pairs);
int bddmma_get_pairs(const bddmma_solver *s, int32_t *pair_var, int32_t *pair_row);

/* Presolve result per variable: -1 free, 0 or 1 fixed.  fixed[n_vars]. */
int bddmma_get_fixed(const bddmma_solver *s, int8_t *fixed);

/* Feasible multipliers lambda_i^j + omega * M-bar_ij (the termination step of
 * Alg. 1; they sum to c_i over J_i) and M-bar itself, in pair order, as
 * doubles.  Either pointer may be NULL.  Does not change the state. */
int bddmma_get_multipliers(bddmma_solver *s, double *lambda_out, double *mm_out);

/* Raw solver state in pair order (lambda, M-bar) and per variable (the
 * averaged term a_i = omega/|J_i| * sum_k M-bar_ik, computed from M-bar).  Any
 * pointer may be NULL.  set_state converts lambda and M-bar to the working
 * precision and resumes from them; its avg argument is ignored because the
 * averaged terms are a function of M-bar. */
int bddmma_get_state(bddmma_solver *s, double *lambda, double *mm, double *avg);
int bddmma_set_state(bddmma_solver *s, const double *lambda, const double *mm, const double *avg);

/* Min-marginal differences M_ij = m^1 - m^0 (Sec. 3, defs. (MM), (MD)) of
 * every pair at the current multipliers, without changing the state.
 * mm_out[n_pairs] in pair order. */
int bddmma_min_marginals(bddmma_solver *s, double *mm_out);

/* Alg. 2 on a copy of the terminated multipliers; the dual state is restored
 * afterwards.  Each round that leaves no conflicting sign decodes x and walks
 * every BDD with it; variables of rejecting rows count as conflicts.  On
 * success x_out[n_vars] (0/1, presolved variables included) satisfies every
 * original row (checked again exactly in int64 on the device), *ub = c^T x,
 * *rounds = perturbation rounds used.  NOT_CONVERGED when max_rounds rounds did
 * not remove every conflict (x_out untouched).  Any output pointer except
 * x_out may be NULL. */
int bddmma_round_primal(bddmma_solver *s, uint8_t *x_out, double *ub, int32_t *rounds);

/* ---- Batches of independent instances (many small problems per launch) ----
 * A batch is k independent ILPs loaded as one block-diagonal ILP: instance k
 * owns the next inst_vars[k] variables and inst_rows[k] rows of the
 * concatenated CSR arrays (same formats as bddmma_load_ilp), and its rows may
 * reference its own variables only.  Tiles never mix instances, so every
 * sweep launch covers the tiles of all instances while each instance follows
 * exactly the trajectory it follows when loaded alone: multipliers, deferred
 * differences and rounded points are bitwise identical (bound sums agree to
 * the last few bits: their summation tree differs).  run_dual / run_sweeps /
 * lower_bound / lb_history act on the whole batch (bounds are sums over the
 * instances); the calls below report per instance.  INFEASIBLE when any
 * instance is.  Instance k's random draws in Alg. 2 use instance-local
 * variable indices and its zero threshold tau from its own costs. */
int bddmma_load_batch(bddmma_solver *s, int64_t n_inst, const int64_t *inst_vars, const int64_t *inst_rows,
                      int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
                      const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs);

/* Number of instances (1 after bddmma_load_ilp).  STATE before load. */
int bddmma_num_instances(const bddmma_solver *s, int64_t *n_inst);

/* Per-instance bounds (arrays of n_inst doubles, each may be NULL):
 * lb_free of the most recent recorded sweep (STATE if there is none since
 * bind / reset / load_state), lb_cert at the dual-feasible multipliers and
 * the largest multiplier residual, as bddmma_lower_bound computes them for the
 * whole problem.  With lb_cert and max_res both NULL the certificate pass and
 * the residuals are skipped.  Synchronises the stream. */
int bddmma_batch_bounds(bddmma_solver *s, double *lb_free, double *lb_cert, double *max_res);

/* Alg. 2 for every instance of the loaded problem (dual state restored
 * afterwards).  Rounds run while some instance has conflicts; each instance
 * closes, and its point is taken, in the first round in which it has no
 * conflict and all of its BDDs accept the decoded point: the round at which
 * Alg. 2 on that instance alone stops.  Per instance k (arrays of n_inst):
 * status[k] = OK, NOT_CONVERGED (max_rounds reached) or STATE (point
 * violates an original row); rounds[k] = round at which it closed (or the
 * last round); for OK instances ub[k] = objective and x_out[i] for its
 * variables (x_out has n_vars entries; other entries untouched).
 * bddmma_round_primal is this call followed by: OK only if every instance is
 * OK, *ub = sum of the instance objectives, *rounds = largest round. */
int bddmma_batch_round(bddmma_solver *s, uint8_t *x_out, double *ub, int32_t *rounds, int32_t *status);

/* ---- Serving pool: continuous batching of independent instances ----
 * Instances arrive at any time (bddmma_pool_submit); host worker threads
 * presolve, compile and pack each one alone (Sec. 5 construction, the tile
 * layout it has in a solver of its own).  Each bddmma_pool_step admits ready
 * instances in submission order while the resident batch fits its half of the
 * bound arena, their table images fit the image region and the batch holds
 * at most max_active instances (an admitted instance's tables are uploaded
 * once, as an image), re-assembles the batch on the device when its
 * membership changed (member images copied into the batch tables with their
 * index shifts, lambda and M of continuing members copied device to device),
 * runs the given number of
 * Alg. 1 iterations on all members at once (fewer when a member has fewer
 * left: no member runs past its n_iter), computes every member's lb_free
 * (as bddmma_batch_bounds; lb_cert and the residual for the members that
 * retire) and retires the members that reached their
 * iteration count or, with options.rel_tol > 0, whose lb_free moved by less
 * than rel_tol * max(1, |lb_free|) over the step.  A member follows exactly
 * the trajectory of a solver loaded with it alone and run for the same
 * number of iterations (exactly its n_iter unless it retires by rel_tol), so its
 * multipliers are bitwise those of the solo run.  Retiring copies the
 * member's terminated multipliers and M to the host (BDDMMA_POOL_KEEP_MULTIPLIERS)
 * and, with BDDMMA_POOL_ROUND, runs Alg. 2 for the retiring members in a
 * batch of their own (assembled from their images in the free arena half,
 * their state copied over), which gives each the point, UB and round count
 * it gets from bddmma_round_primal when solved alone.  Once
 * an instance is compiled, a worker thread uploads its image on a stream of
 * its own if image space is free, overlapping the running batch; admission
 * passes over an instance whose upload is still running (it joins at a
 * later step), so a step never waits for one.
 *
 * Threads: bddmma_pool_submit, _submit_loaded, _wait_compiled, _poll,
 * _result, _primal, _release and _get_counters may be called from any thread,
 * also while another thread is inside bddmma_pool_step.  Calls of
 * bddmma_pool_step must not overlap each other, bddmma_pool_bind comes before
 * the first step, and bddmma_pool_destroy must not overlap any call. */
typedef struct bddmma_pool bddmma_pool;

#define BDDMMA_POOL_QUEUED 0   /* submitted, host compilation pending or running */
#define BDDMMA_POOL_READY  1   /* compiled, waiting for admission */
#define BDDMMA_POOL_ACTIVE 2   /* member of the resident batch */
#define BDDMMA_POOL_DONE   3   /* retired; bounds and multipliers final */
#define BDDMMA_POOL_FAILED 4   /* compilation failed (error holds the code) or
                                  it can never fit (NO_MEMORY) */

typedef struct {
    int32_t state;           /* BDDMMA_POOL_* */
    int32_t error;           /* FAILED: INVALID_ARG / INFEASIBLE / NO_MEMORY */
    int32_t iters;           /* Alg. 1 iterations run so far */
    int32_t n_iter;          /* iterations requested at submission */
    int64_t n_vars, n_pairs; /* of the instance (valid from READY on) */
    int64_t steps;           /* pool steps it has been a member of */
    double lb_free;          /* after its last step (NaN before) */
    double lb_cert, max_residual;   /* at retirement (NaN before) */
    uint64_t workspace_bytes; /* device bytes of the instance alone */
    int32_t rounded;         /* 1 once Alg. 2 ran for it at retirement (BDDMMA_POOL_ROUND) */
    int32_t round_status;    /* then: OK, NOT_CONVERGED or STATE (point violates a row) */
    int32_t rounds;          /* rounds Alg. 2 used */
    int32_t reserved_;
    double ub;               /* c^T x of the rounded point (OK only) */
} bddmma_pool_info;

#define BDDMMA_POOL_KEEP_MULTIPLIERS 1   /* copy terminated multipliers to the host at retirement */
#define BDDMMA_POOL_ROUND            2   /* run Alg. 2 for members when they retire */

/* opt as for bddmma_create (rel_tol is applied per step as described above;
 * Alg. 2 uses its delta0, alpha, reopt_iters, max_rounds, tau, seed and
 * perturb_scale); max_active >= 1; host_threads = worker threads
 * (compilation, image uploads), 0 = min(8, cores); flags: a combination of
 * BDDMMA_POOL_KEEP_MULTIPLIERS and BDDMMA_POOL_ROUND (0: bounds only). */
int bddmma_pool_create(const bddmma_options *opt, int32_t max_active, int32_t host_threads, int32_t flags,
                       bddmma_pool **out);

/* Device arena owned by the caller (256-byte aligned, 8 MiB + 3 KiB at least) and
 * the stream every pool launch is ordered on.  8 MiB hold the copy
 * descriptors of an assembly; of the rest, a third holds member images and
 * two equal halves the resident batch and the next one while it is
 * assembled.  An instance fits when the workspace bytes of all members (each
 * as if alone, an upper bound on the batch's) stay within one half and its
 * image fits the free image space.  The pool also allocates a pinned host
 * buffer of 1 MiB (hipHostMalloc; freed by bddmma_pool_destroy) for its
 * batches' readbacks.  Once per pool. */
int bddmma_pool_bind(bddmma_pool *p, void *dev_ptr, size_t bytes, void *hip_stream);

/* Queue one ILP (arguments as bddmma_load_ilp, copied during the call) for
 * n_iter >= 1 iterations; *ticket identifies it until released.  Input errors
 * are reported by the state FAILED, not by this call. */
int bddmma_pool_submit(bddmma_pool *p, int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
                       const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs,
                       int32_t n_iter, int64_t *ticket);

/* Queue an instance the caller has already loaded alone (bddmma_load_ilp,
 * not bound) with the pool's options; the pool takes ownership of s, also on
 * failure (a batch or another precision ends FAILED with INVALID_ARG). */
int bddmma_pool_submit_loaded(bddmma_pool *p, bddmma_solver *s, int32_t n_iter, int64_t *ticket);

/* One step: admission, re-assembly, at most iters >= 1 Alg. 1 iterations
 * (the smallest count a member has left, if that is less), bounds,
 * retirement (see above).  *n_active = members after retirement, *n_retired =
 * instances retired by this step (either may be NULL).  With no member and no
 * ready instance the step returns at once.  Synchronises the stream. */
int bddmma_pool_step(bddmma_pool *p, int32_t iters, int32_t *n_active, int32_t *n_retired);

/* Block until no submitted instance is still being compiled or having its
 * image uploaded by a worker. */
int bddmma_pool_wait_compiled(bddmma_pool *p);

int bddmma_pool_poll(bddmma_pool *p, int64_t ticket, bddmma_pool_info *info);

/* DONE instances: terminated multipliers lambda + omega M and M in the
 * instance's own pair order (STATE unless the pool keeps multipliers), and
 * the pairs (variable, row) as bddmma_get_pairs gives them for the instance
 * alone; every pointer may be NULL, arrays hold n_pairs entries. */
int bddmma_pool_result(bddmma_pool *p, int64_t ticket, double *lambda, double *mm, int32_t *pair_var,
                       int32_t *pair_row);

/* Counters of the pool since creation: steps run, batch re-assemblies,
 * instances admitted and retired; wall milliseconds spent writing and
 * uploading the images of admitted instances, building the batch's host
 * tables (merge), assembling it on the device and carrying the
 * members' state (bind), running the iterations, computing bounds,
 * retiring members and rounding them; and the arena split: bytes of one
 * batch half, of the member-image region and of its free part. */
typedef struct {
    int64_t steps, assemblies, admitted, retired;
    double image_ms, merge_ms, bind_ms, run_ms, bounds_ms, retire_ms, round_ms;
    uint64_t batch_capacity, image_capacity, image_free;
} bddmma_pool_counters;
int bddmma_pool_get_counters(bddmma_pool *p, bddmma_pool_counters *out);

/* The rounded point x_out[n_vars] of a DONE instance whose Alg. 2 returned OK
 * (presolved variables included); STATE otherwise. */
int bddmma_pool_primal(bddmma_pool *p, int64_t ticket, uint8_t *x_out);

/* Forget a DONE or FAILED instance (STATE otherwise). */
int bddmma_pool_release(bddmma_pool *p, int64_t ticket);

void bddmma_pool_destroy(bddmma_pool *p);

/* Checkpoint of the dual state (multipliers, deferred differences, sweep
 * counter, bound history).  With buf == NULL sets *bytes to the
 * size needed.  load_state requires the same loaded problem and precision;
 * resuming from it is bitwise identical to not stopping. */
int bddmma_save_state(const bddmma_solver *s, void *buf, size_t *bytes);
int bddmma_load_state(bddmma_solver *s, const void *buf, size_t bytes);

/* Ablation of the deferred scheme: the serial min-marginal averaging it
 * replaces (Sec. 3, update (dual_update_serial)).  Needs options.serial_mma =
 * 1 (STATE otherwise).  Starts from the terminated multipliers lambda + omega
 * M-bar of the current state and runs n_iter iterations, each a sweep over
 * the variables in ascending and then in descending id order; for each
 * variable i the min-marginal differences M_ik of all subproblems k in J_i are
 * taken at the current multipliers and lambda_i^k <- (lambda_i^k - M_ik) +
 * (1/|J_i|) sum_k M_ik (ascending row order) before the next variable.  The
 * device runs the variables level by level (a variable's level follows its
 * predecessors in every subproblem containing it), one launch per level.
 * After every sweep sum_j E^j + constant is a lower bound; these bounds are
 * appended to the bound history and, when lb_hist is not NULL, written to
 * lb_hist[2 * n_iter].  Afterwards the state is the serial multipliers with
 * M-bar = 0, so lower_bound, round_primal and further run_dual calls continue
 * from them.  Synchronises the stream. */
int bddmma_run_serial(bddmma_solver *s, int32_t n_iter, double *lb_hist);

/* Per-kernel timing with HIP events recorded on the bound stream around the
 * sweeps of run_dual / run_sweeps.  enable = n > 0 starts a new collection
 * that brackets the forward and backward sweep of every n-th iteration (n = 1:
 * all of them); enable <= 0 stops collecting.  A sweep may be several launches
 * (one per tile class); its events bracket all of them.  Only sweeps are
 * bracketed, so BDDMMA_K_AVERAGE and BDDMMA_K_LB_REDUCE report no launches;
 * they are kept for ABI stability.  bddmma_kernel_time synchronises and
 * reports launches and total milliseconds. */
#define BDDMMA_K_SWEEP_FWD 0
#define BDDMMA_K_SWEEP_BWD 1
#define BDDMMA_K_AVERAGE   2
#define BDDMMA_K_LB_REDUCE 3
#define BDDMMA_K_COUNT     4
int bddmma_profile(bddmma_solver *s, int enable);
int bddmma_kernel_time(bddmma_solver *s, int kernel, int64_t *launches, double *total_ms);

/* Encoding of rows whose BDDs would be too wide (the paper leaves such rows to
 * additional encodings, Sec. 7).  Reads an ILP in the bddmma_load_ilp format
 * and writes an equivalent one in which every row whose partial sums can
 * take more than max_states values (min(2^k, sum |a| + 1) over its k nonzero
 * terms) is replaced by a binary adder network over auxiliary variables
 * appended after the original n_vars:
 *  - one complement variable per variable with a negative coefficient in
 *    such a row, with the row x + xbar = 1;
 *  - one equality row per bit column of the weights, summing the column's
 *    inputs and the previous column's carry bits into a sum bit and new
 *    carry bits;
 *  - one comparison row sum_k 2^k s_k (sense) B.
 * Every auxiliary value is determined by the original ones, so the feasible
 * points of the output, restricted to the first n_vars entries, are those of
 * the input.  Auxiliary variables cost 0; other rows are copied, normalised
 * (zero coefficients dropped, columns ascending).  Two calls: with costs_out
 * NULL only the sizes are written (n_vars_out, n_rows_out, nnz_out and
 * n_encoded = rows replaced); then every output array with those sizes.
 * INVALID_ARG on bad input, max_states < 2, or an encoded row whose weight
 * sum reaches 2^30.  All arrays are host memory owned by the caller. */
int bddmma_encode_rows(int64_t n_vars, const double *costs, int64_t n_rows, const int64_t *row_ptr,
                       const int32_t *col, const int32_t *coef, const int8_t *sense, const int64_t *rhs,
                       int64_t max_states, int64_t *n_vars_out, int64_t *n_rows_out, int64_t *nnz_out,
                       int64_t *n_encoded, double *costs_out, int64_t *row_ptr_out, int32_t *col_out,
                       int32_t *coef_out, int8_t *sense_out, int64_t *rhs_out);

/* Autotuner for the launch schedule: which kernels sweep which tiles
 * (register-resident fast path or general kernels; mixed per-lane tiles for
 * small problems; layer-class merging; shortest paths in LDS or device
 * memory; node-parallel kernel for wide BDDs; averaging inside the sweep) and
 * whether sweeps are replayed from HIP graphs.  The ILP (as for
 * bddmma_load_ilp) is compiled once; a greedy search then changes one option
 * at a time among fast_path {1, 0}, small_tiles {2048, 0, 2^30},
 * class_merge_kib {32768, 0, 4096, 262144}, sp_in_lds_max_nodes {0, -1},
 * wide_min_width {4, 0, 2, 16, 64}, wide_lanes {32, 16, 64}, fused_average
 * {1, 0}, graph_sweeps {64, 0} and persistent {0, 1}, starting from base
 * (NULL: defaults) and keeping a
 * change that is at least 2 % faster.  Each candidate is packed, bound to
 * dev_ptr (bytes of caller-owned device memory; candidates that need more are
 * skipped) and timed over `sweeps` (>= 2) Alg. 1 sweeps with HIP events on
 * hip_stream after as many warm-up sweeps (the faster of two timed runs).  The options only choose kernels
 * and layouts, never the arithmetic, so every candidate follows the same
 * trajectory.  *best gets the fastest options (other fields as in base),
 * *us_per_sweep (may be NULL) their time.  NO_MEMORY if no candidate fits. */
int bddmma_autotune(const bddmma_options *base, int64_t n_vars, const double *costs, int64_t n_rows,
                    const int64_t *row_ptr, const int32_t *col, const int32_t *coef, const int8_t *sense,
                    const int64_t *rhs, void *dev_ptr, size_t bytes, void *hip_stream, int32_t sweeps,
                    bddmma_options *best, double *us_per_sweep);

/* Bandwidth ceiling of the updating sweep (for the roofline of Alg. 1's
 * sweeps).  An updating sweep reads the multipliers and differences of each
 * slot and writes both back in place; this call moves the same bytes in the
 * same shape and computes nothing else: each wave owns 9 consecutive rows of
 * 64 elements of both device arrays a and b (n elements each), loads all of
 * them, then stores a_i + 1 and b_i * 2; blocks map to rows as the sweeps'
 * blocks map to tiles (consecutive rows on one XCD).  elem_bytes 4 (float) or 8
 * (double).  One call moves 4 * n * elem_bytes bytes; its time at a given n
 * bounds an updating sweep over arrays of that size on this device, including
 * the last-level cache's share when both arrays fit in it.  The arrays are
 * caller-owned device memory; asynchronous on hip_stream.  n = 0 does
 * nothing.  INVALID_ARG for n < 0, another elem_bytes, or a NULL array with
 * n > 0. */
int bddmma_stream_probe(void *a, void *b, int64_t n, int32_t elem_bytes, void *hip_stream);

const char *bddmma_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BDDMMA_H */
