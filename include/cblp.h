/*
 * cblp.h - C ABI of libcblp.so: full-batch SPFOM for the choice-based LP
 * (CBLP) under the generalized attraction model, on one AMD Instinct MI355X
 * (gfx950).
 *
 * The method is the parallel primal-dual iteration of the paper (Algorithm 3,
 * Section 4.3, with every segment sampled in every iteration): each segment
 * solves its inner assortment problem exactly against the current capacity
 * duals (Section 4.1, inner problem z_i), the segment sales are summed into
 * product and resource rows (A s), and the duals take the projected,
 * optionally regularised step of eq. 16.  Instances follow the problem
 * statement of Section 3 (segments with arrival rates, consideration sets,
 * nominal and shadow attractions of the GAM, revenues, capacities) and the
 * resource-matrix form of Section 5.2 (NRM with bundling).
 *
 * Notation used below: segments l in [L], products j in [n], resources
 * i in [m].  v is the nominal and w the shadow attraction (the paper writes
 * them the other way round), v0 the no-purchase attraction, lambda the
 * arrival rate, r the revenue, c the capacity, eta the capacity duals.
 *
 * Conventions for every entry point:
 *  - Pointers marked [dev] are device pointers on the current HIP device;
 *    [host] are host pointers.  Real arrays have the instance's dtype
 *    (CBLP_F32: float, CBLP_F64: double) unless typed explicitly.
 *  - stream is a hipStream_t passed as void*; NULL is the null stream.
 *    Work is enqueued on it; entry points that return host results
 *    synchronise that stream before returning.
 *  - Return value: CBLP_OK (0) or a CBLP_E* code; cblp_last_error() then
 *    describes the failure (thread-local, valid until the next call on the
 *    same thread).  No C++ exception crosses this boundary.
 *  - Results are bitwise reproducible for a given instance, dtype, params
 *    and device: product sales are summed in 64-bit fixed point and every
 *    floating-point reduction has a fixed order.
 */
#ifndef CBLP_H
#define CBLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CBLP_OK = 0,
    CBLP_EINVAL = 1,        /* bad size, pointer or value in the instance/params */
    CBLP_ENOMEM = 2,        /* device or host allocation failed */
    CBLP_EHIP = 3,          /* a HIP runtime call failed */
    CBLP_ENONFINITE = 4,    /* an iterate or reduction became NaN/Inf */
    CBLP_ENOTCONVERGED = 5  /* spfom_solve hit max_iters; stats are filled */
};

enum { CBLP_F32 = 1, CBLP_F64 = 2 };

/* Step rules for the dual update eta_i <- max(0, (1 - t_i mu) eta_i - t_i (c_i - u_i)). */
enum {
    SPFOM_STEP_CONST = 0,   /* t_i = tau_i: the constant step of Algorithm 2 (optionally
                               shrunk geometrically, see spfom_params.tau_decay) */
    SPFOM_STEP_POLYAK = 1   /* t_i = tau_i * gamma (D^t - LB) / sum_k tau_k g_k^2 */
};

/* Columns of one trace row (FP64), one row per iteration. */
enum {
    SPFOM_TR_DUAL = 0,      /* D^t = c . eta^{t-1} + sum_l lambda_l R*_l(eta^{t-1}) */
    SPFOM_TR_PRIMAL = 1,    /* P^t = sum_j r_j S^t_j, revenue of the best responses */
    SPFOM_TR_Z = 2,         /* sum_l lambda_l R*_l */
    SPFOM_TR_ETA2 = 3,      /* ||eta^{t-1}||^2, the duals the pass was taken at */
    SPFOM_TR_INFEAS = 4,    /* sum_i (u^t_i - c_i)^+ / sum_i c_i (the plain sum when sum c = 0) */
    SPFOM_TR_DBEST = 5,     /* min_{s<=t} D^s (upper bound on the LP optimum) */
    SPFOM_TR_LB = 6,        /* best certified feasible revenue (lower bound, see SPFOM_BOUND_*) */
    SPFOM_TR_GAP = 7,       /* (DBEST - LB) / |DBEST| */
    SPFOM_TR_STEP = 8,      /* step multiplier (1 for CONST) */
    SPFOM_TR_THETA = 9,     /* min_i min(1, c_i / ubar_i) at the last check */
    SPFOM_NTRACE = 10
};

/* Certified lower bounds (spfom_params.bound).  Both scale the primal
 * average of the current window (the window restarts at t = 1 and whenever t
 * doubles its start): offering segment l its averaged sales a fraction
 * theta_l of the time and the empty assortment otherwise keeps every
 * resource within capacity when theta_l <= c_i / ubar_i for each resource i
 * that a product of N_l uses, so sum_l theta_l pbar_l <= OPT.
 *   GLOBAL:  theta_l = min_i min(1, c_i / ubar_i) for every segment
 *   SEGMENT: theta_l = min over the resources of N_l (tighter; keeps a
 *            running FP64 revenue sum per segment, 8 bytes per segment, and
 *            takes one pass over the consideration sets at each check)
 * LB is the largest such bound over the checks so far. */
enum { SPFOM_BOUND_GLOBAL = 0, SPFOM_BOUND_SEGMENT = 1 };

typedef struct cblp_instance* cblp_t;

/* Iteration parameters (host struct). */
typedef struct {
    int32_t rule;           /* SPFOM_STEP_CONST or SPFOM_STEP_POLYAK */
    int32_t check_every;    /* K >= 1: certified lower bound refreshed every K iterations */
    double tau;             /* scalar tau_i when tau_vec is NULL (> 0) */
    const void* tau_vec;    /* [dev] optional per-resource tau_i [m], instance dtype, > 0 */
    double gamma;           /* Polyak multiplier (0, 2] */
    double mu;              /* regularisation mu >= 0 of eq. 15/16 (0: Algorithm 2) */
    double tol;             /* spfom_solve: stop when the certified gap <= tol */
    int64_t max_iters;      /* spfom_solve: iteration cap */
    int32_t bound;          /* SPFOM_BOUND_GLOBAL or SPFOM_BOUND_SEGMENT */
    double tau_decay;       /* CONST rule: the step is tau_i * tau_decay^k in iterations
                               k*decay_every+1 .. (k+1)*decay_every (counted from the
                               last reset); 0 or 1: constant.  In (0, 1]. */
    int64_t decay_every;    /* >= 1 when tau_decay is used */
} spfom_params;

/* Result summary (host struct, FP64). */
typedef struct {
    int64_t iters;          /* iterations since the last reset */
    double trace[SPFOM_NTRACE]; /* the last trace row */
    double seconds;         /* wall time of the call (spfom_solve only) */
    int32_t status;         /* CBLP_OK, CBLP_ENOTCONVERGED or CBLP_ENONFINITE */
} spfom_stats;

/*
 * cblp_create - validate an instance and build a solver handle.
 *
 * seg_ptr [dev] int64 [L+1]: CSR row pointers of the consideration sets N_l
 *         (Section 3); seg_ptr[0] = 0, non-decreasing.
 * prod_idx [dev] int32 [nnz]: product ids in [0, n), distinct within a row.
 * v, w [dev] [nnz]: nominal and shadow attraction per (segment, product);
 *         0 <= w < v, finite.  (GAM choice probability, Section 3.)
 * v0, lambda [dev] [L]: no-purchase attraction (> 0) and arrival rate (>= 0).
 * r [dev] [n]: revenues (finite).   c [dev] [m]: capacities (>= 0, finite).
 * a_ptr [dev] int64 [n+1], a_idx [dev] int32 [nnzA], a_val [dev] [nnzA]:
 *         resource matrix A by product (CSC), entries a_ij >= 0 (Section 5.2,
 *         eq. 26).  All three NULL means A = identity and requires m == n.
 * dtype: CBLP_F32 (iterate in FP32, reductions in FP64) or CBLP_F64.
 *
 * Ownership: the instance arrays are BORROWED - the caller keeps them alive
 * and unchanged until cblp_destroy.  The handle owns its workspace (about
 * 8 (L + 3n + 3m) bytes plus A's transpose).  Validation runs on the
 * device; any violation returns CBLP_EINVAL and no handle.
 */
int cblp_create(cblp_t* out, int64_t L, int64_t n, int64_t m,
                const int64_t* seg_ptr, const int32_t* prod_idx,
                const void* v, const void* w, const void* v0, const void* lambda,
                const void* r, const int64_t* a_ptr, const int32_t* a_idx,
                const void* a_val, const void* c, int32_t dtype, void* stream);

/* Release the handle and its workspace.  NULL is a no-op. */
void cblp_destroy(cblp_t h);

/* Clear the solver state (iteration count, Dbest, LB, averaging window). */
int spfom_reset(cblp_t h, void* stream);

/*
 * cblp_refresh - re-read new attractions and capacities into the handle: the
 * re-solves of a multi-period problem (Section 5.1), where each period's
 * customers bring their own preference weights and the remaining capacity
 * shrinks.  The caller has overwritten, in place, the v, w and c arrays it
 * gave cblp_create; the row pointers, product ids, v0, lambda, r and A must
 * be those of creation (the copies and fixed-point scales built from them
 * are kept).  The new values are validated as in cblp_create (CBLP_EINVAL
 * leaves the handle's copies inconsistent until a valid refresh), the
 * per-segment warm starts restart from 0 and the solver state is reset as by
 * spfom_reset.  A batch over the handle follows the refresh (it reads the
 * handle's buffers).  Synchronises the stream.
 */
int cblp_refresh(cblp_t h, void* stream);

/*
 * spfom_iterate - run `iters` SPFOM iterations from eta, continuing the
 * handle's solver state (Algorithm 3 with every segment sampled; dual step
 * of eq. 16).
 * eta [dev] [m], in/out: the duals eta^0 on entry, eta^iters on return.
 * trace [host] nullable, FP64 [iters x SPFOM_NTRACE]: one row per iteration.
 * out [host] nullable: summary of the last iteration.
 * If trace or out is non-NULL the call synchronises the stream.
 */
int spfom_iterate(cblp_t h, void* eta, const spfom_params* p, int64_t iters,
                  double* trace, spfom_stats* out, void* stream);

/*
 * spfom_solve - reset the state and iterate from eta until the certified
 * relative gap (Dbest - LB)/|Dbest| <= p->tol or p->max_iters iterations;
 * the gap is read back every p->check_every iterations.  Returns CBLP_OK on
 * convergence, CBLP_ENOTCONVERGED at the cap (out still filled).
 * eta [dev] [m] in/out: warm start (or zeros) in, final duals out.
 */
int spfom_solve(cblp_t h, void* eta, const spfom_params* p, spfom_stats* out, void* stream);

/*
 * spfom_minibatch - `iters` iterations of stochastic minibatch SPFOM
 * (Algorithm 2, Section 4.1; Algorithm 3 with k B < L, Section 4.3): the
 * segments batch[t*B .. t*B+B-1] of iteration t re-solve their inner
 * problems at the current duals, every other segment keeps the sales of the
 * last pass that solved it (0 before its first), and the duals take the step
 * of eq. 16 with the sales of ALL segments.  The per-segment sales persist in
 * the handle between calls (made on first use: 4 bytes per consideration-set
 * entry for CBLP_F32, 8 for CBLP_F64, plus 8 per product and 8 per segment)
 * and restart from 0 at spfom_reset.
 * eta [dev] [m] in/out.  p: rule CONST with constant tau (tau_decay 0 or 1);
 * bound and the certificate fields are not used.
 * batch [dev] int32 [iters x B]: caller segment ids, each in [0, L) and
 * distinct within its iteration; an id out of range or listed twice returns
 * CBLP_EINVAL and leaves the minibatch state undefined until spfom_reset.
 * 1 <= B <= L.
 * trace [host] nullable [iters x SPFOM_NTRACE]: PRIMAL (revenue of the kept
 * sales), ETA2, INFEAS (of the kept sales) and STEP; the other columns are 0
 * (a dual bound needs every segment at one eta: cblp_gap gives it).
 * Synchronises the stream.
 */
int spfom_minibatch(cblp_t h, void* eta, const spfom_params* p, const int32_t* batch, int64_t B,
                    int64_t iters, double* trace, void* stream);

/*
 * cblp_gap - one best-response pass at fixed eta [dev] [m] (no dual step, no
 * state change).  Fills out->trace with DUAL = D(eta), PRIMAL, Z, ETA2 and
 * INFEAS; the other columns are 0.  Synchronises the stream.
 */
int cblp_gap(cblp_t h, const void* eta, spfom_stats* out, void* stream);

/*
 * cblp_sales - best responses at fixed eta [dev] [m] (the per-segment inner
 * problem of Section 4.1 in its GAM form, solved exactly).
 * S_out [dev] double [n] nullable: product sales S_j = sum_l s_lj.
 * u_out [dev] double [m] nullable: resource usage u = A S.
 * seg_R_out [dev] [L] nullable, instance dtype: R*_l per segment.
 * s_out [dev] double [nnz] nullable: per-entry sales s_lj in the caller's CSR
 *         order (entry q of seg_ptr[l]..seg_ptr[l+1]); 0 for products outside
 *         the best response S*_l.  Each value is the one the library summed
 *         into S (a multiple of its fixed-point quantum), so S_j is exactly
 *         the sum of s_lj over l.
 * Synchronises the stream.
 */
int cblp_sales(cblp_t h, const void* eta, double* S_out, double* u_out, void* seg_R_out,
               double* s_out, void* stream);

/*
 * cblp_recover - the choice-based LP solution behind per-entry sales
 * (Section 4.4, the recovery lemma, in its GAM form).  y [dev] double [nnz]:
 * sales s_lj in the caller's CSR order that satisfy each segment's SBLP rows
 * (balance and scale) - a best response from cblp_sales, an average of
 * several, or the kept sales of minibatch iterations.  Each segment's
 * products are ordered by y_lj / v_lj, decreasing (ties by CSR position);
 * the recovered solution offers only the nested sets S_q of the first q
 * products, S_q a share of the time proportional to
 * (key_q - key_{q+1}) (v_l0 + sum_{N_l} w + sum_{S_q} (v - w)), which
 * reproduces y exactly.  (The lemma as printed leaves the no-purchase term
 * out of this sum; it is needed for the sales to come out as y.)
 * rank [dev] int32 [nnz]: position of each entry in its segment's order.
 * alpha [dev] double [nnz]: probability of offering the set of the entries
 *         ranked at or before this one.
 * alpha0 [dev] double [L]: probability of offering nothing.
 * A segment with lambda_l = 0 gets alpha 0 and alpha0 1.  Enqueued on the
 * stream, no synchronisation.
 */
int cblp_recover(cblp_t h, const double* y, int32_t* rank, double* alpha, double* alpha0,
                 void* stream);

/*
 * cblp_launch_info - the launch shape chosen at cblp_create: number of
 * segment-kernel blocks, number of LDS sales bins per block (products
 * [0, bins) are accumulated in LDS, the others by global atomics), how many
 * of them are 64-bit (products [0, bins64); the rest are 32-bit bins whose
 * wraps are carried to the global sums), the fixed-point fraction bits of the
 * sales accumulators, the segment kernel (0: FP32 three-part kernel with all
 * prices in LDS; 1, 2: the same with the popular head of the prices in LDS,
 * 16- or 32-bit product ids; 3, 4: FP64 8-lane kernel, 16- or 32-bit ids)
 * and the places of its slot-major copy of the consideration sets (each row
 * padded to its wave-tile's longest, in units of entries).  Each [host]
 * pointer is nullable.
 */
int cblp_launch_info(cblp_t h, int32_t* seg_grid, int32_t* bins, int32_t* bins64,
                     int32_t* fx_bits, int32_t* kernel, int64_t* slot_entries);

/*
 * cblp_timing - enable (1) or disable (0) per-launch timing: while enabled,
 * every launch of the segment kernel (id 0) and every dual phase (id 1: the
 * sales fold, reductions and dual-step kernels of one iteration) is
 * bracketed by a pair of HIP events on the launch stream.  Enabling
 * clears earlier records.
 * cblp_timing_read - synchronise the stream and return the summed kernel
 * times ms[2] (milliseconds) and launch counts launches[2] ([host] arrays
 * indexed by kernel id) recorded since the last read, then clear them.
 */
int cblp_timing(cblp_t h, int32_t enable);
int cblp_timing_read(cblp_t h, double* ms, int64_t* launches, void* stream);

/* ------------------------------------------------------------------ batches
 * Many independent instances advanced together: the re-solves of the periods
 * of a multi-period problem (Section 5.1), each with its own remaining
 * capacities.  One iteration of every active instance is one persistent
 * segment launch (a shared work list of tile ranges) plus two dual-phase
 * launches; the duals and trace rows equal those of the instances' own
 * spfom_iterate bit for bit (integer sales and Z sums, the single path's
 * grouping of the FP64 partials).  Identity resource matrix only.
 */
typedef struct cblp_batch* cblp_batch_t;

/* Build a batch over count handles (same dtype, A = identity).  The batch
 * uses the handles' device buffers: do not use a handle on its own while its
 * batch is in use, and destroy the batch before its handles. */
int cblp_batch_create(cblp_batch_t* out, int32_t count, const cblp_t* handles, void* stream);
void cblp_batch_destroy(cblp_batch_t b);

/* iters iterations of every instance from etas[q] ([dev] [m_q], in/out),
 * continuing the batch's per-instance solver state.  tau_vecs nullable, or
 * per-instance [dev] tau vectors (NULL entries use p->tau).  rows [host]
 * nullable: the last trace row of each instance, [count x SPFOM_NTRACE]. */
int spfom_batch_iterate(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                        const spfom_params* p, int64_t iters, double* rows, void* stream);

/* Reset every instance and iterate until each one's certified gap <= p->tol
 * or p->max_iters: p->check_every iterations are captured once in a hipGraph
 * and replayed; converged instances drop out of the work list.  As in
 * spfom_solve, the last block is cut to the iterations left below max_iters
 * (run without the graph), and the gap is tested only after a whole block of
 * check_every iterations.  p->bound must be SPFOM_BOUND_GLOBAL; the constant
 * step may decay (p->tau_decay, p->decay_every) as in spfom_iterate, by each
 * instance's own iteration count.  outs [host]
 * [count] receives each instance's iterations, last trace row, elapsed
 * seconds and status.  Returns CBLP_OK if every instance converged. */
int spfom_batch_solve(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                      const spfom_params* p, spfom_stats* outs, void* stream);

/* Autotune the batched segment pass: every usable kernel variant (copy
 * layout and group widths, price placement) with 2, 4, 8 and 16 work items
 * per segment block, timing iters iterations of each pair on this batch, and
 * keep the fastest.  The duals in etas change, the solver state is reset
 * afterwards and the handles' per-segment warm starts are restored (so a
 * later solve follows the same iterates as on untouched handles).  chosen
 * [host] nullable receives the variant kept.  CBLP_ENOMEM if the copy of the
 * warm starts (4 or 8 bytes per segment) cannot be allocated. */
int cblp_batch_tune(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                    const spfom_params* p, int32_t iters, int32_t* chosen, void* stream);

/* cblp_batch_tune through a cache file (cache_path [host], a text file of
 * lines "key variant items_per_block", appended to): the key is the GPU's
 * architecture name, the dtype, the instance count and the power-of-two
 * buckets of the total entries, total segments and largest product count.
 * A hit applies the stored choice without timing; a miss tunes and appends
 * the result.  chosen, items_per_block [host] nullable. */
int cblp_batch_tune_cached(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                           const spfom_params* p, int32_t iters, const char* cache_path,
                           int32_t* chosen, int32_t* items_per_block, void* stream);

/* Work items, persistent grid and kernel variant of the batch ([host], nullable). */
int cblp_batch_info(cblp_batch_t b, int32_t* items, int32_t* grid, int32_t* variant);

/* Select the batched segment-kernel variant (one of the autotuner's
 * candidates, 0-3; every variant gives the same duals bit for bit).
 * CBLP_EINVAL if the variant cannot run on this batch. */
int cblp_batch_select(cblp_batch_t b, int32_t variant);

/* How spfom_batch_solve runs: mode 1 solves every instance in one launch,
 * one persistent 1024-thread block per instance that runs its iterations,
 * folds and gap tests itself (the same bits as the per-iteration launches;
 * each instance stops at the same iteration); 0 always launches the three
 * kernels of each iteration (replayed from the graph); -1 (the default)
 * takes the one-launch form when every instance has at most 2^18 entries.
 * The one-launch form keeps each instance's product state in LDS for the
 * whole solve; it needs at most 2048 products per instance, every product in
 * a 64-bit LDS bin, the handles' slot-major copies with one product id type,
 * and the largest instance's bins, prices, product state and fold partials
 * within one block's LDS: CBLP_EINVAL for mode 1 when the batch does not
 * meet that (mode -1 then keeps the per-iteration launches). */
int cblp_batch_persistent(cblp_batch_t b, int32_t mode);

/* Instances that take part in the batch's next spfom_batch_iterate and
 * spfom_batch_solve calls: take_part [host] [count], nonzero = takes part;
 * NULL = every instance (the state after cblp_batch_create).  The others
 * keep their duals untouched; a solve still resets their state and reports
 * them with iters 0 and status CBLP_OK. */
int cblp_batch_mask(cblp_batch_t b, const int32_t* take_part);

/* ------------------------------------------------- bid-price policy simulation
 * The global optimisation (GO) policy of Section 5.1 with bid-price control,
 * on the synthetic market of Figure 4, for `runs` independent runs at once.
 * In every batch (period) t of T and run: products out of stock leave the
 * offer and the LP; if at most K remain they are all offered; otherwise the batch's
 * sales-based LP is re-solved by SPFOM from the previous batch's duals and
 * the bid-price rule offers the products with r_j - eta_j >= 0, cut to the K
 * largest margins (ties: lower j).  The batch's customers then choose under
 * the basic attraction model (no-purchase attraction 1): customer i with
 * uniform u_i buys the first offered product (ascending j) whose running
 * preference sum exceeds u_i (1 + sum of the offered preferences), or
 * nothing; product j sells min(its demand, its stock).  The batch LP has the
 * batch's customers as segments (arrival rate 1, every product in the
 * consideration set, preference = nominal attraction, no shadow attraction)
 * and capacities c_j = stock_j / (T - t) (t counted from 0): the remaining
 * stock spread evenly over the batches left.  Decisions are taken in FP64
 * from the dtype's values; results are exact and reproducible.
 *
 * Layouts (row-major): r, eta, tau, c [runs x n] (dtype); inv [runs x n]
 * int64 (stock, in/out); prefs [T x runs x N x n] (dtype); u [T x runs x N]
 * double in [0, 1); offers [T x runs x K] int32 (ascending, -1 padded);
 * sales [T x runs x n] int64; revenue [T x runs] double.  n <= 8192,
 * 1 <= K <= 64.
 */

/* Capacities, dual steps and starting duals of the current batch's LP, for
 * every run: c_j = inv_j / periods_left and tau_j = tau0 max_k r_k / c_j
 * (zero capacity: the smallest positive one's step, or capacity 1 if none),
 * each rounded once to dtype (tau from the rounded c); a product out of
 * stock leaves the LP - its dual is raised to at least r_j, where its
 * margin r_j - eta_j <= 0 keeps it out of every segment's assortment (zero
 * sales at zero capacity, no term in c . eta), and the step leaves it there.
 * [dev] inv, r in; c, tau out; eta (nullable) in/out. */
int gosim_lp_inputs(int32_t runs, int64_t n, const int64_t* inv, int64_t periods_left,
                    double tau0, const void* r, void* c, void* tau, void* eta, int32_t dtype,
                    void* stream);

/* One batch of every run at the given duals: the offer, the N customers'
 * choices, sales and the stock left.  [dev] eta, r, prefs [runs x N x n]
 * (this batch's), u [runs x N] in; inv in/out; offer [runs x K], sales
 * [runs x n], revenue [runs] out; in_stock [runs] (nullable) out: products
 * still in stock afterwards. */
int gosim_period(int32_t runs, int64_t N, int64_t n, int32_t K, const void* eta, const void* r,
                 const void* prefs, const double* u, int64_t* inv, int32_t* offer,
                 int64_t* sales, double* revenue, int32_t* in_stock, int32_t dtype, void* stream);

/* T batches of the GO policy over the batch b of `runs` handles.  Handle q
 * holds run q's batch LP: N segments listing products 0..n-1 in order,
 * w = 0, v0 = lambda = 1, A = I, with its v, c and r at offset q of one
 * [runs x N x n], [runs x n] and [runs x n] array each (r: the r argument);
 * its v and c arrays are the simulation's work buffers (overwritten).
 * Per batch: gosim_lp_inputs into the handles' c and tau_work [dev]
 * [runs x n], this batch's preferences copied into the handles' v,
 * cblp_refresh of the runs with more than K products in stock, one
 * spfom_batch_solve of those runs (p: tol, max_iters, check_every, step
 * rule; tau_vec unused - each run steps by its tau_work row; an instance
 * that does not reach tol keeps its last duals) from eta [dev] [runs x n]
 * (in/out: the duals carried from batch to batch), then gosim_period.
 * lp_iters, lp_gap [host] [T x runs] (nullable): SPFOM iterations and the
 * last certified gap per batch and run (0: no LP solved).  The batch's
 * participation mask is cleared on return. */
int gosim_run(cblp_batch_t b, int32_t periods, int32_t K, const void* prefs, const double* u,
              const void* r, int64_t* inv, void* eta, void* tau_work, const spfom_params* p,
              double tau0, int32_t* offers, int64_t* sales, double* revenue, int64_t* lp_iters,
              double* lp_gap, void* stream);

/* ---------------------------------------------------------- learned warm start
 * A small network maps four features of each dual's row (a product for the
 * identity resource matrix, m = n; a resource - a base product of the
 * bundles of Section 5.2 - otherwise) to a starting capacity dual for
 * spfom_solve.  Not part of the paper's method, which leaves learned starts
 * to future work (Section 7); it only changes the initial duals eta^0 that
 * SPFOM takes as an input (Algorithm 2, Section 4.1; its parallel form
 * Algorithm 3, Section 4.3), so every certificate (the dual bound D and the
 * averaged-primal lower bound) keeps its meaning.
 *
 * Per product j: d_j = sum_l lambda_l v_lj / (v_l0 + sum_{i in N_l} v_li),
 * the sales of j when every segment is offered its whole consideration set;
 * mass_j = sum_l v_lj; deg_j = number of segments whose set holds j.  For a
 * resource i these become D_i = sum_j a_ij d_j, M_i = sum_j a_ij mass_j and
 * G_i = sum_j deg_j over the products j with an entry in row i of A.  The
 * scale of a dual is r_j (A = I) or s_i = max r_j / a_ij over the entries of
 * row i with a_ij > 0 (0 if none): the largest revenue per unit of the
 * resource.  Features, written as X[i*4 + k] (FP32, [m x 4] row-major):
 *   k=0  min(c_i / D_i, 4)  (4 where D_i = 0)
 *   k=1  s_i / max_k s_k    (0 if no scale is positive)
 *   k=2  log1p(M_i * m / L)
 *   k=3  log1p(G_i * m / L)
 * The product sums are taken in 64-bit fixed point (then FP64 over each
 * resource's entries in a fixed order), so X is bitwise reproducible.
 *
 * Network: y = w3 . GELU(W2^T GELU(W1^T x + b1) + b2) + b3 with hidden width
 * 256, GELU(z) = z Phi(z) (exact, erf form).  Parameters are one FP32 vector
 * of wsnet_num_params() = 67329 entries laid out as W1 [4 x 256] (row k holds
 * the weights of input k), b1 [256], W2 [256 x 256] (row i = hidden unit i of
 * the first layer), b2 [256], w3 [256], b3 [1].  Every weight is used rounded
 * to BF16 (nearest even); the second layer multiplies BF16(h1) by BF16(W2) on
 * the matrix cores (16x16x32 BF16) with FP32 accumulation; everything else is
 * FP32.  The predicted dual is eta_i = max(0, y_i) * scale_i.
 *
 * Training: mean squared error over rows, L = (1/rows) sum (y - t)^2, minimised
 * by Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 parameters.  Backward
 * uses BF16(dZ2) against BF16(H1) and BF16(W2) on the matrix cores.  A step is
 * two launches: blocks of 16 waves take 32-row chunks through forward, loss
 * and backward and write per-block gradient sums (FP32 over their rows), which
 * the second launch adds in block order in FP64 before the Adam update.
 *
 * All pointers named X, Y, y, grads, eta are [dev].  The net owns its
 * parameters and workspaces it grows on demand (calls on one net must not
 * overlap).
 */
typedef struct wsnet* wsnet_t;

int64_t wsnet_num_params(void);

/* New network with He-normal weights drawn from seed, zero biases. */
int wsnet_create(wsnet_t* out, uint64_t seed, void* stream);
void wsnet_destroy(wsnet_t w);

/* get [host] nullable receives the parameters; set [host] nullable replaces
 * them (and clears the Adam state).  Synchronises the stream. */
int wsnet_params(wsnet_t w, float* get, const float* set, void* stream);

/* Features of the instance behind h into X [dev] [m x 4].  Synchronises. */
int wsnet_features(cblp_t h, float* X, void* stream);

/* y [dev] [rows] = network(X [dev] [rows x 4]). */
int wsnet_forward(wsnet_t w, const float* X, int64_t rows, float* y, void* stream);

/* Loss (host, nullable) and gradient grads [dev] [num_params] (nullable) of
 * the mean squared error against targets Y [dev] [rows]; no update. */
int wsnet_gradients(wsnet_t w, const float* X, const float* Y, int64_t rows, float* grads,
                    double* loss, void* stream);

/* One Adam step of rate lr on the batch (X, Y); loss [host] nullable is the
 * batch loss before the step (synchronises only when loss is requested). */
int wsnet_train_step(wsnet_t w, const float* X, const float* Y, int64_t rows, float lr,
                     double* loss, void* stream);

/* epochs passes of Adam over (X [dev] [rows x 4], Y [dev] [rows]) in
 * minibatches of batch rows (the last one smaller), each epoch in a fresh
 * random order drawn on the host from seed (mt19937_64, Fisher-Yates); each
 * minibatch takes one wsnet_train_step.  losses [host] [epochs] nullable
 * receives each epoch's mean squared error, the batch losses before their
 * steps.  Synchronises once per epoch. */
int wsnet_train_epochs(wsnet_t w, const float* X, const float* Y, int64_t rows, int64_t batch,
                       int32_t epochs, float lr, uint64_t seed, double* losses, void* stream);

/* Training targets of the instance behind h: Y [dev] [m] = eta_i / scale_i,
 * 0 where scale_i <= 0 (eta [dev] [m], h's dtype). */
int wsnet_targets(cblp_t h, const void* eta, float* Y, void* stream);

/* Predicted duals of the instance behind h into eta [dev] [m] (h's dtype). */
int wsnet_predict(wsnet_t w, cblp_t h, void* eta, void* stream);

/* The warm start with its cold fallback: predict eta as wsnet_predict does,
 * then keep the prediction only if its dual bound D(eta) is below D(0) (the
 * dual bound of the cold start); otherwise eta is set to 0.  used [host]
 * nullable receives 1 if the prediction was kept, 0 otherwise; d_pred and
 * d_zero [host] nullable receive the two bounds.  Leaves the handle's solver
 * state as it found it.  Synchronises the stream. */
int wsnet_start(wsnet_t w, cblp_t h, void* eta, int32_t* used, double* d_pred, double* d_zero,
                void* stream);

/* ------------------------------------------------------ without allocation
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * cblp_gap_static - cblp_gap and cblp_sales' product sales for an instance
 * given by its arrays (cblp_create's arguments and their rules) instead of a
 * handle: one best-response pass at eta [dev] [m].  Allocates nothing: every
 * intermediate (prices, 64-bit sales sums, partial sums) lives in a static
 * 8 MiB device array of the library, one per GPU, found once per device.
 * S_out [dev] double [n] nullable: product sales S_j (the same bits as
 *         cblp_sales' S for the same instance and eta).
 * bounds [dev] double [2]: D(eta) = c . eta + sum_l lambda_l R*_l and
 *         P = r . S; NaN when the data break cblp_create's index rules or
 *         the arrival rates are too large for the fixed-point sums (the
 *         call itself does not validate them otherwise).
 * CBLP_EINVAL when n or m exceeds cblp_gap_static_max_products() (about
 * 490,000) or an argument is NULL.  Enqueued on the stream; no
 * synchronisation, no copy to the host, no memset (capturable).  Calls on
 * one GPU share the static array: calls that overlap on one GPU (different
 * streams or threads) race and must be ordered by the caller. */
int cblp_gap_static(int64_t L, int64_t n, int64_t m, const int64_t* seg_ptr,
                    const int32_t* prod_idx, const void* v, const void* w, const void* v0,
                    const void* lambda, const void* r, const int64_t* a_ptr,
                    const int32_t* a_idx, const void* a_val, const void* c, int32_t dtype,
                    const void* eta, double* S_out, double* bounds, void* stream);

/* The largest n (and m) cblp_gap_static accepts. */
int64_t cblp_gap_static_max_products(void);

/* Describe the last failure on this thread ("" if none). */
const char* cblp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CBLP_H */
