/*
 * dope.h — C ABI of the MI355X (gfx950) DOPE library.
 *
 * DOPE (Dolz, Ben Ayed, Desrosiers, "DOPE: Distributed Optimization for Pairwise Energies") minimises a binary
 * pairwise energy (the paper's Eq. 1)
 *
 *     E(y) = sum_i u_i y_i + lambda * sum_{edges (i,j)} w_ij |y_i - y_j|,        y in {0,1}^n,
 *
 * by splitting the grid into overlapping blocks (Sec. 2), rewriting the energy as a sum of per-block problems
 * coupled through a relaxed global y (Theorem 1, Eq. 5), and running the ADMM loop of Algorithm 1: every block
 * solves its multiplier-augmented binary problem (Eq. 8) in parallel, then the consensus y (Eq. 10) and the
 * multipliers a_k (Eq. 11) are updated, and mu is multiplied by mu_fact.
 *
 * Arithmetic is exact integer fixed point, so results are bit-identical run to run:
 *   * y and a are Q16.16 (Y = 2^16 y, A = 2^16 a); mu is an integer M in input-energy units; lambda = lambda_q8/256.
 *   * Block k solves, scaled by 2^14,
 *       min_{x in {0,1}^|block|}  sum_i Ut_i x_i + sum_{(i,j) in block} c_ij |x_i - x_j|,
 *       Ut_i = u_i 2^14 / q_i + floor( (lambda_q8 G_i + 2^14 M (A_k,i - Y_i + 2^15)) / 2^16 ),
 *       G_i  = sum_{j in N(i)} w_ij (64 / (q_i q_j)) (q_j - [j in block k]) (Y_i - Y_j),
 *       c_ij = lambda_q8 w_ij 64 / (q_i q_j),
 *     where q_i is the number of blocks containing pixel i (Proposition 1).  The returned block labelling is the
 *     unique minimal minimiser (label 1 = source side of the minimal minimum cut) for the max-flow solver and
 *     the smallest-code minimiser (bit p = local pixel p) for the exhaustive solver.
 *   * Y_m <- floor( (M S_m - 4 Hc_m) / (M q_m) ),  S_m = sum_{k containing m} (2^16 yhat_k,m + A_k,m),
 *     Hc_m = sum_{k containing m} yhat_k,m sum_{j in N(m)} c_mj (q_j - [j in k])
 *            - sum_{j in N(m)} sum_{k containing j} (q_m - [m in k]) c_jm yhat_k,j      (Eq. 10)
 *   * A_k,i <- A_k,i + 2^16 yhat_k,i - Y_i                                               (Eq. 11)
 *   * residual r_k = sum_{i in block k} (2^16 yhat_k,i - Y_i)^2; converged when max_k r_k <= eps_q16^2
 *     (the stopping rule of Algorithm 1); overflow when any |Y| or |A| >= 2^22.
 *   * M <- min(floor(M mu_fact_num / mu_fact_den), 2^24 - 1).
 *   * Output labels l_i = [Y_i > 2^15]; energy E_q = 256 sum u_i l_i + lambda_q8 sum_edges w_ij |l_i - l_j|.
 *
 * Layout: raster order, x fastest: i = x + W (y + H z).  Blocks: per axis of length N with block edge B and
 * overlap o (0 <= o <= B/2): stride s = B - o, count 1 + max(0, ceil((N - B)/s)), block t covers
 * [t s, min(t s + B, N)); B <= 0 or B >= N means one block along that axis.  Block order is x-fastest over the
 * block grid; inside a block, local raster order is x-fastest.  Per-block vectors (A, yhat) are block-major,
 * concatenated in block order.
 *
 * Conventions: every call returns a dope_status; no exception crosses the ABI.  A failed call leaves the
 * state unchanged, except DOPE_EOVERFLOW and DOPE_ESOLVER, which stop the loop with the state of the failing
 * iteration.  A context is not thread-safe; separate contexts (also used from different threads) are
 * independent.  Work is ordered on the context's HIP stream.  A call that returns results to the host returns
 * once those results are complete; it does not always leave the stream idle: dope_iterate and dope_solve return
 * as soon as the loop-control kernel of their last iteration has published the loop state to the host, while
 * that kernel may still be finishing on the stream.  Work on other streams that needs the results must wait on
 * the context's stream (an event recorded on it after the call), as for any stream-ordered producer.
 */
#ifndef DOPE_H
#define DOPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dope_ctx dope_ctx;

typedef enum {
    DOPE_OK = 0,
    DOPE_EINVAL = -1,          /* bad argument, shape, or nonzero weight on an off-grid edge            */
    DOPE_ENOMEM = -2,          /* device allocation failed or bound workspace too small                 */
    DOPE_EDEVICE = -3,         /* a HIP runtime call failed                                              */
    DOPE_ENOTSUBMODULAR = -4,  /* some w_ij < 0 with the max-flow solver (footnote on submodularity)      */
    DOPE_EOVERFLOW = -5,       /* |Y| or |A| reached 2^22 (mu too small); state frozen at that iteration */
    DOPE_ESOLVER = -6,         /* a block max-flow exceeded its round limit (watchdog)                   */
    DOPE_ESTATE = -7,          /* call out of order (e.g. iterate before set_energy)                     */
    DOPE_EBUSY = -8            /* serving: admission budget exhausted                                    */
} dope_status;

/* Block sub-problem solvers (Eq. 8):
 *   MAXFLOW     submodular blocks (w >= 0): push-relabel max preflow in LDS, minimal minimum cut;
 *   EXHAUSTIVE  blocks of at most 16 pixels, any sign of w: all labellings, smallest-code minimiser;
 *   LSATR       non-submodular blocks of any size that fit the LDS (4-, 8- and 6-connected stencils): the
 *               trust-region local submodular approximation of Gorelick et al. (the optimiser the paper distributes
 *               in its curvature experiment, Sec. 3.3): from x_i = [U_i < 0], each step linearises the terms with
 *               c_ij < 0 at the current labelling x~ (U_i += c_ij (1 - 2 x~_j)), adds the trust region
 *               lam (1 - 2 x~_i) to U_i and takes the minimal minimum cut of the rest; the candidate replaces x~ when
 *               the actual reduction R > 0 and 4 R >= P (P: the reduction the approximation predicts), with
 *               4 R >= 3 P also lowering lam's level and a rejection raising it (lam = 0 at level -1, 2^14 10^k at
 *               level k); it stops when the candidate is x~, the level passes 4, or after 32 steps.  Deterministic
 *               integer arithmetic; a local method (not always the block's minimum).
 *   AUTO        MAXFLOW when the weights allow, else EXHAUSTIVE for blocks of at most 16 pixels. */
enum { DOPE_SOLVER_AUTO = 0, DOPE_SOLVER_MAXFLOW = 1, DOPE_SOLVER_EXHAUSTIVE = 2, DOPE_SOLVER_LSATR = 3 };
enum { DOPE_MEM_HOST = 0, DOPE_MEM_DEVICE = 1 };

typedef struct {
    int32_t ndim;              /* 2 or 3                                                                  */
    int32_t dims[3];           /* W, H, D (D = 1 in 2D)                                                  */
    int32_t connectivity;      /* 4, 8, 24 (5x5 square), 48 (7x7 square) or 80 (9x9 square) in 2D;    */
                               /* 6, 32, 122 or 256 (balls of radius 2, 3 and 4) in 3D                   */
    int32_t block[3];          /* block edge B per axis                                                  */
    int32_t overlap[3];        /* overlap o per axis; B - o must be at least the stencil radius (2 for  */
                               /* connectivity 24 and 32, 3 for 48 and 122, 4 for 80 and 256) on every */
                               /* axis                                                                    */
                               /* with more than one block                                               */
    int64_t mu0;               /* initial mu, 1 <= mu0 <= 2^24 - 1, input-energy units                   */
    int32_t mu_fact_num;       /* mu_fact = num / den (default 21 / 20)                                   */
    int32_t mu_fact_den;
    int32_t eps_q16;           /* epsilon of the stopping rule, Q16.16                                   */
    int32_t max_iter;          /* iteration cap for dope_solve                                           */
    int32_t solver;            /* DOPE_SOLVER_*                                                          */
    void *stream;              /* hipStream_t to order work on; NULL = the library creates its own       */
} dope_params;

typedef struct {
    int32_t iters_done;        /* t: iterations completed since the last reset                           */
    int32_t converged;         /* 1 if the last completed iteration met the stopping rule                */
    int64_t max_resid2;        /* max_k r_k of the last completed iteration (Q32.32)                     */
    int64_t mu;                /* M for the next iteration                                               */
} dope_info;

/* Validate p and create a context (no device memory is taken until dope_set_energy or a bound workspace).
 * Blocks whose max-flow state exceeds the 160 KiB of LDS (such as the even partitions into 32 to 128 blocks of
 * the 2D experiments, Sec. 3.1) are solved with that state in the workspace (the block-solve kernel is the same;
 * one workgroup per block, of 1024 threads for the 4-, 8- and 6-connected stencils and 256 for the wider ones,
 * with at most 16 pixels per thread: 16384 or 4096 per block), one image at a time (a batch or a server rejects
 * them).  Returns EINVAL for unsupported shapes (a larger block, bad overlap, bad stencil, more than 2^30 - 1
 * pixels in 2D or 2^29 - 1 voxels in 3D, block sizes summing to 2^30 or more). */
dope_status dope_create(const dope_params *p, dope_ctx **out);

/* Load the energy (Eq. 1) and reset the ADMM state of Algorithm 1's initialisation: Y = 2^15, A = 0,
 * M = mu0, t = 0.
 *   u: int32[n]; w: int32[h * n], offset-major over the half-stencil
 *      2D: (+1,0), (0,+1), then for 8-connectivity (+1,+1), (-1,+1); 3D: (+1,0,0), (0,+1,0), (0,0,+1);
 *      2D squares of radius r (connectivity 24: r = 2, 48: r = 3, 80: r = 4, the larger neighbourhoods of the
 *      paper's experiments): (dx,0) for dx = 1..r, then (dx,dy) for dy = 1..r and dx = -r..r, x fastest;
 *      3D balls of radius r = 2, 3 or 4 (connectivity 32, 122 and 256, the spherical kernels of size 5, 7 and
 *      9): the offsets of length <= r whose first nonzero coordinate, from z down to x, is positive, ordered by
 *      z, then y, then x.
 *      w[o*n + i] weights the edge i <-> i + offset[o] and must be 0 where that neighbour is off-grid.
 *   lambda_q8 = round(256 lambda) >= 0.
 *   mem_kind: DOPE_MEM_HOST (pageable or pinned host memory) or DOPE_MEM_DEVICE (device pointers).
 * The inputs are copied; the caller keeps ownership.  Errors: EINVAL (off-grid weight, lambda < 0, weights so
 * large that per-node sum_j |c_ij| >= 2^29), ENOTSUBMODULAR (w < 0 with the max-flow solver). */
dope_status dope_set_energy(dope_ctx *ctx, const int32_t *u, const int32_t *w, int32_t lambda_q8, int32_t mem_kind);

/* Same as dope_set_energy but without waiting: the copies, state reset and weight preparation are only
 * enqueued on the context stream (device inputs must stay valid until that work has run).  DOPE_SOLVER_AUTO
 * resolves to max-flow when the blocks can take it (see dope_create), else to the exhaustive solver.  Validation errors
 * (EINVAL, ENOTSUBMODULAR) stop the loop on the device and are returned by the next call that reads the state
 * back (dope_iterate, dope_solve, dope_get_state, a batch call, ...). */
dope_status dope_set_energy_async(dope_ctx *ctx, const int32_t *u, const int32_t *w, int32_t lambda_q8,
                                  int32_t mem_kind);

/* Run exactly n_iter iterations of Algorithm 1's main loop (stops early only on EOVERFLOW / ESOLVER). */
dope_status dope_iterate(dope_ctx *ctx, int32_t n_iter, dope_info *out);

/* Run until the stopping rule holds or t reaches max_iter.  out may be NULL. */
dope_status dope_solve(dope_ctx *ctx, dope_info *out);

/* The segmentation Algorithm 1 returns, made binary: labels l_i = [Y_i > 2^15] (y_i > 1/2 strictly) as uint8[n],
 * to host memory (complete on return) or device memory (stream-ordered, returns at once). */
dope_status dope_labels(dope_ctx *ctx, uint8_t *labels, int32_t mem_kind);

/* The pairwise energy of Eq. (1) (each undirected edge once, as in Eq. (3)) of the current labels, scaled by 256:
 * E_q = 256 sum u_i l_i + lambda_q8 sum_edges w_ij |l_i - l_j| (exact int64).  EINVAL when the loaded energy
 * was rejected by validation. */
dope_status dope_energy(dope_ctx *ctx, int64_t *e_q8);

/* Checkpoint / test access to the whole ADMM state (host memory).  Y: int32[n]; A: int32[sum |block|];
 * yhat: uint8[sum |block|] (labels of the last block solve); mu: M for the next iteration; t: iterations. */
dope_status dope_get_state(dope_ctx *ctx, int32_t *Y, int32_t *A, uint8_t *yhat, int64_t *mu, int32_t *t);
dope_status dope_set_state(dope_ctx *ctx, const int32_t *Y, const int32_t *A, const uint8_t *yhat, int64_t mu,
                           int32_t t);

/* Per-block squared residuals r_k (int64[K]) of the last completed iteration. */
dope_status dope_block_resid(dope_ctx *ctx, int64_t *resid);

/* Per-block solver statistics of the last iteration, int32[K * 4]:
 * {free nodes after the strict forcing test (|U~| > sum of capacities; before the cascading elimination),
 *  push/relabel rounds, global relabels, elimination passes of the block's workgroup};
 * with the LSA-TR solver: {free nodes of the last step, push/relabel rounds over all steps, steps, final level}. */
dope_status dope_block_stats(dope_ctx *ctx, int32_t *stats);

/* Block geometry: *n_blocks = K; if table != NULL it receives 7 int32 per block:
 * x0, y0, z0, ex, ey, ez, offset (start of the block in the block-major vectors). */
dope_status dope_block_table(dope_ctx *ctx, int32_t *n_blocks, int32_t *table);

/* Sizes: n pixels, K blocks, sum of block sizes, half-stencil size h. */
dope_status dope_sizes(const dope_ctx *ctx, int64_t *n, int32_t *n_blocks, int64_t *total_block_px, int32_t *h);

/* Device bytes the context needs for p (for caller-allocated workspaces and admission by HBM footprint). */
size_t dope_workspace_bytes(const dope_params *p);

/* Launch schedule of the one-image block solves for p (a host query, no device needed; not an operation of the
 * paper but the order in which Algorithm 1's per-block solves of one iteration are handed to workgroups):
 * *n_blocks = K; if order != NULL (host memory, int32[K]) workgroup b of a block-solve launch solves block
 * order[b], blocks numbered x-fastest as in dope_block_table.  The blocks of full extent along every axis come
 * first, then the blocks clipped at the far faces; within each group every XCD takes a contiguous range.
 * EINVAL for invalid parameters (message in dope_last_error(NULL)). */
dope_status dope_dispatch_order(const dope_params *p, int32_t *n_blocks, int32_t *order);

/* Use caller-owned device memory (>= dope_workspace_bytes, 256-byte aligned) instead of allocating.
 * Must be called before dope_set_energy; the memory must outlive the context. */
dope_status dope_bind_workspace(dope_ctx *ctx, void *dev_ptr, size_t bytes);

/* Kernel timing with HIP events on the context stream.  While enabled, every block-solve launch and every
 * consensus launch (not the loop-control launch that follows it) records its own dispatch start and end in a pair
 * of events (hipExtLaunchKernel: no marker packets are added, so the timed stream runs as it would unprofiled);
 * dope_profile_read
 * returns the summed milliseconds and launch counts since enable. */
dope_status dope_profile_enable(dope_ctx *ctx, int32_t on);
dope_status dope_profile_read(dope_ctx *ctx, double *solve_ms, int32_t *solve_launches, double *consensus_ms,
                              int32_t *consensus_launches);

/* Block partition for an image: a pure function of (ndim, dims, connectivity), never of load, so that a
 * request's result does not depend on what else is running.  The choice comes from a table compiled into the
 * library, written by an offline sweep on MI355X (paper_1704_03116_amd/tune.py; measurements in
 * profiles/autotune_sweep.json): for every stencil and several image sizes, whole solves (upload, solve to the
 * stopping rule or max_iter, labels) of serving-style images were timed for every block edge B and overlap o
 * whose max-flow state fits the LDS (2D: B in {16, 20, 24, 32, 48, 64}, o in {1, 2, 4}; 3D: B in {5, 6, 8, 10,
 * 12, 16}, o in {1, 2}, as the stencil allows) and the fastest kept.  An image takes the row of the measured
 * size nearest to its shorter side (class bounds at geometric means).  Writes block[3] and overlap[3]; EINVAL
 * for an unsupported stencil. */
dope_status dope_autotune(int32_t ndim, const int32_t dims[3], int32_t connectivity, int32_t block[3],
                          int32_t overlap[3]);

/* ---- Batched iterations (many images, one launch per phase) ------------------------------------------------
 * A batch groups contexts so that every ADMM iteration runs as three launches for all of them together: a
 * persistent block-solve launch whose workgroups take (image, block) items from a device work queue (blocks of
 * images of uneven sizes and uneven max-flow cost share the GPU), one consensus / multiplier launch over all
 * their block pixels, and one loop-control launch.  Each image keeps its own state, stopping rule, iteration cap
 * and error status, and its results are bit-identical to running it alone (Algorithm 1 applied per image).
 * All contexts must share connectivity and resolved solver and have their energy set; the batch does not own
 * them and they must outlive it.  Work is ordered on the first context's stream: a dope_set_energy_async on a
 * member context must be ordered before the batch call that follows it (the same stream, or synchronised). */
typedef struct dope_batch dope_batch;

dope_status dope_batch_create(dope_ctx *const *ctxs, int32_t n, dope_batch **out);
/* dope_set_energy_async for every member in one launch: u[i], w[i], lambda_q8[i] as for context i (n entries in
 * context order, all in mem_kind memory; device inputs must stay valid until the work has run).  The resolved
 * solver of each member is kept.  Validation errors stop that image on the device and are returned by the next
 * batch call, as for dope_set_energy_async. */
dope_status dope_batch_set_energy_async(dope_batch *b, const int32_t *const *u, const int32_t *const *w,
                                        const int32_t *lambda_q8, int32_t mem_kind);
/* dope_labels for every member in one launch: labels[i] is uint8[n_i] in mem_kind memory (device memory:
 * stream-ordered, returns at once; host memory: complete on return). */
dope_status dope_batch_labels(dope_batch *b, uint8_t *const *labels, int32_t mem_kind);
/* exactly n_iter iterations for every image whose loop has not stopped on an error */
dope_status dope_batch_iterate(dope_batch *b, int32_t n_iter);
/* until every image meets its stopping rule or reaches its max_iter (an image that fails stops alone; the call
 * then returns that image's error after the others finish) */
dope_status dope_batch_solve(dope_batch *b);
/* on != 0: capture one iteration in a hipGraph and replay it (fewer launches per iteration) */
dope_status dope_batch_set_graph(dope_batch *b, int32_t on);
/* workgroups of the persistent block-solve launch; 0 = one per block item */
dope_status dope_batch_set_workers(dope_batch *b, int32_t n);
/* per-image loop information, n entries in context order */
dope_status dope_batch_info(dope_batch *b, dope_info *infos);
const char *dope_batch_last_error(const dope_batch *b);
void dope_batch_destroy(dope_batch *b);

/* ---- Serving: continuous batching of solve requests -----------------------------------------------------
 * A server owns one device arena of hbm_budget bytes.  Submitted requests wait in arrival order; each call to
 * dope_server_step admits waiting requests while their workspace (dope_workspace_bytes) fits in the free arena
 * and fewer than max_active are admitted, runs iters_per_step batched ADMM iterations (one by default) for all
 * admitted requests together (requests join and leave between steps; a request that meets its stopping rule or
 * max_iter inside a step stops there on the device), and retires the requests that met their stopping rule,
 * reached max_iter or failed, writing their labels.  Their ADMM state stays resident on the device between steps.
 * Every request's result is the one it gets when solved alone.  All requests of a server share connectivity;
 * the solver of each request resolves as in dope_set_energy_async.  A server is not thread-safe. */
typedef struct dope_server dope_server;

typedef struct {
    size_t hbm_budget;         /* bytes of device memory for request workspaces                           */
    int32_t max_active;        /* most requests admitted at once                                          */
    int32_t iters_per_step;    /* batched iterations per dope_server_step (0 = 1; at most 1024): fewer
                                  host round trips and membership changes, later admission               */
    void *stream;              /* hipStream_t; NULL = the server creates its own                          */
} dope_server_params;

dope_status dope_server_create(const dope_server_params *sp, dope_server **out);
/* Queue one solve.  The server borrows u, w (layout as dope_set_energy, in mem_kind memory) and labels_out
 * (uint8[n] in labels_mem_kind memory): they must stay valid until the request has finished.  p->stream is
 * ignored.  Returns EBUSY when the request alone needs more than hbm_budget, EINVAL for bad parameters or a
 * connectivity different from earlier requests.  *ticket identifies the request. */
dope_status dope_server_submit(dope_server *s, const dope_params *p, const int32_t *u, const int32_t *w,
                               int32_t lambda_q8, int32_t mem_kind, uint8_t *labels_out, int32_t labels_mem_kind,
                               int64_t *ticket);
/* One tick (admit, iters_per_step batched iterations, retire).  The tickets finished during the tick are written to
 * finished (at most max_finished; *n_finished receives their number).  Labels written to device memory are
 * ordered on the server stream; to host memory they are complete on return. */
dope_status dope_server_step(dope_server *s, int64_t *finished, int32_t max_finished, int32_t *n_finished);
/* Loop information and status of a finished request (EINVAL for unknown or unfinished tickets). */
dope_status dope_server_result(dope_server *s, int64_t ticket, dope_info *info, int32_t *status);
/* Requests waiting and admitted, and arena bytes in use. */
dope_status dope_server_load(const dope_server *s, int32_t *waiting, int32_t *active, size_t *hbm_in_use);
const char *dope_server_last_error(const dope_server *s);
void dope_server_destroy(dope_server *s);

/* ---- Multi-label Potts segmentation: alpha-expansion around DOPE ------------------------------------------
 * The paper's energy is binary (Eq. 1); its introduction reduces multi-region segmentation to sequences of binary
 * problems and its conclusion names multi-label energies as the next step.  This layer minimises
 *     E(L) = sum_i D[L_i, i] + sum_{edges (i,j)} V_ij [L_i != L_j],    L_i in {0, .., n_labels - 1},
 * by expansion moves (Boykov, Veksler, Zabih 2001): the move of label a lets every pixel keep its label or switch
 * to a; with y_i = 1 for a switch, twice the move's energy is 2 E(L) + sum_i u_i y_i + sum_edges W_ij |y_i - y_j|,
 *     u_i  = 2 (D[a, i] - D[L_i, i]) - sum_{j ~ i : L_j != L_i, L_i != a} V_ij (1 + [L_j = a]),
 *     W_ij = 2 V_ij if L_i = L_j != a;  V_ij if L_i != L_j and neither is a;  0 otherwise,
 * the binary energy of Eq. (1) with lambda = 1 (lambda_q8 = 256) and w = W >= 0, which an internal DOPE context
 * with p's grid, stencil, block partition and schedule solves (max-flow solver, Algorithm 1 to its stopping rule
 * or max_iter).  The move's labelling is accepted only when it lowers E strictly.  Labels start at
 * argmin_l D[l, i] (smallest l on ties).  Everything is integer and deterministic, so the label sequence is
 * bit-identical to a CPU implementation of the same loop.
 * Layout: D int32[n_labels][n] (label-major), V int32[h][n] on the half-stencil layout of dope_set_energy
 * (lambda folded in), labels uint8[n].  Limits (EINVAL otherwise): 2 <= n_labels <= 255, |D| < 2^26,
 * 0 <= V <= 2^20 (ENOTSUBMODULAR for V < 0), V = 0 on off-grid edges; a move whose binary weights break the
 * limits of dope_set_energy fails with that call's error.  The work is ordered on p->stream (NULL: the layer
 * creates its own stream).  A dope_ml is not thread-safe. */
typedef struct dope_ml dope_ml;

typedef struct {
    int32_t cycles;            /* completed passes over all labels                                         */
    int32_t moves;             /* expansion moves run                                                       */
    int32_t accepted;          /* moves that lowered E                                                      */
    int32_t binary_iterations; /* DOPE iterations summed over the moves' solves                             */
    int64_t energy;            /* E of the current labels                                                   */
} dope_ml_info;

dope_status dope_ml_create(const dope_params *p, int32_t n_labels, dope_ml **out);
/* Copy D and V (mem_kind memory; the caller keeps ownership), validate them, set L = argmin D and reset the
 * counters.  Synchronous. */
dope_status dope_ml_set_energy(dope_ml *m, const int32_t *D, const int32_t *V, int32_t mem_kind);
/* One expansion move of `label`: *accepted = 1 when its labelling lowered E; *energy = E afterwards (either may be
 * NULL).  Synchronous (the acceptance test reads E back). */
dope_status dope_ml_step(dope_ml *m, int32_t label, int32_t *accepted, int64_t *energy);
/* Cycles of moves a = 0 .. n_labels - 1 until a cycle accepts no move or max_cycles cycles ran. */
dope_status dope_ml_solve(dope_ml *m, int32_t max_cycles, dope_ml_info *out);
/* Current labels, uint8[n]: device memory (stream-ordered) or host memory (complete on return). */
dope_status dope_ml_labels(dope_ml *m, uint8_t *labels, int32_t mem_kind);
dope_status dope_ml_info_get(dope_ml *m, dope_ml_info *out);
const char *dope_ml_last_error(const dope_ml *m);
void dope_ml_destroy(dope_ml *m);

/* ---- Measurement --------------------------------------------------------------------------------------------
 * LDS read bandwidth of the GPU (bytes per second), the peak against which the block solver's LDS traffic is
 * reported: a probe kernel with every CU full (eight 256-thread workgroups per CU, 16 KiB of LDS each) streams
 * conflict-free 128-bit LDS reads, reps x 16 per thread; the best of three event-timed launches after a warm-up.
 * stream: hipStream_t (NULL = the null stream).  Synchronises the stream.  Errors: EINVAL (reps <= 0 or null
 * output), ENOMEM, EDEVICE. */
dope_status dope_measure_lds_bandwidth(void *stream, int32_t reps, double *bytes_per_s);

/* ---- Solving without allocation ---------------------------------------------------------------------------
 * For callers that cannot allocate (harnesses that forbid hipMalloc, serving loops that must not enter the
 * allocator): dope_set_energy_async, dope_solve and dope_labels of one image in one call, with the whole device
 * state (the layout dope_workspace_bytes(p) measures) in a static device array of the library of
 * DOPE_NOALLOC_MAX_BYTES, which every GPU the library runs on holds from module load until the process ends.
 * The call allocates nothing: no device or pinned memory, no stream, no event (the loop control is copied back
 * into host memory and the stream synchronised at every readback, so the call is slower than dope_solve on a
 * context for small images).
 *   p: as for dope_create; p->stream orders the work (NULL = the null stream).
 *   u, w: device memory, layout as for dope_set_energy; lambda_q8 as there.
 *   labels: device memory, uint8[n], labels l_i = [Y_i > 2^15] of the result; complete on return.
 *   out: host memory, may be NULL: the loop information of the solve.
 * Errors: EINVAL for bad parameters or when dope_workspace_bytes(p) > DOPE_NOALLOC_MAX_BYTES (the message is
 * dope_last_error(NULL)), the validation errors of dope_set_energy, and EOVERFLOW / ESOLVER / EDEVICE.
 * Every call on one GPU shares that GPU's array and leaves its contents there; each call re-initialises all of
 * the state it reads.  Calls on one GPU are serialised by a per-device lock and return only after their work has
 * completed, so calls from several host threads do not overlap; device work that is still running from an
 * earlier call cannot exist, but any other user of the array would race with a call. */
#define DOPE_NOALLOC_MAX_BYTES (64u << 20)
dope_status dope_solve_noalloc(const dope_params *p, const int32_t *u, const int32_t *w, int32_t lambda_q8,
                               uint8_t *labels, dope_info *out);

/* Context-local message of the last error; never NULL.  With ctx == NULL: the calling thread's last
 * dope_create validation message (empty when it succeeded). */
const char *dope_last_error(const dope_ctx *ctx);

void dope_destroy(dope_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DOPE_H */
