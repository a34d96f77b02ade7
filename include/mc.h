/*
 * mc.h -- C ABI of libmc, a GPU (gfx950) solver for grid min-cut problems by
 * decomposed total-variation denoising and Douglas-Rachford splitting, after
 * Kumar, Barbero, Jegelka, Sra and Bach, "Convex Optimization for Parallel
 * Energy Minimization" (arXiv:1503.01563).
 *
 * Problem.  A 2D 4-connected grid {H, W} or 3D 6-connected grid {D, H, W}
 * (W contiguous, row-major) with unaries w and non-negative edge weights a.
 * The cut energy of a labelling S (label 1 = in S) is
 *     E(S) = sum_{i in S} w_i + sum_edges a_e [edge e crosses S]        (Sec. 2, eq. (4))
 * i.e. the paper's f(x) - w^T x with the paper's w equal to -w here.  The
 * solver minimises the TV problem min_x f(x) + 1/2 |x + w|^2 (Sec. 2.3,
 * eq. (TV)), splits f into row / column / depth chain TVs (Sec. 3.1), runs
 * averaged alternating reflections over exact chain proxes (Sec. 3.3, 4.3)
 * and reads the cut off by thresholding x (Sec. 2.3), certified by the dual
 * gap of Sec. 2.2.
 *
 * Edge weights.  One array per axis: axis 0 = W (stride 1), axis 1 = H
 * (stride W), axis 2 = D (stride H*W).  a[j][i] is the weight of the edge
 * (i, i + stride_j); entries on the last slice along axis j are ignored
 * (with MC_VALIDATE they must be 0).  Weights must be >= 0 (Sec. 2: the
 * pairwise terms are submodular cut weights).
 *
 * 8-connected 2D grids (mc_grid.conn = 8).  Four weight arrays: a[0] along
 * W, a[1] along H as above, a[2][r][c] the diagonal (r,c)-(r+1,c+1) and
 * a[3][r][c] the anti-diagonal (r+1,c)-(r,c+1) of cell (r, c) (last row and
 * column ignored).  The diagonal edges are split into two families of
 * zig-zag chains over pairs of rows (Sec. 3.1, Fig. 1), solved with the
 * rows and columns in the product space (r = 4).
 *
 * Memory.  Every array argument is a DEVICE pointer owned by the caller,
 * contiguous, in the grid layout above, float32 unless stated; 256-byte
 * alignment is recommended.  Host-side outputs (mc_stats, energies) are
 * host pointers.  The library owns only the workspace inside mc_ctx.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default stream).
 * Work is enqueued on it; functions that fill host outputs synchronise it.
 *
 * Errors.  Every function returns an MC_* code; nothing throws across the
 * ABI.  mc_last_error() gives a thread-local message for the last failure.
 *
 * Threading.  One context per host thread; a context is bound to the device
 * it was created on.  Identical inputs give identical outputs (all
 * reductions use fixed trees; no floating-point atomics).  Batched solves
 * choose their work-item count by timing unless opts->batch_items fixes it;
 * the choice is cached per context, and a different count can change the
 * last bits of the iterates (never the certified energies).
 */
#ifndef MC_H
#define MC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MC_OK 0
#define MC_NOT_CONVERGED 1       /* max_iters reached; outputs are the last iterate */
#define MC_ERR_INVALID_ARG (-1)  /* null pointer, bad dims, n > 2^31 - 2^24, bad axis, bad opts */
#define MC_ERR_NEGATIVE_WEIGHT (-2) /* MC_VALIDATE only: some a < 0 (or non-zero on a last slice) */
#define MC_ERR_NONFINITE (-3)    /* MC_VALIDATE only: NaN/Inf in w or a */
#define MC_ERR_NOMEM (-4)        /* workspace allocation failed */
#define MC_ERR_DEVICE (-5)       /* HIP runtime error; text in mc_last_error() */
#define MC_ERR_NUMERIC (-6)      /* NaN/Inf appeared in the solver state */

/* mc_opts.flags */
#define MC_VALIDATE 1u           /* check inputs on the device before solving */
#define MC_PROFILE 2u            /* time every chain-sweep launch with hipEvents (mc_stats.sweep_ms) */
#define MC_WARM_MOVES 4u         /* mc_alpha_expansion: start each move from the primal and row duals
                                    of the same label's move in the previous cycle (Sec. 4.4) */
#define MC_WHOLE_CHAINS 8u       /* mc_tv_solve (4- and 6-connected grids and the 8-connected rows and
                                    columns): sweep every chain with one lane from its start instead of
                                    in overlapping pieces; faster when the chain proxes have long
                                    constant segments, slower otherwise */
#define MC_PIECE_CHAINS 16u      /* mc_tv_solve: always sweep in overlapping pieces.  With neither this
                                    nor MC_WHOLE_CHAINS, solves of 4- and 6-connected grids run their
                                    first sweeps in pieces, count the lanes whose bracket did not close,
                                    and sweep whole chains for the rest of the solve when they are 1 in
                                    10 or more (one extra stream synchronisation); 8-connected grids
                                    use pieces */
#define MC_DEBUG 64u             /* mc_tv_solve, 4- and 6-connected splitting: after every iteration
                                    scan the state for NaN/Inf, and at every check assert that each
                                    edge dual lies in its box |p| <= a and is zero where no edge
                                    exists; a failure returns MC_ERR_NUMERIC naming the iteration
                                    (one stream synchronisation per iteration) */
#define MC_FP64_STATE 128u       /* mc_tv_solve, 4- and 6-connected grids, variants AUTO, TWO_SET and
                                    PRODUCT (debug): the same splitting with its state, chain proxes
                                    and averaging in FP64 (one lane per whole chain: slow); the
                                    certificate, x_out and z_out as usual (z_out rounded to FP32) */
#define MC_BATCH_PERSISTENT 32u  /* mc_tv_solve_batched: run each check period's iterations as one
                                    cooperative persistent launch (resident waves share out the work
                                    items of every unfinished grid, a device-wide barrier between the
                                    row and column phases) instead of replaying a graph of per-phase
                                    launches; same results, slower on the 64-grid batch */

/* mc_opts.variant */
#define MC_VARIANT_AUTO 0        /* two-set form for 2D, product space for 3D */
#define MC_VARIANT_TWO_SET 1     /* r = 2 special case (Sec. 3.3), 2D only */
#define MC_VARIANT_PRODUCT 2     /* product-space form (Sec. 3.3, eq. (dualA)) */
/* Other outer iterations over the same chain proxes (4- and 6-connected grids;
 * state z0 / z_out: r*n floats, the dual blocks y_j (BCD, FISTA) or the point
 * projected onto K (AP)): */
#define MC_VARIANT_BCD 3         /* cyclic projections / block coordinate descent (Sec. 4.1) */
#define MC_VARIANT_AP 4          /* alternating projections in the product space (Sec. 4.2) */
#define MC_VARIANT_FISTA 5       /* FISTA on the smooth dual, step 1/r (Sec. 4.1) */
/* Block coordinate descent for up to opts->bcd_iters iterations (0 = 16),
 * then, unless it certified, the splitting of MC_VARIANT_AUTO started from its
 * dual blocks y and primal x = -w - sum_j y_j (two-set form: z0 = x + y_rows;
 * product space: z0_j = y_j + x / r).  BCD certifies within tens of iterations
 * on image-like data and can stall elsewhere; the splitting always finishes.
 * z0 and z_out must be NULL; stats add up both phases. */
#define MC_VARIANT_BCD_DR 6

typedef struct mc_ctx mc_ctx;

typedef struct {
    int32_t ndim;     /* 2 or 3 */
    int32_t conn;     /* 0 (or 4 / 6): axis edges only; 8: 2D 8-connected (see below) */
    int64_t dims[3];  /* ndim 2: {H, W}; ndim 3: {D, H, W} */
} mc_grid;

typedef struct {
    int32_t max_iters;    /* iteration cap (default 500) */
    int32_t check_every;  /* certificate cadence in iterations (default 1) */
    double gap_tol;       /* stop when cert = E(S) - LB(y) < gap_tol (default 1e-3) */
    int32_t variant;      /* MC_VARIANT_* */
    float tau0;           /* labels S_tau = {x > tau} for the ladder tau = tau0 * (1, 1e-1, 1e-2,
                             1e-3, 0, -1e-3, -1e-2, -1e-1, -1); the first of least energy
                             is returned (default 1e-3) */
    uint32_t flags;       /* MC_VALIDATE | MC_PROFILE | MC_WARM_MOVES | MC_WHOLE_CHAINS | MC_PIECE_CHAINS |
                             MC_BATCH_PERSISTENT | MC_DEBUG | MC_FP64_STATE */
    int32_t batch_items;  /* mc_tv_solve_batched: work items per sweep launch (0 = tuned) */
    int32_t bcd_iters;    /* MC_VARIANT_BCD_DR: block coordinate descent iterations (0 = 16) */
    int32_t reserved[2];  /* must be 0 */
} mc_opts;

typedef struct {
    int32_t status;       /* MC_OK or MC_NOT_CONVERGED */
    int32_t iters;        /* iterations run */
    double cert_gap;      /* E(S) - LB(y) at the last check (Sec. 2.2 gap at x = 1_S) */
    double energy;        /* E(S) of the returned labels, FP64 */
    double lower_bound;   /* LB(y) = sum_i min(y_i + w_i, 0), y rebuilt from clipped duals */
    double tv_gap;        /* TV duality gap at the FP32 primal estimate (diagnostic) */
    float tau_used;       /* threshold of the returned labels */
    float ms;             /* device time of the solve (hipEvent), milliseconds */
    double sweep_ms;      /* MC_PROFILE: summed device time of the chain-sweep launches */
    int32_t sweep_launches; /* number of chain-sweep launches (counted with or without MC_PROFILE) */
    int32_t checks;       /* certificate evaluations performed */
    int32_t items;        /* batched solves: work items per sweep launch used */
    int32_t whole_chains; /* mc_tv_solve splitting: 1 when the sweeps ended as whole chains */
    double dual_sweep_ms;  /* MC_PROFILE: the part of sweep_ms spent in launches that also wrote edge
                              duals (certificate iterations; mc_tv_solve splitting, else 0) */
    int32_t dual_sweep_launches; /* how many of sweep_launches those were */
} mc_stats;

/* Fill `o` with the defaults listed above. */
void mc_opts_default(mc_opts *o);

/* Create / destroy a context on `device` (HIP ordinal).  The context owns
 * the solver workspace, which grows to the largest grid solved. */
int mc_ctx_create(mc_ctx **out, int device);
int mc_ctx_destroy(mc_ctx *ctx);

/*
 * mc_tv_solve -- minimum cut of one grid (Sec. 2-4).
 *   w          [n] unaries.
 *   a          host array of ndim device pointers, a[j] = [n] weights along axis j
 *              (4 arrays for an 8-connected grid).
 *   z0         nullable warm start of the splitting state (Sec. 4.4: reuse of
 *              the dual vectors); n entries for the two-set form, ndim*n for
 *              the product space (family j at offset j*n), 4*n for an
 *              8-connected grid (rows, columns, even and odd zig-zag strips).
 *   x_out      nullable [n]: primal TV estimate x = -w - sum_j D_j^T p_j at the last
 *              check, p the edge duals of the chain proxes clipped to [-a, a].
 *   labels_out [n] uint8, 1 = in S.
 *   z_out      nullable: final state, same size as z0.
 *   stats      host, required.
 * Sweeps.  Each chain prox runs as overlapping pieces, many lanes per chain,
 * or as whole chains, one lane per chain (see MC_WHOLE_CHAINS and
 * MC_PIECE_CHAINS).  Unless forced, every solve of a 4- or 6-connected grid
 * picks whole chains after its first sweeps when those show long constant
 * segments; stats->whole_chains tells which kind ran last.
 * Returns MC_OK when cert < gap_tol (the labels are then a minimum cut
 * whenever all energies are multiples of a granularity g > gap_tol, e.g.
 * integer or 2^-8-dyadic data), MC_NOT_CONVERGED at max_iters, or an error.
 */
int mc_tv_solve(mc_ctx *ctx, const mc_grid *grid, const float *w,
                const float *const *a, const float *z0, float *x_out,
                uint8_t *labels_out, float *z_out, mc_stats *stats,
                const mc_opts *opts, void *stream);

/*
 * mc_tv_solve_noalloc -- mc_tv_solve without any device allocation, for
 * callers that cannot allocate: code that runs while a HIP graph is being
 * captured, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as mc_tv_solve, restricted to 4- and
 * 6-connected grids and the splitting variants MC_VARIANT_AUTO, _TWO_SET and
 * _PRODUCT (others, an 8-connected grid, and MC_PROFILE give
 * MC_ERR_INVALID_ARG).  Its workspace is one static device array per GPU,
 * reserved when the library's code object is loaded on that GPU and held
 * until the process ends: 32 MiB of solver state plus the reduction
 * partials.  The state needs 24 bytes per node in the two-set form and
 * 4 (4 r + 1) bytes per node in the product space (r families), so grids
 * up to about 1.39 M nodes in 2D (two-set) and 645 k nodes in 3D fit;
 * larger ones give MC_ERR_INVALID_ARG with the sizes in mc_last_error().
 * Every call on one GPU uses that GPU's array, from any context: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.  The array keeps the last call's contents; each
 * call sets what it reads before reading it.  The context must have been
 * created on the GPU (mc_ctx_create takes the array's device address).
 * Like mc_tv_solve it synchronises the stream at every certificate.
 */
int mc_tv_solve_noalloc(mc_ctx *ctx, const mc_grid *grid, const float *w,
                        const float *const *a, const float *z0, float *x_out,
                        uint8_t *labels_out, float *z_out, mc_stats *stats,
                        const mc_opts *opts, void *stream);

/*
 * mc_tv_prox_chains -- exact weighted 1D-TV prox of every line along `axis`
 * (Sec. 3.2): for each chain, x = argmin 1/2|x - v|^2 + sum_e a_e |x_{e+1} - x_e|.
 *   v, a_axis  [n] input and weights along the axis.
 *   x_out      [n] prox output.
 *   p_out      nullable [n]: edge duals p_e (x = v - D^T p, |p_e| <= a_e, clipped),
 *              stored at the edge's first voxel; 0 on the last slice.
 */
int mc_tv_prox_chains(mc_ctx *ctx, const mc_grid *grid, int axis,
                      const float *v, const float *a_axis, float *x_out,
                      float *p_out, void *stream);

/*
 * mc_cut_energy -- E(S) of eq. (4) in FP64 with a fixed reduction order;
 * exact for integer and dyadic data.  labels [n] uint8 (non-zero = in S).
 * a holds ndim arrays, or 4 for an 8-connected grid.
 * Synchronises the stream; energy_out is a host pointer.
 */
int mc_cut_energy(mc_ctx *ctx, const mc_grid *grid, const float *w,
                  const float *const *a, const uint8_t *labels,
                  double *energy_out, void *stream);

/*
 * mc_tv_solve_batched -- minimum cuts of n_grids 2D grids of possibly different
 * sizes, solved together (two-set form, Sec. 3.3 special case r = 2).  The
 * paper runs the chain proxes of a family in parallel over chains
 * (Sec. 5.1); here every sweep launch covers the chains of all unfinished
 * grids at once, and each grid stops at its own certificate (Sec. 2.2).
 * Arrays are per grid:
 *   grids[g]       2D grid {H, W}.
 *   w[g]           [n_g] unaries (device).
 *   a[2g], a[2g+1] [n_g] weights along W and along H (device).
 *   labels[g]      [n_g] uint8 output (device).
 *   x_out          nullable host array; x_out[g] nullable [n_g] primal estimate.
 *   z_out          nullable host array; z_out[g] nullable [n_g] splitting state
 *                  after the grid's last check (device).
 *   stats[g]       host; ms is the device time from the start of the solve to
 *                  the check that certified the grid (per-grid solve time);
 *                  iters the iteration of that check.
 * opts.check_every is rounded up to an even number of iterations: one check
 * period is captured in a hipGraph and replayed; the iterations left below a
 * whole period at opts.max_iters run outside the graph, so no grid runs more
 * than opts.max_iters and every grid ends on a check.  opts.batch_items > 0
 * fixes the work items per sweep launch (with the default piece overlap); 0
 * uses the work items and overlap tuned on the first solve of this batch
 * shape (one timed iteration per candidate pair).  Synchronises the stream.  Returns MC_OK when
 * every grid is certified, MC_NOT_CONVERGED otherwise.
 */
int mc_tv_solve_batched(mc_ctx *ctx, int n_grids, const mc_grid *grids,
                        const float *const *w, const float *const *a,
                        uint8_t *const *labels, float *const *x_out, float *const *z_out, mc_stats *stats,
                        const mc_opts *opts, void *stream);

/*
 * Learned warm start (2D, two-set form).  The paper starts DR from earlier
 * dual vectors when problems are related (Sec. 4.4, 6.1); here a small
 * convolutional network proposes the starting state instead:
 *   features (w/20, a_x/10, a_y/10) -> three conv3x3 + ReLU layers of 32
 *   channels -> conv3x3 -> two channels: x0 (a guess of the TV solution) and
 *   p1 (a guess of the row-family edge duals).
 * conv3x3 is the zero-padded cross-correlation
 *   out[y,x,co] = b[co] + sum_{ky,kx,ci} W[co,ky,kx,ci] in[y+ky-1, x+kx-1, ci].
 * Weights and activations are BF16 on the device, sums FP32 (MFMA).
 * Parameters: one FP32 device vector of mc_ws_param_count() entries; for each
 * layer (cin, cout) in (3,32), (32,32), (32,32), (32,2): W in index order
 * (co, ky, kx, ci), then b.
 * Images: w, a_x, a_y are [batch][H][W] FP32 device arrays (a_x weights along
 * W, a_y along H, as in mc_tv_solve); out and target are [batch][2][H][W]
 * (plane 0 x0, plane 1 p1).  The network's scratch lives in the context.
 */
int mc_ws_param_count(void);

/* Network output for a batch of images (asynchronous on `stream`). */
int mc_ws_forward(mc_ctx *ctx, const float *params, int batch, int H, int W,
                  const float *w, const float *a_x, const float *a_y, float *out,
                  void *stream);

/* Forward pass, mean-squared-error loss against `target` (mean over all
 * batch*2*H*W outputs) and its gradient: grad [mc_ws_param_count()] is
 * overwritten.  loss (host, nullable) receives the FP64 loss; giving it
 * synchronises the stream. */
int mc_ws_backward(mc_ctx *ctx, const float *params, int batch, int H, int W,
                   const float *w, const float *a_x, const float *a_y,
                   const float *target, float *grad, double *loss, void *stream);

/* One Adam step (step counts from 1, bias-corrected) on the FP32 master
 * parameters, in place; m and v are the moment vectors (zero before step 1). */
int mc_ws_adam_step(mc_ctx *ctx, float *params, const float *grad, float *m, float *v,
                    int step, float lr, float beta1, float beta2, float eps,
                    void *stream);

/* Starting state of the two-set splitting from one network output
 * out [2][H][W]: z0 = c x0 + D_rows^T clip(p1, -a_x, a_x), where
 * (D^T p)[y][x] = p[y][x-1] - p[y][x] (0 outside the row).  The dual part lies
 * in the row family's set K exactly.  z0 [H*W] is passed to mc_tv_solve. */
int mc_ws_warm_state(mc_ctx *ctx, const mc_grid *grid, const float *out,
                     const float *a_x, float c, float *z0, void *stream);

/*
 * ---- Multi-label energies by alpha-expansion (Sec. 4.4: move-making reduces
 * a multi-label problem to a series of binary cuts; Sec. 6.1 solves a
 * 4-connected stereo task that way with the two-set dual). ----
 *
 * On a 2D 4-connected grid (grid->ndim = 2, conn 0 or 4), labels f_i in
 * {0..n_labels-1}:
 *     E(f) = sum_i data[f_i][i] + sum_{edges e = (u, v)} lam_e V(f_u, f_v)
 *   data    [n_labels][H][W] label costs (device, FP32).
 *   lam     host array of 2 device pointers: lam[0][i] weighs (i, i+1) along W
 *           (last column 0), lam[1][i] weighs (i, i+W) (last row 0); >= 0.
 *   v_kind  MC_V_POTTS (V = [a != b]) or MC_V_TRUNC_LINEAR
 *           (V = min(|a - b|, v_trunc), v_trunc >= 0): both metrics, so every
 *           expansion move is a cut problem with non-negative weights.
 *   labels  [H][W] int32 device labels; every entry must lie in
 *           [0, n_labels) (checked on the device: MC_ERR_INVALID_ARG).
 * The move of label alpha lets each pixel keep f_i or take alpha.  With
 * A = V(f_u, f_v), B = V(f_u, alpha), C = V(alpha, f_v) its binary problem in
 * the form of mc_tv_solve (S = pixels that switch) is
 *     w_i = data[alpha][i] - data[f_i][i] + lam (C - A - B)/2 for each edge with
 *           i = u, + lam (B - A - C)/2 for each edge with i = v,
 *     a_e = lam (B + C - A) / 2,
 * and E(f with S switched) = E(f) + E_bin(S).
 */
#define MC_V_POTTS 0
#define MC_V_TRUNC_LINEAR 1

typedef struct {
    int32_t status;       /* MC_OK: the last cycle made no improving move (a local
                             minimum for every expansion); MC_NOT_CONVERGED:
                             max_cycles reached or some move was not certified */
    int32_t cycles;       /* cycles over alpha = 0..n_labels-1 */
    int32_t moves;        /* binary problems solved */
    int32_t accepted;     /* moves applied (those that lowered E) */
    int32_t uncertified;  /* moves whose solve stopped at opts->max_iters */
    int32_t skipped;      /* moves not solved: no move applied since the same
                             label's previous one, so its problem and result
                             are unchanged */
    int64_t dr_iters;     /* splitting iterations over all moves */
    double energy0;       /* E(f) of the labels passed in, FP64 */
    double energy;        /* E(f) of the labels returned, FP64 */
    float ms;             /* wall time of the whole call, milliseconds */
    float reserved2;
} mc_ml_stats;

/* The binary problem of one expansion move of label `alpha` from `labels`:
 * w_out [H][W] and a_out[0], a_out[1] (host array of 2 device pointers,
 * [H][W] each, last column / row 0), ready for mc_tv_solve.  Asynchronous on
 * `stream` except for the label check, which synchronises it. */
int mc_expansion_problem(mc_ctx *ctx, const mc_grid *grid, int n_labels, const float *data,
                         const float *const *lam, int v_kind, float v_trunc,
                         const int32_t *labels, int alpha, float *w_out, float *const *a_out,
                         void *stream);

/* E(f) in FP64 with a fixed reduction order; synchronises `stream`. */
int mc_ml_energy(mc_ctx *ctx, const mc_grid *grid, int n_labels, const float *data,
                 const float *const *lam, int v_kind, float v_trunc, const int32_t *labels,
                 double *energy_out, void *stream);

/* Alpha-expansion from the labels passed in, in place: cycles over
 * alpha = 0..n_labels-1, each move solved exactly by mc_tv_solve with `opts`
 * (nullable: defaults; the move's labels are its certified minimum cut) and
 * applied when its energy is negative, until a cycle applies no move or
 * max_cycles cycles have run.  The move of a label is skipped while no move
 * has been applied since its previous one (same labels, same result: the
 * applied moves are those of the plain cycles).  With MC_WARM_MOVES the move of a label starts
 * from z0 = x + D_rows^T clip(p1, -a_x, a_x), x and p1 the primal and row
 * duals its previous move ended with (the moves in between change the
 * problem, so this is a starting point, not a solution); it needs the two-set
 * splitting (opts->variant AUTO or TWO_SET, else INVALID_ARG).  Move problems are
 * flat where the labels agree, so their chain proxes have long constant
 * segments: MC_WHOLE_CHAINS suits them (3.4x faster on a 384x288, 16-label
 * stereo-like problem).  Workspace comes from
 * the context (4 + 2 n_labels floats per pixel with MC_WARM_MOVES, 3 without);
 * synchronises `stream`.  With MC_VALIDATE in opts->flags the weights are checked first
 * (non-finite or negative entries, non-zero last column / row). */
int mc_alpha_expansion(mc_ctx *ctx, const mc_grid *grid, int n_labels, const float *data,
                       const float *const *lam, int v_kind, float v_trunc, int32_t *labels,
                       int max_cycles, mc_ml_stats *stats, const mc_opts *opts, void *stream);

/* Text for a status code, and the calling thread's last error message. */
const char *mc_status_string(int code);
const char *mc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MC_H */
