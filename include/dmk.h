/*
 * dmk.h -- C ABI of the MI355X (gfx950) implementation of the DMK
 * (dual-space multilevel kernel-splitting) point code of Jiang & Greengard,
 * "A dual-space multilevel kernel-splitting framework for discrete and
 * continuous convolution", arXiv 2308.00292.
 *
 * The library computes, for N points x_i with charges q_i (sources equal
 * targets),
 *
 *     pot_i = sum_{j != i, |x_i - x_j| > 0} K(|x_i - x_j|) q_j,
 *     K(r) = 1 / (4 pi r)        (3-D Laplace, eq. laplacesum), or
 *     K(r) = -log(r) / (2 pi)    (2-D Laplace),
 *
 * to a requested relative precision tol, with the O(N) scheme of Sec. 3.3
 * and Sec. 3.5 ("The linear scaling full DMK algorithm", "The full DMK
 * algorithm for discrete sources"), the PSWF kernel split of Sec. 3.7 in
 * 3-D and its Fourier-space form (Sec. 4.6, with the windowed root kernel of
 * Sec. 4.7) in 2-D, where K(r) = K_0(lambda r) is also available.  Pairs at
 * distance exactly zero (the self pair and coincident points) contribute
 * nothing.  A plan may hold many independent 2-D point sets
 * (dmk_plan_batched); each is solved in its own root box and every stage
 * runs over the boxes of all of them at once.
 *
 * The volume entry points (dmk_vol_*) compute the continuous convolution
 *
 *     u(x) = int_{B_0} rho(y) / (4 pi |x - y|) dy,   B_0 = [-1/2, 1/2]^3,
 *
 * at the Chebyshev nodes of an adaptive tree that resolves rho (Sec. 3.6,
 * "Modification of DMK for continuous sources"), with the Gaussian split of
 * Sec. 3.2 and a sum-of-Gaussians near field (Sec. 3.6, Sec. 4.4).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (memory of the current HIP
 *    device), unless the argument is documented as a host pointer.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Work is enqueued on it asynchronously unless stated otherwise.
 *  - Status codes only; no C++ exception crosses the ABI.  After a non-zero
 *    status, dmk_last_error() returns a message for the calling thread.
 *  - Implemented: DMK_LAPLACE and DMK_YUKAWA in 2-D and 3-D; DMK_POWER2 in 3-D.
 */
#ifndef DMK_H
#define DMK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMK_OK = 0,
    DMK_ERR_ARG = -1,          /* invalid argument                           */
    DMK_ERR_UNSUPPORTED = -2,  /* kernel / dim / tol not implemented         */
    DMK_ERR_NOMEM = -3,        /* device allocation failed                   */
    DMK_ERR_HIP = -4,          /* a HIP runtime call failed                  */
    DMK_ERR_PRECISION = -5,    /* precision mode incompatible with tol       */
    DMK_ERR_STATE = -6         /* plan busy or in an unusable state          */
} dmk_status;

/* DMK_LAPLACE: 1/(4 pi r) in 3-D, -log(r)/(2 pi) in 2-D.
 * DMK_YUKAWA: e^{-lambda r}/(4 pi r) in 3-D, K_0(lambda r) in 2-D (lambda in
 * dmk_opts); both split in Fourier space with the PSWF (Sec. 4.6).
 * DMK_POWER2: 1/r^2 in 3-D (no constant factor), split in physical space
 * with the PSWF power-function window (Sec. 4.5, alpha = 2). */
typedef enum { DMK_LAPLACE = 0, DMK_YUKAWA = 1, DMK_POWER2 = 2 } dmk_kernel;

/* Arithmetic of the eval pipeline.  Input and output are always FP64. */
typedef enum {
    DMK_FP64 = 0,   /* every stage in double precision                     */
    DMK_MIXED = 1   /* transforms and residual sums in FP32, box-relative
                       offsets, small-r residuals and the final sum in FP64 */
} dmk_precision;

/* Options; a zero field selects the default.  Pass NULL for all defaults. */
typedef struct {
    int32_t  leaf_max;    /* n_s, the leaf capacity (default 64)              */
    int32_t  max_depth;   /* depth cap of the tree (default 20 in 3-D, 30 in
                             2-D, at most the key bits per axis: 21 in 3-D,
                             31 in 2-D, fewer in a batch, see dmk_plan_batched) */
    int32_t  precision;   /* dmk_precision (default DMK_FP64)                 */
    int32_t  reserved0;
    uint64_t flags;       /* DMK_FLAG_* bits (DMK_FLAG_BATCHED)               */
    double   lambda;      /* Yukawa parameter in input units (DMK_YUKAWA)     */
    int32_t  p;           /* proxy (Chebyshev) order per axis; 0: from tol    */
    int32_t  n_f;         /* plane-wave half width of D_l (N_1 = 2 n_f + 1);
                             0: from tol.  A nonzero p and/or n_f must name a
                             compiled pair: (9, 6), (15, 10) or (18, 12); the
                             missing member is taken from that pair          */
    double   pswf_c;      /* PSWF parameter c in [2, 40]; 0: from tol         */
} dmk_opts;

/* Batched execution of dmk_eval: the middle of the pipeline (upward pass,
 * root window, plane-wave stages over all levels, local values, leaf
 * evaluation) is captured once into a HIP graph and replayed, and the
 * residual sums run on a second stream concurrently with it.  Without the
 * flag every stage is launched eagerly, one after the other, on the caller's
 * stream.  Results are identical either way. */
#define DMK_FLAG_BATCHED 2ull

/* The plan allocates no eval workspace (gathered charges, proxies, plane
 * waves, local values, partial potentials): such a plan is evaluated only
 * with dmk_eval_noalloc, which takes the workspace from the library's static
 * scratch; dmk_eval, dmk_eval_parts and dmk_copy_box_data return
 * DMK_ERR_STATE on it.  Ignored by dmk_vol_plan. */
#define DMK_FLAG_NO_WORKSPACE 4ull

/* Schedule of the upward pass and of the local values.  Queue-fed: one
 * launch per stage over all levels, in which a grid takes the boxes from a
 * device work queue in dependency order (finest level first for the upward
 * pass, coarsest first for the local values) and a box waits on flags until
 * the boxes it reads are done.  Per level: one launch per tree level, one
 * workgroup per box.  Each box is computed by the same code either way, so
 * the results are bit-identical.  Default: queue-fed in 3-D (point and
 * volume plans), per level in 2-D (where a box is p^2 values and the queue's
 * own cost outweighs what it saves).  The two flags force one schedule;
 * both together are DMK_ERR_ARG. */
#define DMK_FLAG_LEVEL_LAUNCHES 8ull
#define DMK_FLAG_QUEUE_LAUNCHES 16ull

/* Size of the static device scratch of dmk_eval_noalloc, per device. */
#define DMK_NOALLOC_MAX_BYTES (128ll << 20)

typedef struct dmk_plan_s *dmk_plan_t;

/* Sizes of a plan (host struct filled by dmk_plan_info). */
typedef struct {
    int64_t n;            /* points                                          */
    int64_t nbox;         /* boxes of all levels                             */
    int32_t nlevels;      /* levels 0 .. nlevels-1                           */
    int32_t p;            /* Chebyshev proxy order per dimension             */
    int32_t nf;           /* plane-wave half width of D_l                    */
    int32_t nw;           /* plane-wave half width of the windowed W_0       */
    double  c;            /* PSWF parameter                                  */
    double  tol;
    int32_t leaf_max;
    int32_t precision;
    int64_t nleaf;        /* leaves holding at least one point               */
    int64_t nfout;        /* boxes with F_out                                */
    int64_t nfin;         /* non-empty boxes with F_in                       */
    int64_t npairs;       /* candidate (target, source) pairs of the residual */
    int64_t device_bytes; /* device memory held by the plan                  */
    double  center[3];    /* root box centre of problem 0 (input units)      */
    double  side;         /* root box side of problem 0 (input units)        */
    int32_t dim;
    int32_t nprob;        /* independent problems in the plan                */
    int64_t nsrc, ntgt;   /* sources and targets (both n unless the plan has
                             separate target sets; then n = nsrc + ntgt)    */
    int32_t queue_timeouts; /* waits of the queue-fed kernels that ran out of
                             their poll bound, over all evals of the plan so
                             far (read from the device: synchronise the eval
                             streams first).  0 in every correct run; any
                             other value means results since then are wrong. */
    int32_t reserved1;
} dmk_plan_stats;

/*
 * dmk_plan -- build the adaptive tree and all tables for one point set.
 *
 * Paper: Step 0 (initialisation: level-restricted adaptive tree, flags
 * F_leaf/F_out/F_in) and Step 1 (precomputation of the 1-D transforms and
 * plane-wave weights) of Sec. 3.5; tree conventions of Sec. 3.2; parameters
 * c, N_1 = 2 n_f + 1, p of Table 1 (Sec. 3.7).
 *
 *  dim     2 or 3.
 *  kernel  DMK_LAPLACE (dim 3: 1/(4 pi r); dim 2: -log(r)/(2 pi)), or
 *          DMK_YUKAWA (dim 3: e^{-lambda r}/(4 pi r); dim 2: K_0(lambda r)),
 *          or DMK_POWER2 (dim 3 only: 1/r^2),
 *          lambda = opts->lambda > 0 in input units.  Limits (else
 *          DMK_ERR_UNSUPPORTED): dim 3, lambda S in [1e-3, 1000]; dim 2,
 *          lambda S <= 50 per problem (S the root box side).
 *  tol     in [1e-12, 1e-2] (else DMK_ERR_ARG).  Parameters (c, n_f, p):
 *          for tol = 1e-3, 1e-6 (Table 1) or 1e-5 (c = log 1e5, n_f = 10,
 *          p = 15) the table's row; for any other tol, or when opts sets
 *          pswf_c, c = opts->pswf_c or log(1/tol) (eq. pswfcvalue) and the
 *          smallest n_f and p whose plane-wave and proxy errors on the
 *          level-0 difference kernel stay within tol (the rule that gives
 *          Table 1's N_1 and p at its tolerances), rounded up to the
 *          smallest compiled (p, n_f) pair: (9, 6), (15, 10), (18, 12).
 *          Tolerances that need more (below about 1e-6, including Table 1's
 *          1e-9 and 1e-12 rows: p = 28 and 38) give DMK_ERR_UNSUPPORTED:
 *          those proxy grids (p^3 = 22k and 55k values per box) do not fit
 *          the kernels' per-box LDS staging.  The chosen values are reported
 *          by dmk_plan_info.  DMK_MIXED requires tol >= 1e-6 (else
 *          DMK_ERR_PRECISION).
 *  n       number of points, 0 <= n < 2^31.
 *  pts     device, [n][dim] FP64, row-major, input order.  Read during the
 *          call only; the plan keeps its own sorted copy.  Non-finite
 *          coordinates give DMK_ERR_ARG.
 *  opts    host pointer or NULL.
 *  stream  work is enqueued on it; the call synchronises it before return.
 *  out     host pointer receiving the plan handle (NULL on failure).
 *
 * The plan owns its device memory until dmk_plan_destroy.
 */
dmk_status dmk_plan(int dim, dmk_kernel kernel, double tol, int64_t n, const double *pts,
                    const dmk_opts *opts, void *stream, dmk_plan_t *out);

/*
 * dmk_plan_targets -- a plan with targets distinct from the sources:
 * u(x_i) = sum_j K(x_i - y_j) q_j at ntgt targets x_i from nsrc sources y_j
 * (pairs at distance 0 excluded, as for dmk_plan).
 *
 * Paper: the general problem of Sec. 3.5, whose input is N sources and
 * targets; the tree is refined while a box holds more than n_s points of
 * the union (Sec. 3.2), sources carry the outgoing expansions and the
 * residual sums, targets the local expansions and evaluations (Steps 2-4).
 *
 *  dim      must be 3 (2-D: DMK_ERR_UNSUPPORTED).
 *  kernel, tol, opts, stream, out  as dmk_plan.
 *  nsrc, src  device, [nsrc][3] FP64 source points, input order.
 *  ntgt, tgt  device, [ntgt][3] FP64 target points, input order.
 *  nsrc + ntgt < 2^31.  Either set may be empty.
 * dmk_eval (and dmk_eval_parts, dmk_eval_noalloc) on such a plan take
 * charges [nsrc] (source order) and return pot [ntgt] (target order).
 * dmk_export_tree describes the tree of the union, whose input indices are
 * the sources 0..nsrc-1 followed by the targets nsrc..nsrc+ntgt-1.
 */
dmk_status dmk_plan_targets(int dim, dmk_kernel kernel, double tol, int64_t nsrc, const double *src, int64_t ntgt,
                            const double *tgt, const dmk_opts *opts, void *stream, dmk_plan_t *out);

/*
 * dmk_plan_batched -- one plan for nprob independent point sets.
 *
 * Paper: the same steps as dmk_plan, applied to every problem; each problem
 * gets its own root box from its own bounding box (Sec. 3.1).  The trees
 * form a forest: level 0 holds the nprob roots, boxes of all problems are
 * interleaved level by level, and every stage of dmk_eval is one launch over
 * the boxes of all problems.
 *
 *  dim      2 or 3 (3-D batches of the Yukawa kernel, whose tables depend
 *           on each problem's lambda S_b: DMK_ERR_UNSUPPORTED).
 *  nprob    >= 1.
 *  offsets  HOST, [nprob+1] int64, offsets[0] = 0, non-decreasing; problem b
 *           is points offsets[b] .. offsets[b+1]-1 (empty problems allowed).
 *  pts      device, [offsets[nprob]][dim] FP64, the problems concatenated.
 *  Other arguments as dmk_plan.  Keys hold ceil(log2 nprob) bits of problem
 *  index, leaving (63 - those bits)/dim bits per axis (at most 31), which
 *  caps max_depth.
 * dmk_eval on such a plan takes the concatenated charges and returns the
 * concatenated potentials, problem by problem, with no interaction between
 * problems.
 */
dmk_status dmk_plan_batched(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets,
                            const double *pts, const dmk_opts *opts, void *stream, dmk_plan_t *out);

/*
 * dmk_tune_leaf -- the leaf-capacity tuner: picks n_s among candidates by
 * timing dmk_eval on the caller's points and charges.
 *
 * Paper: n_s balances the cost of the local (residual) interactions against
 * all other steps and is chosen by experiment (remark at the end of Sec.
 * 3.5; Sec. 5.1 quotes the values used).  Every candidate gives a result
 * within tol; only the time differs.
 *
 *  dim, kernel, tol, opts  as dmk_plan / dmk_plan_batched (opts->leaf_max is
 *                          ignored; opts->flags and precision apply).
 *  nprob, offsets          HOST offsets [nprob+1]; a single point set is
 *                          nprob = 1, offsets = {0, n}.
 *  pts, charges            device, as for dmk_plan_batched and dmk_eval.
 *  cand                    HOST [ncand] leaf capacities (>= 1).
 *  reps                    timed evaluations per candidate (after one warm-up).
 *  best                    HOST, receives the fastest candidate.
 *  ms                      HOST [ncand] or NULL: mean eval time of each (ms).
 * Builds and destroys one plan per candidate; synchronous on `stream`.
 */
dmk_status dmk_tune_leaf(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets,
                         const double *pts, const double *charges, const dmk_opts *opts, const int32_t *cand,
                         int32_t ncand, int32_t reps, void *stream, int32_t *best, double *ms);

/*
 * dmk_tune -- the autotuner: picks the proxy order and plane-wave width
 * (p, n_f) and the leaf capacity n_s for the caller's points and charges.
 *
 * Paper: the parameters of Table 1 (Sec. 3.7) are chosen for the method's
 * error bound, and n_s by experiment (remark at the end of Sec. 3.5).  The
 * tuner measures instead of bounding: direct sums (the definition, FP64,
 * compensated) at up to 256 evenly spaced targets give an accuracy gate; the
 * coarsest compiled (p, n_f) pair whose sampled relative l2 error is within
 * tol at n_s = cand[0] is kept (the pairs are tried from the coarsest; the
 * caller's p/n_f if opts sets them), then every candidate n_s is timed and
 * the fastest kept; if that configuration misses tol, the next pair is
 * timed.  c stays that of the tolerance (opts->pswf_c if set).
 *
 *  dim, kernel, tol, nprob, offsets, pts, charges, opts  as dmk_tune_leaf.
 *  cand, ncand, reps  HOST leaf capacities to time, evals per candidate.
 *  best   HOST, receives opts with leaf_max, p, n_f and pswf_c filled in.
 *  ms     HOST [ncand] or NULL: mean eval time of each candidate (ms), for
 *         the pair kept.
 *  err    HOST or NULL: sampled relative l2 error of the configuration kept.
 * Builds and destroys one plan per trial; synchronous on `stream`; needs at
 * least two points.
 */
dmk_status dmk_tune(int dim, dmk_kernel kernel, double tol, int32_t nprob, const int64_t *offsets,
                    const double *pts, const double *charges, const dmk_opts *opts, const int32_t *cand,
                    int32_t ncand, int32_t reps, void *stream, dmk_opts *best, double *ms, double *err);

/*
 * dmk_problem_info -- root box of problem `prob` of a plan (input units):
 * centre [dim] and side, both HOST pointers (either may be NULL).
 */
dmk_status dmk_problem_info(dmk_plan_t plan, int32_t prob, double *center, double *side);

/*
 * dmk_eval -- potentials of one charge vector on a planned point set.
 *
 * Paper: Steps 2-5 of Sec. 3.5 (upward pass, downward pass, direct
 * interactions with the residual kernel, self-interaction correction).
 *
 *  charges device, [n] FP64, input order.
 *  pot     device, [n] FP64, input order, overwritten.
 *  stream  asynchronous: pot is valid once the stream has been synchronised.
 *
 * A plan owns its workspace: a second dmk_eval on the same plan while one
 * is in flight on another host thread returns DMK_ERR_STATE.  Evals on one
 * plan are ordered whatever streams they use: each one records a completion
 * event on its stream and the next one makes its stream wait on it (not
 * while the stream is being captured into a graph: the capture orders the
 * work).  Calls may be issued back to back.
 */
dmk_status dmk_eval(dmk_plan_t plan, const double *charges, double *pot, void *stream);

/*
 * dmk_eval_noalloc -- dmk_eval for callers that cannot allocate device
 * memory at call time (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).
 *
 * Same arguments and the same result as dmk_eval (bit for bit, as the eager
 * form of dmk_eval).  The eval workspace comes from a static device array of
 * DMK_NOALLOC_MAX_BYTES that the library holds on every device it runs on
 * until the process ends, not from the plan, so plans built with
 * DMK_FLAG_NO_WORKSPACE hold none of their own.  The call allocates nothing:
 * no hipMalloc, no hipFree, no events.  Stages run as eager launches on
 * `stream` (no graph replay, no second stream, no stage timing).
 *
 *  plan     a point plan (dmk_plan or dmk_plan_batched); volume plans give
 *           DMK_ERR_ARG.
 *  charges  device, [n] FP64, input order.
 *  pot      device, [n] FP64, input order, overwritten.
 *  stream   asynchronous, as dmk_eval.
 * Errors: DMK_ERR_ARG if the plan's workspace (sum of its buffers, each
 * rounded up to 256 bytes) exceeds DMK_NOALLOC_MAX_BYTES; otherwise as
 * dmk_eval.  Every call on one device shares the one array, which keeps the
 * last call's contents: calls that overlap in time on one device (other
 * streams, other threads, other plans) race and give wrong results; calls
 * on one stream, or ordered by the caller, are safe.
 */
dmk_status dmk_eval_noalloc(dmk_plan_t plan, const double *charges, double *pot, void *stream);

/*
 * dmk_eval_parts -- like dmk_eval, but returns the far-field part (the
 * windowed and difference kernels through plane waves and Chebyshev
 * interpolation, eq. farpotential) and the near part (residual kernel sums
 * plus the self correction, eq. nearpotential and Step 5) separately, both
 * in input order and input units (3-D: both scaled by 1/(4 pi S); 2-D: the
 * constant -log(S)/(2 pi) of the unit change is carried by the far part for
 * the total charge and by the near part for pairs at distance zero).
 * pot = far + near.
 * Either output pointer may be NULL.
 */
dmk_status dmk_eval_parts(dmk_plan_t plan, const double *charges, double *far_part,
                          double *near_part, void *stream);

/* dmk_plan_info -- sizes of a plan; st is a host pointer. */
dmk_status dmk_plan_info(dmk_plan_t plan, dmk_plan_stats *st);

/*
 * dmk_export_tree -- copy the tree to caller-owned HOST arrays (for
 * bit-exact comparison with an independent tree builder).  Any pointer may
 * be NULL to skip that array.  Sizes: n = points, B = nbox (dmk_plan_info).
 *   perm       [n]       int64  sorted position -> input index
 *   level      [B]       int32
 *   bkey       [B]       uint64 Morton prefix of the box at its level, with
 *                               the problem index above it (batched plans)
 *   parent     [B]       int64  (-1 for a root)
 *   child0     [B]       int64  first of 2^dim contiguous children, -1 for a leaf
 *   pstart     [B]       int64  first sorted point of the box
 *   pcount     [B]       int64  points in the box
 *   flags      [B]       uint8  bit0 leaf, bit1 F_out, bit2 F_in, bit3 terminal
 *   colleague  [B][3^dim] int64 same-level neighbours by offset (dx,dy[,dz]),
 *                               lexicographic from (-1,..,-1); -1 if absent
 *   ncoarse    [B]       int32  number of coarse-neighbour leaves
 *   coarse     [B][2^dim-1] int64 coarse-neighbour leaves (first ncoarse valid)
 * Boxes are ordered level by level, in key order within a level (problem
 * index first, then Morton order).
 * Synchronous.
 */
dmk_status dmk_export_tree(dmk_plan_t plan, int64_t *perm, int32_t *level, uint64_t *bkey,
                           int64_t *parent, int64_t *child0, int64_t *pstart, int64_t *pcount,
                           uint8_t *flags, int64_t *colleague, int32_t *ncoarse, int64_t *coarse);

/*
 * dmk_export_near_lists -- the residual interaction lists in gather form:
 * for every leaf holding points, the boxes whose sources act on its targets
 * with the residual kernel of the source box's level.  HOST arrays:
 *   leaf_box  [nleaf]        int64  the target leaves, in list order
 *   offsets   [nleaf+1]      int64  CSR offsets into src_box
 *   src_box   [offsets[nleaf]] int64 source (terminal) boxes
 * Call first with src_box = NULL to learn offsets[nleaf].  Synchronous.
 */
dmk_status dmk_export_near_lists(dmk_plan_t plan, int64_t *leaf_box, int64_t *offsets,
                                 int64_t *src_box);

/*
 * dmk_copy_box_data -- after a dmk_eval on `plan`, copy per-box data of
 * box `box` to the HOST array `out` (p^dim FP64 values, index (i*p + j)*p + k
 * for Chebyshev node indices i, j, k along x, y, z; i*p + j in 2-D).
 *   what = 0: proxy charges (boxes with F_out only);
 *   what = 1: local values of the far potential on the box's Chebyshev grid,
 *             held by the root and by every box with points and F_in (any
 *             other box's far potential is the polynomial of its nearest
 *             such ancestor, by the exactness of Lemma 2.2).
 * Values are in normalised units (root box [-1/2,1/2]^dim; kernel 1/r in
 * 3-D; in 2-D -log(r)/(2 pi) with the root values holding the constant of
 * the unit change); the mixed path's FP32 values are widened to FP64.
 * Returns DMK_ERR_ARG if the box holds no such data.  Synchronous.
 */
dmk_status dmk_copy_box_data(dmk_plan_t plan, int what, int64_t box, double *out);

/*
 * dmk_precompute_probe -- HOST-only view of the tables that Step 1 of
 * Sec. 3.5 builds for a tolerance; no device is touched, so it also runs on
 * machines without a GPU.  x and out are host arrays of n entries.
 *   what = 0: psi_0^c(x_i) / psi_0^c(0) for any real x_i (the PSWF of the
 *             tolerance's c, continued off [-1,1] by the eigen-relation of
 *             the Appendix on PSWFs);
 *   what = 1: g(t_i) = Phi(sqrt t_i)/sqrt t_i for t_i in [0,1], as the
 *             residual stage evaluates it (R_l(r) = 1/r - g(r^2/s_l^2)/s_l);
 *   what = 2: plane-wave weight of D_0 at |m|^2 = x_i (eq.
 *             differencekernelft3 with the factor (h_0/2pi)^3), NaN if no
 *             mode of the table has that |m|^2;
 *   what = 3: plane-wave weight of the windowed W_0 at |m|^2 = x_i;
 *   what = 4: out[0..3] = psi(0), c_0, c_2, lambda_0 (n >= 4, x unused);
 *   what = 5: out[0..5] = c, n_f, p, n_w, h_w, degree of g (n >= 6);
 * 2-D tables (kernel -log(r)/(2 pi), Fourier-space split of Sec. 4.6):
 *   what = 6: plane-wave weight of D_l at |m|^2 = x_i (the same at every
 *             level), NaN if no mode of the table has that |m|^2;
 *   what = 7: plane-wave weight of the windowed W_0 (Sec. 4.7) at |m|^2 = x_i;
 *   what = 8: m(x_i), the smooth part of the residual
 *             R_l(r) = -log(x)/(2 pi) - m(x), x = r/s_l in [0,1];
 *   what = 9: out[0..3] = m(0), n_w, h_w, degree of m (n >= 4).
 * Parameter search (Sec. 3.7 rule for c; smallest n_f and p meeting tol):
 *   what = 10: x[0] = c (0: log(1/tol)); out[0..4] = c, n_f, p and the
 *             plane-wave and proxy errors of those values (n >= 5).
 * 3-D 1/r^2 tables (PSWF power-function split, Sec. 4.5, alpha = 2):
 *   what = 12: g2(t_i) = Phi2(sqrt t_i)/t_i for t_i in [0,1]
 *             (R_l(r) = 1/r^2 - g2(r^2/s_l^2)/s_l^2);
 *   what = 13: plane-wave weight of D_0 at |m|^2 = x_i (level l: 4^l times);
 *   what = 14: plane-wave weight of the windowed root kernel at |m|^2 = x_i.
 * DMK_ERR_UNSUPPORTED for a tolerance outside the table, DMK_ERR_ARG for a
 * bad `what` or n.
 */
dmk_status dmk_precompute_probe(double tol, int what, int64_t n, const double *x, double *out);

/* Stages of dmk_eval, in pipeline order (indices into the arrays of
 * dmk_stage_times and dmk_stage_work). */
enum {
    DMK_STAGE_GATHER = 0,    /* charges into tree order                      */
    DMK_STAGE_UPWARD = 1,    /* proxy charges of F_out boxes (Step 2)        */
    DMK_STAGE_ROOT = 2,      /* windowed kernel W_0 at the root              */
    DMK_STAGE_PROXY2PW = 3,  /* outgoing plane waves (Step 3)                */
    DMK_STAGE_LOCAL = 4,     /* parent -> child local values (Step 3)        */
    DMK_STAGE_PWSHIFT = 5,   /* diagonal translation to colleagues (Step 3)  */
    DMK_STAGE_PW2GRID = 6,   /* incoming plane waves -> local values         */
    DMK_STAGE_LEAF = 7,      /* far potential at leaf targets                */
    DMK_STAGE_RESIDUAL = 8,  /* residual-kernel sums and self term (4-5)     */
    DMK_STAGE_FINALIZE = 9,  /* scaling and scatter to input order           */
    DMK_NSTAGES = 10
};

/*
 * dmk_stage_timing -- enable (1) or disable (0) per-stage HIP events in the
 * following dmk_eval calls of the plan (the per-stage breakdown the paper
 * reports in Table 2).  Enabling resets the totals.
 */
dmk_status dmk_stage_timing(dmk_plan_t plan, int enable);

/*
 * dmk_stage_times -- totals since timing was enabled, per stage: elapsed
 * milliseconds between events recorded on the eval stream before and after
 * each kernel launch (HOST array ms[nstages]) and the number of launches
 * (HOST array launches[nstages]).  Synchronises the plan's last stream.
 */
dmk_status dmk_stage_times(dmk_plan_t plan, double *ms, int64_t *launches, int nstages);

/*
 * dmk_stage_work -- algorithmic work of ONE dmk_eval per stage, from the
 * plan's box and pair counts (HOST arrays of nstages entries): flops (0 for
 * stages bound by memory) and bytes that must cross HBM at least once.
 * The per-unit figures are documented beside the kernels.
 */
dmk_status dmk_stage_work(dmk_plan_t plan, double *flops, double *bytes, int nstages);

/* ------------------------------------------------------------ volume code
 * Continuous sources (Sec. 3.6, "Modification of DMK for continuous
 * sources").  Domain: the unit cube B_0 = [-1/2,1/2]^3 (fixed; no scaling).
 *
 * Tree.  Level-restricted adaptive octree whose leaves carry q x q x q
 * first-kind Chebyshev nodes; leaf B with centre c and side s has node
 * (i, j, k) at c + (s/2) (cos(pi (i+1/2)/q), cos(pi (j+1/2)/q),
 * cos(pi (k+1/2)/q)).  A box is split while its level is below min_level or
 * while the sum of |c_ijk| over the coefficients of the Chebyshev
 * interpolant of rho on its nodes with max(i,j,k) >= q-2 exceeds
 * tol * rho_scale, or while it contains a caller-given feature point whose
 * requested side is below its own (node samples cannot see features much
 * narrower than the node spacing), up to max_level; then the minimal
 * refinement that makes adjacent leaves (face, edge or corner) differ by at
 * most one level.
 * Leaves are ordered by Morton key (x most significant).  Point layout of
 * every node array: leaf-major in that order, node (i, j, k) with k fastest,
 * [npoints] for values, [npoints][3] for coordinates.
 *
 * Split.  1/r = W_0 + sum_{l<L} D_l + R_L with Gaussians (Sec. 3.2, eqs.
 * mlks, kerneldef, deltavalue): sigma_l = 2^-l / sqrt(log(1/tol)).  Proxy
 * charges of a leaf: Gauss-Legendre weights times rho at the Legendre nodes,
 * anterpolated to the parent's Chebyshev grid.  Far field on the anchors'
 * grids, evaluated at the leaf nodes.  Near field: R_L of each source leaf as
 * a sum of Gaussians (Gauss-Legendre in log t from 1/sigma_L to
 * t_a = 2 tol^(-1/6) / s_target), each separable into three q x q matrices
 * per (source, target) pair; Gaussians beyond t_a over R^3 by the expansion
 * rho + Lap rho/(4t^2) + Lap^2 rho/(32 t^4) of the target leaf's polynomial
 * (Sec. 4.4).  That expansion extends rho's polynomial beyond B_0 for nodes
 * within about 3/t_a of the boundary, so densities that do not vanish on the
 * boundary of B_0 carry an error there of the order of that part.
 */

/* density callback: out[i] = rho(xyz[3i], xyz[3i+1], xyz[3i+2]), i < n
 * (HOST arrays, called from the planning thread, in batches of up to all
 * boxes of one level) */
typedef void (*dmk_density_fn)(int64_t n, const double *xyz, double *out, void *ctx);

/*
 * dmk_vol_plan -- build the tree (host, by calls of `density`), then the box
 * structures, lists and tables on the device.
 *  tol        1e-3: the Gaussian split of Sec. 3.2 (p = 18 proxies, 25
 *             plane waves per axis), the residual as a quadrature of
 *             Gaussians in t (Sec. 3.6);
 *             1e-6: the PSWF split of Sec. 3.7 (the point code's 1e-6 far
 *             field, p = 18, 25 plane waves per axis), the residual
 *             (1 - Phi(r/s_L))/r as Gaussians: a quadrature in t from 5/s_L
 *             plus 20 Gaussians fitted to the rest by least squares at plan
 *             time (Sec. 3.6 leaves the construction open), and the same
 *             asymptotic part;
 *             else DMK_ERR_UNSUPPORTED.
 *  q          8 (leaf grid order; else DMK_ERR_UNSUPPORTED).
 *  rho_scale  > 0, the density magnitude the refinement tolerance is
 *             relative to.
 *  min_level  >= 1 (the root is always split), <= max_level.
 *  max_level  <= 19.
 *  nfeat, feat  HOST array feat[nfeat][4] = (x, y, z, h): every box that
 *             contains (x, y, z) (lo <= x < hi per axis) is split while its
 *             side exceeds h > 0; nfeat may be 0 (feat NULL).
 *  opts       precision: DMK_FP64, or DMK_MIXED (the far-field transforms
 *             and the near-field factor products in FP32, the asymptotic
 *             part and the final sums in FP64); flags: DMK_FLAG_LEVEL_LAUNCHES
 *             or DMK_FLAG_QUEUE_LAUNCHES only (others ignored); leaf_max, max_depth, lambda, p, n_f,
 *             pswf_c ignored; NULL for defaults.
 *  stream     for the device work; returns after it completes.
 * The plan holds at most 2^31 - 1 nodes (nleaf q^3).  Free with
 * dmk_plan_destroy.  A volume plan is evaluated with dmk_vol_eval only.
 */
dmk_status dmk_vol_plan(double tol, int32_t q, double rho_scale, int32_t min_level, int32_t max_level,
                        int32_t nfeat, const double *feat, dmk_density_fn density, void *ctx,
                        const dmk_opts *opts, void *stream, dmk_plan_t *out);

/* dmk_vol_info -- number of leaves and of nodes (nleaf q^3) of a volume plan */
dmk_status dmk_vol_info(dmk_plan_t plan, int64_t *nleaf, int64_t *npoints);

/* dmk_vol_leaves -- the leaves (HOST arrays): level[nleaf] and the integer
 * cell ijk[nleaf][3] of each leaf at its level (0 <= ijk < 2^level). */
dmk_status dmk_vol_leaves(dmk_plan_t plan, int32_t *level, int32_t *ijk);

/* dmk_vol_nodes -- node coordinates, DEVICE array xyz[npoints][3] */
dmk_status dmk_vol_nodes(dmk_plan_t plan, double *xyz, void *stream);

/*
 * dmk_vol_eval -- u at every node from rho at every node (DEVICE arrays
 * [npoints], layout above).  far_part / near_part (DEVICE, [npoints], may be
 * NULL) receive the far-field part and the near-field part (sum of Gaussians
 * plus the asymptotic part); u = far_part + near_part.  u may be NULL when a
 * part is requested.  Asynchronous on `stream`.
 */
dmk_status dmk_vol_eval(dmk_plan_t plan, const double *rho, double *u, double *far_part, double *near_part,
                        void *stream);

/* dmk_plan_destroy -- free a plan (NULL is ignored).  Synchronises the
 * plan's last stream first. */
void dmk_plan_destroy(dmk_plan_t plan);

/* dmk_last_error -- message of the last failure on the calling thread. */
const char *dmk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
