/*
 * mlmc.h -- C ABI of the MI355X (gfx950) library for the multilevel Monte
 * Carlo estimator of E[AB] and E[x^T y] by uniform-probability sketching
 * (Wu & Polydorides, "A Multilevel Monte Carlo Estimator for Matrix
 * Multiplication", arXiv:1904.00429).
 *
 * The problem (Sec. 3): A (m x n) and B (n x p) are random matrices with
 * known entry laws; n is large.  Estimate E[AB] (more generally E[f(AB)],
 * f entrywise: see mlmc_func) by
 *   Y = sum_{l=0}^{L} Ybar_l                                      (eq. (10))
 *   Ybar_l = (1/N_l) sum_k (Z_l^(k) - Z_{l-1}^(k)),  Ybar_0 = mean_k Z_0^(k)   (eq. (9))
 * where Z_l^(k) = (n / c_l) sum_{t < c_l} A^(k)[:, r_t] B^(k)[r_t, :] is the
 * sketch of eq. (18) with uniform probabilities (eq. (4)) over c_l indices
 * drawn with replacement, and Z_{l-1}^(k) reuses c_{l-1} of the same indices
 * of the same realisation A^(k), B^(k) (Alg. 1).  The coarse sketch takes the
 * first c_{l-1} indices.  N_l is given, or chosen by eq. (28) (Remark 3.6)
 * for a target RMSE.  The inner product (Sec. 2) is the m = p = 1 case.
 *
 * Conventions for every entry point:
 *   - All device pointers are allocated by the caller; the library never
 *     allocates device memory.  Scratch comes in through `workspace`, whose
 *     size in bytes is given by the matching *_workspace_size call.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *     it.  A call returns after enqueueing, except that the target-RMSE mode
 *     and a non-NULL `report` synchronise the stream (the scheduler and the
 *     report need level statistics on the host).
 *   - No exception crosses the ABI.  A non-zero mlmc_status is returned and a
 *     thread-local message is available from mlmc_last_error().  On MLMC_EINVAL
 *     and MLMC_EWORKSPACE nothing has been enqueued.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`.
 *     Index draw t of realisation k at level l uses counter
 *     (t/2, k, 0, 1<<28 | l<<20 | problem); element e of the column vector
 *     [A^(k)[:, j]; B^(k)[j, :]] uses word e%4 of counter
 *     (e/4, k, j, 2<<28 | l<<20 | problem).  With MLMC_FLAG_SHARED_SAMPLES
 *     every level uses l = 0xFF (realisations and indices shared by all
 *     levels; for testing the telescoping identity).
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLMC_OK = 0,
    MLMC_EINVAL = 1,      /* invalid argument (sizes, ladder, null pointer, mode) */
    MLMC_EDEVICE = 2,     /* a HIP runtime call failed */
    MLMC_EBUDGET = 3,     /* the scheduled sum_l N_l c_l exceeds max_total_draws */
    MLMC_EWORKSPACE = 4   /* workspace missing or smaller than required */
} mlmc_status;

typedef enum {
    MLMC_LAW_NORMAL = 0,  /* loc + scale * N(0, 1), i.i.d. entries */
    MLMC_LAW_UNIFORM = 1, /* loc + scale * U(-1, 1), i.i.d. entries */
    MLMC_LAW_REPARAM = 2, /* mean + stdev (entrywise) * N(0, 1) */
    /* The laws of the experiments of Sec. 4, independent entries whose law
     * depends on the column j (counted from 1); K ~ Poisson(loc),
     * E ~ Exp(1), z, z' ~ N(0, 1), u ~ U(0, 1).  Both operands take one of
     * them or neither does (EINVAL); not with FP8 operands (EINVAL).
     * Element e of column j of realisation k draws its own Philox call,
     * counter (e, k, j, 3 << 28 | level << 20 | problem), with uniforms
     * u0, u1, u2: z = sqrt(-2 ln u0) cos(2 pi u1), z' the sine half; K the
     * smallest integer with P(Poisson <= K) >= u0 (CDF summed term by term
     * from exp(-loc)); E = -ln u1; the mask is u2 < scale (4) or u1 < scale
     * (6).  Evaluated in FP64 in every precision. */
    MLMC_LAW_RAMP_NORMAL = 3,     /* (j scale)(loc - z): Sec. 4.1's x (scale 1/50, loc 0.4) */
    MLMC_LAW_COS_POISSON_EXP = 4, /* cos(K + 2E) [u < scale]: Sec. 4.1's y (loc 10, scale 0.05);
                                     loc in (0, 500], scale in [0, 1] */
    MLMC_LAW_SIN_RAMP = 5,        /* sin(x) + z' x, x = (j scale)(loc - z): Sec. 4.2's A
                                     (scale 1e-4, loc 0.5) */
    MLMC_LAW_COS_POISSON_STEP = 6 /* cos(K) H(5 - K) [u < scale]: Sec. 4.2's B (loc 2,
                                     scale 0.2); loc in (0, 500], scale in [0, 1] */
} mlmc_law;

typedef enum {
    MLMC_PREC_FP64 = 0,   /* values, products and sums in FP64 */
    MLMC_PREC_FP32 = 1,   /* values and contraction in FP32, statistics FP64 */
    MLMC_PREC_BF16 = 2,   /* gathered operands BF16 (RNE), FP32 accumulation (MFMA) */
    MLMC_PREC_FP8 = 3     /* gathered operands OCP FP8 e4m3 (RNE, saturated at +-448), FP32
                             accumulation on v_mfma_scale_f32_32x32x64_f8f6f4: every row i of A
                             and column q of B is multiplied by a power of two 2^s before its
                             rounding, s the largest exponent with 2^s bound <= 256 (clamped to
                             [-20, 20]), where bound = fma(6, |scale|, |loc|) (normal),
                             |loc| + |scale| (uniform), or the maximum over the n columns of
                             fma(6, |stdev|, |mean|) (reparameterised, per row / column); the
                             MFMA's E8M0 operand scales undo the factors */
} mlmc_prec;

/* Target function f (Sec. 3): the estimate is of E[f(AB)] (E[f(x^T y)] for
 * the inner product), f applied entrywise to both sketches of every
 * realisation, so the level sample is D = f(Z_l) - f(Z_{l-1}) (f(Z_0) at
 * level 0).  H is the Heaviside step, read as H(0) = 1. */
typedef enum {
    MLMC_FUNC_IDENTITY = 0,     /* f(x) = x */
    MLMC_FUNC_ABS_STEP = 1,     /* f(x) = |x| H(theta0 - x)                (Sec. 4.2: theta0 = 2) */
    MLMC_FUNC_INV_ABS_STEP = 2  /* f(x) = 1 / (|x| H(x + theta0) + theta1) (Sec. 4.1: theta0 = 0.4,
                                   theta1 = 0.01); theta1 > 0 */
} mlmc_func;

#define MLMC_FLAG_SHARED_SAMPLES 1u
#define MLMC_FLAG_TIMING 2u       /* time every kernel launch with HIP events on `stream` */
/* Adaptive number of levels (Alg. 2's loop over L; target mode, single-product
 * entry points): c[] is the longest ladder allowed.  Levels are added one at a
 * time; a new level first runs pilot_samples realisations, then eq. (28) over
 * the levels so far gives every N_l and each level is extended to
 * max(N_l, its realisations so far), reusing them.  From three levels on the
 * loop stops once the finest level mean Ybar_L passes the bias test:
 * ||Ybar_L||_F < (sqrt(M) + 1) eps / sqrt(2) (matrix, Remark 3.5, eq. (27)) or
 * |Ybar_L| < (sqrt(M) - 1) eps / sqrt(2) (inner product, Sec. 2, eq. (15)),
 * M = c[L] / c[L-1].  Levels never reached report N_l = 0 and add nothing. */
#define MLMC_FLAG_ADAPTIVE_LEVELS 4u
/* Stride coupling (Sec. 3.1): the coarse sketch of level l >= 1 takes every
 * M-th of the c_l fine draws, r_{jM} for j = 1 .. c_{l-1} (0-based draws
 * M - 1, 2M - 1, ...), M = c_l / c_{l-1}, as the paper writes it.  Without
 * the flag it takes the first c_{l-1} draws (prefix coupling).  Both subsets
 * give level samples of the same law (the draws are i.i.d.); only the prefix
 * nests the levels, so with shared realisations only the prefix makes the
 * telescoping sum exact.  Every entry point accepts it, the batched ones
 * included. */
#define MLMC_FLAG_STRIDE_COUPLING 8u
/* Index draws from 32-bit words (inner product only, n a power of two,
 * uniform draws, laws 0-2): draw t takes word t % 4 of the index-stream call
 * (t / 4, k, 0, 1 << 28 | level << 20 | problem) and r = floor(w n / 2^32),
 * the top log2 n bits of w: exactly uniform, four draws per Philox call
 * instead of two.  A different stream from the default 64-bit draws, so
 * the estimates differ realisation by realisation (not in law).  EINVAL
 * otherwise. */
#define MLMC_FLAG_INDEX_WORD32 16u
/* Values from 16-bit uniforms (matrix products, batched included, and the
 * adjoint, which regenerates the forward's values; laws 0-2): element e of column j takes half (e & 1: high, else
 * low) of word (e / 2) % 4 of the value-stream call (e / 8, k, j,
 * 2 << 28 | level << 20 | problem), u = (h + 1/2) 2^-16, so one Philox call
 * gives eight values instead of four; normals by Box-Muller on the two halves
 * of a word (pairs (e & ~1, e | 1) as in the default stream).  The normal is
 * then truncated at 4.85 standard deviations (variance low by about 1e-5
 * relative, mean exact by symmetry).  EINVAL otherwise. */
#define MLMC_FLAG_VALUE16 32u
/* Set form of every realisation (the note after Alg. 1 in Sec. 3.1: the
 * index tuple (r_1, ..., r_{c_l}) mapped to a set of distinct indices with
 * multiplicities): before the gather, each realisation's distinct indices
 * are counted (coarse draws and the others apart) and each distinct column
 * of A^(k) and row of B^(k) is generated once, at the first position that
 * drew it, weighted by the sum of the weights of its draws; the repeats stay
 * zero.  The estimate equals the default tuple form up to the order of the
 * sums, and a realisation generates at most min(c_l, n) columns.  Matrix
 * products (batched included), FP64 or FP32 operands, f = identity, uniform
 * index draws; EINVAL otherwise.  The contraction still runs over all c_l
 * positions. */
#define MLMC_FLAG_SET_FORM 64u
#define MLMC_MAX_LEVELS 32

/* Kernel classes of mlmc_report.kernel_ms (MLMC_FLAG_TIMING). */
#define MLMC_KERNEL_SAMPLE 0      /* level sampling: inner-product level kernel, matrix sketch kernel */
#define MLMC_KERNEL_GATHER 1      /* generation of the sampled columns (matrix product) */
#define MLMC_KERNEL_MERGE 2       /* merge of partial statistics into the level state */
#define MLMC_KERNEL_FINAL 3       /* level variances, telescoping sum, resets */
#define MLMC_KERNEL_CLASSES 4

/* Entry law of A (m x n) or B (n x p).  For MLMC_LAW_REPARAM, `mean` and
 * `stdev` are FP32 device arrays: for A column-major (entry (i, j) at
 * j*ld + i, ld >= m), for B row-major (entry (j, q) at j*ld + q, ld >= p);
 * for the inner product x and y are vectors (ld ignored, entry j at j). */
typedef struct {
    int32_t law;          /* mlmc_law */
    double loc;
    double scale;
    const float* mean;
    const float* stdev;
    int64_t ld;
} mlmc_dist;

/* The level ladder and the sampling mode (Alg. 2 with a fixed finest level).
 *   c[l]: indices per realisation at level l (host array, num_levels entries);
 *         c[0] >= 1, c[l] an integer multiple >= 2 of c[l-1], c_L < 2^31
 *         (inner product), c_L < 2^28 (matrix products and the adjoint).
 *   Fixed mode: n_samples[l] = N_l >= 1 (host array), rmse_target = 0.
 *   Target mode: n_samples = NULL, rmse_target = eps > 0 (total Frobenius
 *         RMSE: E||Y - E[AB]||_F^2 <= eps^2); pilot_samples >= 2 realisations
 *         per level estimate V_l, eq. (28) gives N_l, each level is extended
 *         to max(N_l, pilot_samples) reusing the pilot realisations.
 *   max_total_draws: 0, or a cap on sum_l N_l c_l (MLMC_EBUDGET if exceeded;
 *         checked before the extension is enqueued). */
typedef struct {
    int32_t num_levels;
    const int64_t* c;
    const int64_t* n_samples;
    double rmse_target;
    int64_t pilot_samples;
    int64_t max_total_draws;
    uint64_t seed;
    int32_t prec;         /* mlmc_prec */
    uint32_t flags;       /* MLMC_FLAG_* */
    uint32_t problem;     /* stream id < 2^20 (independent problems, same seed) */
    int32_t func;         /* mlmc_func; 0 (identity) when the struct is zero-initialised */
    double func_param[2]; /* theta0, theta1 of f (finite) */
    /* Index probabilities (eq. (18) with a general xi): NULL for uniform
     * draws, or a device array of n integer weights w_j >= 1 with
     * xi_j = w_j / W, W = sum_j w_j < 2^64 (mlmc_optimal_index_weights gives
     * Theorem 3.1's xi**).  Draw t uses the same 64-bit word x as the
     * uniform draw: T = floor(x W / 2^64) and r_t is the smallest j with
     * w_0 + ... + w_j > T (all weights 1 give the uniform draw); the sketch
     * weighs draw t by 1 / (c_l xi_{r_t}).  Single-product entry points
     * (matrix, inner product, adjoint) with FP64, FP32 or BF16 operands. */
    const uint32_t* index_weights;
} mlmc_levels;

/* Filled when a non-NULL report is passed (synchronises the stream). */
typedef struct {
    int64_t n_used[MLMC_MAX_LEVELS];     /* N_l actually used */
    double level_var[MLMC_MAX_LEVELS];   /* V_l: vectorised variance of one level sample */
    double rmse_est;                     /* sqrt(sum_l V_l / N_l) */
    int64_t total_draws;                 /* sum_l N_l c_l */
    double kernel_ms[MLMC_KERNEL_CLASSES];        /* MLMC_FLAG_TIMING: summed device time */
    int64_t kernel_launches[MLMC_KERNEL_CLASSES]; /* MLMC_FLAG_TIMING: launches per class */
    int32_t levels_used;                 /* levels run (num_levels unless adaptive) */
    int32_t bias_test_passed;            /* adaptive: 1 if the loop stopped on the bias test */
} mlmc_report;

/* Bytes of device workspace needed by mlmc_matmul_estimate / inner product. */
size_t mlmc_matmul_workspace_size(int64_t m, int64_t n, int64_t p, const mlmc_levels* levels);
size_t mlmc_inner_product_workspace_size(int64_t n, const mlmc_levels* levels);

/* MLMC estimate of E[f(AB)] (Sec. 3, Alg. 1 and Alg. 2; f = levels->func,
 * the identity by default).
 *   out:         device FP64, m x p row-major, receives Y = sum_l Ybar_l.
 *   level_means: NULL, or device FP64 (num_levels x m x p) receiving Ybar_l.
 * Errors: EINVAL (m, n, p < 1; n >= 2^32; bad ladder; bad mode; null
 * pointers; reparam without mean/stdev; unknown f or non-finite or
 * out-of-range f parameters), EWORKSPACE, EBUDGET, EDEVICE. */
mlmc_status mlmc_matmul_estimate(int64_t m, int64_t n, int64_t p, const mlmc_dist* A,
                                 const mlmc_dist* B, const mlmc_levels* levels, double* out,
                                 double* level_means, void* workspace, size_t workspace_bytes,
                                 mlmc_report* report, void* stream);

/* MLMC estimate of E[f(x^T y)] for random x, y of length n (Sec. 2; the
 * m = p = 1 case of the matrix estimator).  out: device FP64 scalar.
 * level_means: NULL or device FP64 [num_levels].  prec: FP64 or FP32.
 * Errors as above. */
mlmc_status mlmc_inner_product_estimate(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                        const mlmc_levels* levels, double* out,
                                        double* level_means, void* workspace,
                                        size_t workspace_bytes, mlmc_report* report,
                                        void* stream);

/* ---- Allocation-free inner product -----------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The same estimate as mlmc_inner_product_estimate (same
 * arguments, modes and results, bit for bit), with its workspace taken from a
 * fixed device array of MLMC_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends (its address is looked up once
 * per device, on the first call there).  The caller still passes the output
 * (and level_means).  Nothing is allocated: no hipMalloc, hipFree or torch
 * allocation.
 *   Limit: the workspace the estimate needs must fit the array; it does for
 *   any n and ladder with uniform draws (about 0.2 MB); weighted draws add
 *   8 n bytes (n up to about 4.9e5).  Beyond it: MLMC_EINVAL.
 *   Every call on one GPU shares that GPU's array and leaves the last call's
 *   contents in it (each call clears what must start at zero); calls that
 *   overlap on one GPU (concurrent streams or threads) race and give wrong
 *   results.  Errors: as mlmc_inner_product_estimate, plus EINVAL above the
 *   limit and EDEVICE if the array's address cannot be obtained. */
#define MLMC_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
size_t mlmc_inner_product_noalloc_limit(void);
mlmc_status mlmc_inner_product_estimate_noalloc(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                                const mlmc_levels* levels, double* out,
                                                double* level_means, mlmc_report* report,
                                                void* stream);

/* ---- Batching --------------------------------------------------------------
 * Many independent products of uneven shapes through one pipeline: every pass
 * gathers the sampled columns of all products in one launch, one persistent
 * sketch launch walks all (product, output tile, group of realisations) work
 * items, and one launch merges the statistics of all products.  The products
 * share the ladder, N_l (fixed mode), seed, precision and flags; each has its
 * own shape, laws, Philox stream id and outputs. */
typedef struct {
    int64_t m, n, p;
    mlmc_dist A, B;
    uint32_t problem;     /* Philox stream id < 2^20 (distinct per product) */
    double* out;          /* device FP64 m x p: Y */
    double* level_means;  /* NULL or device FP64 (num_levels x m x p) */
} mlmc_problem;

/* Launch shape (all zero = defaults; chosen by the autotuner of the Python
 * package): tile = workgroup output tile edge (64 or 128; FP64 uses 64),
 * target_blocks = sketch work items per pass, gather_budget = bytes of
 * gathered operands per pass.  single_launch = 1: the whole estimate (every
 * pass of every level) in one persistent kernel, whose step p gathers pass p
 * into one of three buffers and sketches pass p - 1 from another, its work
 * claimed from per-XCD queues, the sketch of each step behind a bounded
 * grid-wide barrier (workspace: three gather buffers); built for FP32, BF16
 * and FP8 operands, i.i.d. normal or uniform laws, f = identity, and
 * products in whole tiles at tile 64 or of any shape at tile 128 (other
 * tables, and 0, take a gather, a sketch and a merge launch per pass).  It
 * gives the same estimate as the launch-per-pass form with one realisation
 * group per pass.  Its
 * workgroups must all be resident at once: its grid is the device's resident
 * capacity for it, and a barrier that waits past ten seconds makes every
 * output NaN (and the call EDEVICE when it reads level_var). */
typedef struct {
    int32_t tile;
    int64_t target_blocks;
    int64_t gather_budget;
    int32_t single_launch;
} mlmc_tuning;

size_t mlmc_matmul_batched_workspace_size(int32_t nprob, const mlmc_problem* probs,
                                          const mlmc_levels* levels, const mlmc_tuning* tuning);
/* level_var: NULL, or host FP64 [num_levels x nprob] (level-major) receiving
 * V_l of every product (synchronises the stream).  The call synchronises the
 * stream once to upload the product table.  Errors as mlmc_matmul_estimate;
 * EINVAL also for nprob < 1, target mode, duplicate stream ids. */
mlmc_status mlmc_matmul_estimate_batched(int32_t nprob, const mlmc_problem* probs,
                                         const mlmc_levels* levels, const mlmc_tuning* tuning,
                                         void* workspace, size_t workspace_bytes, double* level_var,
                                         void* stream);

/* The same batched estimate captured once into a hipGraph (reset, every pass
 * of every level, finalize) and replayed by mlmc_graph_launch on any stream.
 * The workspace, the outputs and the law arrays must stay valid while the
 * graph exists; each launch recomputes the estimate with the captured seed. */
typedef struct mlmc_graph_s* mlmc_graph;
mlmc_status mlmc_matmul_batched_graph_create(int32_t nprob, const mlmc_problem* probs,
                                             const mlmc_levels* levels, const mlmc_tuning* tuning,
                                             void* workspace, size_t workspace_bytes, void* stream,
                                             mlmc_graph* graph);
mlmc_status mlmc_graph_launch(mlmc_graph graph, void* stream);
mlmc_status mlmc_graph_destroy(mlmc_graph graph);

/* One inner-product estimate (Sec. 2; fixed N_l, or target mode: the pilot,
 * eq. (28) and the extension, all on the device) captured into a hipGraph
 * and replayed by mlmc_graph_launch, with no host synchronisation inside:
 * replays back to back pay one graph launch per estimate instead of the
 * direct call's launches and its readback.  Arguments as
 * mlmc_inner_product_estimate; out, level_means, the workspace and the
 * index weights must stay valid while the graph exists, and each replay
 * recomputes the estimate with the captured seed into out and level_means.
 * The schedule's N_l, V_l and status stay in the workspace: read them with
 * mlmc_inner_product_graph_report.  Errors as mlmc_inner_product_estimate;
 * EINVAL also for a NULL graph or stream, MLMC_FLAG_ADAPTIVE_LEVELS (Alg. 2's
 * bias test runs on the host) and MLMC_FLAG_TIMING. */
mlmc_status mlmc_inner_product_graph_create(int64_t n, const mlmc_dist* x, const mlmc_dist* y,
                                            const mlmc_levels* levels, double* out,
                                            double* level_means, void* workspace,
                                            size_t workspace_bytes, void* stream,
                                            mlmc_graph* graph);
/* After a replay of that graph on `stream`: synchronises the stream, reads
 * V_l (and in target mode N_l and the schedule's status) from the workspace
 * into *report (NULL: status only) and returns the status the direct call
 * would have returned: EBUDGET when eq. (28) asked for more realisations
 * than the counter range or more draws than max_total_draws, EDEVICE for a
 * device error.
 * n, levels and the workspace are the ones the graph was created with. */
mlmc_status mlmc_inner_product_graph_report(int64_t n, const mlmc_levels* levels,
                                            const void* workspace, size_t workspace_bytes,
                                            mlmc_report* report, void* stream);

/* ---- Differentiation ------------------------------------------------------
 * Adjoint of mlmc_matmul_estimate for reparameterised laws A = M_A + S_A o Z,
 * B = M_B + S_B o W (both MLMC_LAW_REPARAM).  Y = sum_l Ybar_l is bilinear in
 * the sampled columns, so for G = dL/dY
 *   dL/da_t = kappa_t G b_t,  dL/db_t = kappa_t G^T a_t,
 *   kappa_t = (n / c_l) w_t / N_l  (w_t = 1 - c_l / c_{l-1} for the first c_{l-1}
 *   draws of level l >= 1, else 1; Alg. 1 with the prefix coupling),
 * and dM_A[:, r_t] += dL/da_t, dS_A[:, r_t] += dL/da_t o z_t (likewise for B).
 * The indices and normals of every realisation are regenerated from the seed
 * exactly as the forward drew them; nothing of the forward is stored.
 *   levels:   the forward's ladder, seed, problem and flags, in fixed mode
 *             (pass the forward report's n_used after a target-RMSE call).
 *   grad_out: device FP64, m x p row-major, dL/dY.
 *   dMA, dSA: device FP32 in the layout of A's mean/stdev (column-major m x n,
 *             ld = A->ld); dMB, dSB: layout of B's (row-major n x p, ld = B->ld).
 *             Gradients are ADDED; zero them first.  No atomics: the draws
 *             of each batch of realisations are sorted by column (a stable
 *             radix sort) and each column's terms are summed in draw order
 *             by one owner, so a call gives the same bits on every run.
 *             Calls that overlap on the same gradient arrays race.
 * Arithmetic (levels->prec): MLMC_PREC_FP32 — FP32 values, FP32 MFMA
 * contraction and accumulation; MLMC_PREC_BF16 — the regenerated values and
 * G rounded to BF16 (nearest even), BF16 MFMA, FP32 accumulation and FP32
 * gradients.  Other precisions: MLMC_EINVAL.
 * Workspace (mlmc_matmul_adjoint_workspace_size, with the same levels,
 * n_samples included): G in the contraction's layouts plus the buffers of
 * one pass of draws (the draws of all levels are taken in passes of as many
 * as fit): room for every draw of the call, capped at 4 GiB (about 0.95 M
 * draws of a 512 x 512 problem).  A smaller workspace also works, down to
 * the buffers of a 64-draw pass (more passes; EWORKSPACE below that, the
 * message giving both sizes); the summation order, and so the last bits,
 * follow the passes.
 * Errors: EINVAL (laws not reparameterised, target mode, f other than the
 * identity, precision other than FP32/BF16, null pointers, and the
 * conditions of mlmc_matmul_estimate), EWORKSPACE, EDEVICE. */
size_t mlmc_matmul_adjoint_workspace_size(int64_t m, int64_t n, int64_t p, const mlmc_levels* levels);
mlmc_status mlmc_matmul_adjoint_reparam(int64_t m, int64_t n, int64_t p, const mlmc_dist* A,
                                        const mlmc_dist* B, const mlmc_levels* levels,
                                        const double* grad_out, float* dMA, float* dSA, float* dMB,
                                        float* dSB, void* workspace, size_t workspace_bytes,
                                        void* stream);

/* ---- Building blocks, exported for testing ------------------------------ */

/* Philox4x32-10 (SC'11) of `count` counters: ctr and out are device arrays of
 * 4*count uint32; key = (seed mod 2^32, seed >> 32). */
mlmc_status mlmc_philox4x32_10(int64_t count, const uint32_t* ctr, uint64_t seed, uint32_t* out,
                               void* stream);

/* Index draws of realisations k0 .. k0+num_samples-1 (uniform on [0, n),
 * eq. (4)), as the estimators draw them: out is device int32,
 * num_samples x c row-major.  level_field is l, or 0xFF for shared mode. */
mlmc_status mlmc_sample_indices(uint64_t seed, uint32_t problem, uint32_t level_field,
                                uint32_t k0, int64_t num_samples, int64_t c, int64_t n,
                                int32_t* out, void* stream);

/* The sampled columns a_t = A^(k)[:, r_t] and rows b_t = B^(k)[r_t, :] as the
 * matrix estimator generates them, converted to FP64: AS is device
 * num_samples x c x m, BS is num_samples x c x p (row-major).  prec selects
 * the generator's arithmetic (FP64, or FP32 / BF16 values widened to FP64). */
mlmc_status mlmc_gather_columns(int64_t m, int64_t n, int64_t p, const mlmc_dist* A,
                                const mlmc_dist* B, uint64_t seed, uint32_t problem,
                                uint32_t level_field, uint32_t k0, int64_t num_samples,
                                int64_t c, int32_t prec, double* AS, double* BS, void* stream);

/* Theorem 3.1's xi** (eq. (20)), proportional to
 * sqrt(E||A_{:,j}||^2 E||B_{j,:}||^2), as integer weights for
 * mlmc_levels.index_weights: s_j = sqrt(EA_j) sqrt(EB_j) with
 * EA_j = sum_i (mean_ij^2 + stdev_ij^2) accumulated in FP64 for i = 0, 1, ...
 * (mean's square first), EB_j likewise over row j of B, and
 * w_j = max(1, floor(2^24 s_j / max_i s_i)).  For i.i.d. laws every column
 * has the same moments and w_j = 2^24.  weights: device uint32[n];
 * scratch: device, at least (n + 1) doubles (reparameterised laws).
 * Errors: EINVAL (sizes, null pointers, mixed law kinds, the laws of
 * Sec. 4). */
mlmc_status mlmc_optimal_index_weights(int64_t m, int64_t n, int64_t p, const mlmc_dist* A,
                                       const mlmc_dist* B, uint32_t* weights, double* scratch,
                                       void* stream);

/* Index draws with probabilities w_j / W, as the estimators draw them with
 * mlmc_levels.index_weights; cum: device uint64[n] scratch that receives the
 * cumulative weights.  Other arguments as mlmc_sample_indices. */
mlmc_status mlmc_sample_indices_weighted(uint64_t seed, uint32_t problem, uint32_t level_field,
                                         uint32_t k0, int64_t num_samples, int64_t c, int64_t n,
                                         const uint32_t* weights, uint64_t* cum, int32_t* out,
                                         void* stream);

const char* mlmc_status_string(mlmc_status status);
const char* mlmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_H */
