/*
 * edaa.h -- C ABI of the MI355X (gfx950) library for Entropic Descent
 * Archetypal Analysis (EDAA, arXiv 2209.11002).
 *
 * The library minimises the archetypal-analysis objective
 *      1/2 || X - X B A ||_F^2
 * over A (p x N, every column on the simplex Delta_p) and B (N x p, every
 * column on Delta_N) with the alternating entropic (mirror) steps of the
 * paper's Algorithm 1, runs ensembles of seeded runs and selects one with the
 * paper's Algorithm 2.
 *
 * Conventions shared by every call
 *   - Arrays are row-major C arrays.  X is [L][N] (one pixel per column,
 *     element (l, i) at l*N + i), A is [p][N], B is [N][p], E = X B is [L][p].
 *     Ensemble outputs stack runs first: A_all [M][p][N], B_all [M][N][p],
 *     E_all [M][L][p].
 *   - Pointers documented "device" are device memory of the context's GPU;
 *     "host" pointers are ordinary host memory.  The caller allocates and owns
 *     every input and output; the context owns (and reuses) its workspace.
 *   - Work is enqueued on the stream given to edaa_create.  A call that fills
 *     a host array synchronises that stream before it returns.
 *   - A context is not thread safe: use one context per host thread/stream.
 *   - Errors: every call validates its arguments before enqueuing anything
 *     and returns EDAA_EINVAL (nothing enqueued) on a bad one; the message is
 *     available from edaa_last_error() on the calling thread.  A HIP runtime
 *     failure returns EDAA_EDEVICE and poisons the context (later calls on it
 *     return EDAA_EDEVICE).
 *   - Sizes: 1 <= p <= 16, p <= N, 1 <= L <= 448, N < 2^31 / (M p).
 */
#ifndef EDAA_H
#define EDAA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct edaa_ctx edaa_ctx;

typedef enum {
    EDAA_OK = 0,
    EDAA_EINVAL = -1,        /* invalid argument; nothing was enqueued          */
    EDAA_ENOMEM = -2,        /* device workspace could not be allocated         */
    EDAA_EDEVICE = -3,       /* HIP runtime error; the context is poisoned      */
    EDAA_ENUMERIC = -4,      /* non-finite result (every run of an ensemble)    */
    EDAA_EUNSUPPORTED = -5   /* valid request outside what the library supports */
} edaa_status;

enum { EDAA_X_F32 = 0, EDAA_X_BF16 = 1 };                   /* storage type of X      */
enum { EDAA_COHERENCE_COSINE = 0, EDAA_COHERENCE_RAW = 1 }; /* reading of eq. coherence */
enum {
    EDAA_FLAG_GRAPH = 1,     /* record the whole run sequence in a HIP graph once
                                per (shape, buffers) and replay it afterwards */
    EDAA_FLAG_TIME_PASSES = 2, /* record HIP events around every A-pass, B-pass
                                and closing-pass launch (eager launches only;
                                see edaa_pass_times) */
    EDAA_FLAG_RAGGED_GROUPED = 4, /* edaa_fit_ragged: run every image with one
                                launch per kernel and group of equal p instead
                                of the persistent kernel */
    EDAA_FLAG_BF16_WIDEN = 8 /* bf16 X (edaa_fit, edaa_ensemble, edaa_abundances,
                                edaa_fit_noalloc): widen X tiles to float32 and
                                run the A- and B-passes on the float32 (and, for
                                the projection of the A-pass, float64) matrix
                                cores, instead of the default bf16 matrix-core
                                passes (X stays bf16; the float32 operand in
                                three bf16 terms) */,
    EDAA_FLAG_F32_MFMA = 16 /* float32 X (edaa_fit, edaa_ensemble,
                                edaa_fit_noalloc): run the B-pass contractions
                                on the float32 matrix cores instead of the
                                default bf16 ones, where both float32 operands
                                are split exactly into three bf16 terms and the
                                six products above float32 rounding are summed
                                (the two agree to float32 rounding, not bit for
                                bit) */
};

/* Parameters of Algorithm 1 / Algorithm 2.  edaa_default_params fills the
 * paper's values: T = 100, K1 = K2 = 5 (Section "Implementation details",
 * paragraph "Hyperparameters"), gamma = 1 (an element of the set S of
 * eq. eta0A), init_scale = 0.1 (eq. initB0), select_threshold = 1.05
 * (Algorithm 2). */
typedef struct {
    int T, K1, K2;           /* outer iterations, A-steps and B-steps per outer  */
    double gamma;            /* eta1 = gamma / sigma_max^2(X B0), eq. eta0A      */
    double eta1, eta2;       /* > 0: explicit step sizes (resume, tests);
                                0: the paper's rule (eq. eta0A, eq. eta0B)       */
    double init_scale;       /* B0 = column softmax(init_scale * U), eq. initB0  */
    double select_threshold; /* Algorithm 2: keep fit_m <= threshold * fit_min   */
    int x_dtype;             /* EDAA_X_F32 or EDAA_X_BF16                        */
    int coherence_mode;      /* EDAA_COHERENCE_COSINE (default) or _RAW          */
    int flags;               /* EDAA_FLAG_*                                      */
    int runs_per_chunk;      /* launch shape: runs that share one pass over an X
                                tile (0: tuned or default; else one of the
                                compiled sizes, EDAA_EUNSUPPORTED otherwise)    */
    int pixel_groups;        /* launch shape: workgroups per chunk of runs
                                (0: tuned or default; capped at ceil(N / 64))    */
    int tiles_per_item;      /* edaa_fit_ragged: 64-pixel tiles per work item of
                                the persistent kernel (0: tuned or default 8)   */
} edaa_params;

/* One image of a ragged batch (edaa_fit_ragged).  All pointers are device
 * pointers with the layouts above; loss_trace is a host array of T+1. */
typedef struct {
    const void* X;           /* [L][N], l2-normalised, dtype params->x_dtype     */
    int L, N, p;
    uint64_t seed;           /* B0 draw, see edaa_fit                             */
    double gamma;
    float* A;                /* out [p][N]                                        */
    float* B;                /* out [N][p]                                        */
    float* E;                /* out [L][p], may be NULL                           */
    double* loss_trace;      /* out, host, T+1 values, may be NULL               */
    int pixel_groups;        /* in: work items (pixel groups) per pass, 0 for
                                the default; out: the number used             */
} edaa_image_desc;

/* Launch shape of a batched problem (edaa_plan). */
typedef struct {
    int runs_per_chunk;      /* runs sharing each pass over an X tile            */
    int chunks;              /* ceil(M / runs_per_chunk)                         */
    int pixel_groups;        /* workgroups per chunk (each strides over tiles)   */
    int double_buffer;       /* 1: the next X tile loads while one is processed  */
    int source;              /* EDAA_PLAN_DEFAULT, _TUNED or _REQUESTED          */
    int bf16_passes;         /* passes on the bf16 matrix cores: bit 0 the B-pass,
                                bit 1 the A-pass (bf16 X tiles; float32 X with
                                its operands in three bf16 terms, where a chunk
                                has at least two column blocks of 16 runs x
                                endmembers); 0: the float32 (and float64)
                                matrix-core passes                            */
} edaa_launch_plan;
enum { EDAA_PLAN_DEFAULT = 0, EDAA_PLAN_TUNED = 1, EDAA_PLAN_REQUESTED = 2 };

/* Fill *params with the paper's defaults (see edaa_params). */
void edaa_default_params(edaa_params* params);

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL
 * for the device's null stream).  *out receives the context. */
edaa_status edaa_create(edaa_ctx** out, int device, void* stream);

/* Release the context and its workspace (no-op on NULL). */
void edaa_destroy(edaa_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* edaa_last_error(void);

/* Environment: EDAA_TUNE_CACHE (see edaa_autotune); EDAA_REDUCE_ROWS = 1..4
 * sets the rows of X B each workgroup of the B-step reduction forms (by
 * default four where a chunk's rows outnumber the CUs, else one; every
 * choice gives the same bits). */

/* The launch shape edaa_fit (M = 1) or edaa_ensemble (M runs) would use for
 * an L x N image with p endmembers under params (its runs_per_chunk and
 * pixel_groups requests, else a tuned shape, else the default).  Pure host
 * function, needs no context or device.  EDAA_EINVAL for bad sizes,
 * EDAA_EUNSUPPORTED when no compiled pass kernels fit the request. */
edaa_status edaa_plan(int L, int N, int p, int M, const edaa_params* params, edaa_launch_plan* out);

/* Launch-shape autotuner.  Times candidate shapes of an ensemble of M runs
 * of p endmembers on X [L][N] (device, params->x_dtype): every compiled
 * runs-per-chunk size that fits, each with half, the default and twice the
 * default pixel groups (multiples of 8, which keep the workgroups sharing an
 * X tile on one XCD) and the count that gives one workgroup per CU; each
 * candidate runs T = 2 and T = 6 outer iterations
 * (K1, K2 from params, seeds 0..M-1, gamma params->gamma) twice after a
 * warm-up, and scores the difference of the best times.  The fastest shape is recorded for the
 * problem's class (L, p, M, x_dtype and ceil(log2(ceil(N / 64)))): later
 * edaa_fit / edaa_ensemble / edaa_plan calls of that class without an
 * explicit runs_per_chunk or pixel_groups use it (plan source
 * EDAA_PLAN_TUNED).  Records live for the process and, if the environment
 * variable EDAA_TUNE_CACHE names a file, are appended to it and read back by
 * later processes.  best (may be NULL) receives the shape, best_us (may be
 * NULL) its microseconds per outer iteration.  Allocates its trial outputs;
 * synchronises the stream. */
edaa_status edaa_autotune(edaa_ctx* ctx, const void* X, int L, int N, int p, int M,
                          const edaa_params* params, edaa_launch_plan* best, double* best_us);

/* The same for a ragged batch: tiles per work item of the persistent kernel
 * (1, 2, 4, ..., 128), timed on the batch itself (the images' outputs are
 * overwritten), recorded for the batch's class (image count,
 * ceil(log2(total tiles)), largest p, x_dtype) and used by later
 * edaa_fit_ragged calls of that class with params->tiles_per_item = 0. */
edaa_status edaa_autotune_ragged(edaa_ctx* ctx, int n_images, edaa_image_desc* images,
                                 const edaa_params* params, int* best_tiles_per_item,
                                 double* best_us);

/* Capacity of the context's cache of captured HIP graphs (EDAA_FLAG_GRAPH),
 * one per (shape, buffers, parameters) key; the least recently captured is
 * dropped when it is full.  Default 16; n >= 1. */
edaa_status edaa_set_graph_cache(edaa_ctx* ctx, int n);

/* Number of kernel launches the last edaa_fit / edaa_ensemble call enqueued
 * (graph replays count the kernels inside the graph). */
long long edaa_last_launch_count(edaa_ctx* ctx);

/* Durations of the pass kernels of the last edaa_fit / edaa_ensemble call made
 * with EDAA_FLAG_TIME_PASSES, from HIP events recorded on the launch stream
 * immediately before and after each launch.  Timing applies to eager launches
 * only: a call that also sets EDAA_FLAG_GRAPH records nothing (count 0).
 * kind: 0 A-pass, 1 B-pass, 2 closing pass.
 * *count receives the number of launches of that kind, *total_ms their summed
 * durations.  Synchronises the context stream. */
edaa_status edaa_pass_times(edaa_ctx* ctx, int kind, int* count, double* total_ms);

/* Per-pixel l2 normalisation of the paper's eq. normalization:
 * x_i <- x_i / ||x_i||_2 for every column i of X_in [L][N] (device, float32).
 * The result goes to X_out (device, [L][N], dtype out_dtype; X_out may equal
 * X_in when out_dtype is EDAA_X_F32).  A pixel of zero norm is written as
 * zeros; if n_zero (host) is not NULL it receives their number and the call
 * synchronises. */
edaa_status edaa_normalize_pixels(edaa_ctx* ctx, const float* X_in, void* X_out,
                                  int L, int N, int out_dtype, int* n_zero);

/* One EDAA run (Algorithm 1) on l2-normalised X [L][N] (device, dtype
 * params->x_dtype).
 *   A0, B0   optional starting points (device, [p][N] and [N][p]; NULL selects
 *            eq. initA0 and eq. initB0).  B0 from the seed is
 *            softmax_columns(init_scale * u) with u[i][j] the Philox4x64-10
 *            draw (Salmon et al., SC'11): word j%4 of the block for counter
 *            (i, j/4, 0, 0) and key (seed, 0), mapped to [0,1) as
 *            (word >> 40) * 2^-24.
 *   A, B     out (device): final abundances [p][N] and pixel weights [N][p].
 *   E        out (device, may be NULL): endmembers X B, [L][p].
 *   loss_trace out (host, may be NULL): T+1 values, loss_trace[0] is
 *            1/2||X - X B0 A0||^2 and loss_trace[t] the objective after outer
 *            iteration t.
 *   eta_out  out (host, may be NULL): {eta1, eta2} used.
 * Returns EDAA_ENUMERIC if the final objective is not finite. */
edaa_status edaa_fit(edaa_ctx* ctx, const void* X, int L, int N, int p,
                     const edaa_params* params, uint64_t seed,
                     const float* A0, const float* B0,
                     float* A, float* B, float* E,
                     double* loss_trace, double* eta_out);

/* edaa_fit for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same run on the same kernels, with every intermediate in a fixed 256 MiB
 * device array that the library holds on each GPU until the process ends,
 * and no host transfer.  It calls no hipMalloc, hipFree or other allocating
 * routine.  Differences from edaa_fit:
 *   loss_trace_dev  out (device, float64, T+1 values, may be NULL)
 *   eta_dev         out (device, float64, {eta1, eta2}, may be NULL)
 *   params->flags   must not hold EDAA_FLAG_GRAPH or EDAA_FLAG_TIME_PASSES.
 * Returns EDAA_EUNSUPPORTED (nothing enqueued) when the run needs more than
 * the 256 MiB (about L * N * 4 bytes for the padded copy of X plus the run's
 * state, e.g. L = 224 with N up to about 250 000).  Nothing is synchronised.
 * All calls on one GPU share that array: two calls whose work overlaps in
 * time on one GPU (different streams or host threads) race and corrupt each
 * other; calls ordered on one stream are safe.  Each call initialises every
 * part of the array it reads. */
edaa_status edaa_fit_noalloc(edaa_ctx* ctx, const void* X, int L, int N, int p,
                             const edaa_params* params, uint64_t seed,
                             const float* A0, const float* B0,
                             float* A, float* B, float* E,
                             double* loss_trace_dev, double* eta_dev);

/* M runs of Algorithm 1 on the same X, all advanced together (one pass over
 * X serves every run), then the l1 fit ||X - E_m A_m||_1 (entrywise), the
 * coherence mu_m of E_m (eq. coherence, reading params->coherence_mode) and
 * the selection of Algorithm 2 (edaa_select).
 *   seeds, gammas  host arrays of M: run m draws B0 from seeds[m] (see
 *                  edaa_fit) and uses gamma gammas[m].
 *   A_all, B_all   out (device) [M][p][N], [M][N][p].
 *   E_all          out (device, may be NULL) [M][L][p].
 *   loss           out (host, may be NULL) [M][T+1].
 *   fit, mu        out (host, may be NULL) [M].
 *   run_status     out (host, may be NULL) [M]: EDAA_OK or EDAA_ENUMERIC.
 *   selected       out (host, may be NULL): selected run, -1 if none.
 * Returns EDAA_ENUMERIC when no run has a finite objective. */
edaa_status edaa_ensemble(edaa_ctx* ctx, const void* X, int L, int N, int p,
                          const edaa_params* params, int M,
                          const uint64_t* seeds, const double* gammas,
                          float* A_all, float* B_all, float* E_all,
                          double* loss, double* fit, double* mu,
                          int* run_status, int* selected);

/* Independent EDAA runs (Algorithm 1) on n_images images of different
 * (L, N, p), all advanced together.  Images with p <= 9 run in one persistent
 * launch: the passes of every image are cut into work items (a pixel group
 * of params->tiles_per_item 64-pixel tiles, a block of band rows of a
 * reduction, ...) that the resident workgroups take in a fixed order, each
 * item starting once its image has finished the items it depends on, so
 * images advance through their outer iterations independently.  Images with
 * p > 9 (and every image under EDAA_FLAG_RAGGED_GROUPED) run with one launch
 * per kernel and group of equal p.  Each image's results equal those of
 * edaa_fit with params->pixel_groups set to that image's pixel_groups.
 * params->T, K1, K2, init_scale and x_dtype apply to every image; gamma and
 * seed come from each descriptor, which also receives pixel_groups.
 * Synchronises the stream.  EDAA_EDEVICE if a wait of the persistent kernel
 * exceeds its bound (a fault of the schedule; the kernel still ends). */
edaa_status edaa_fit_ragged(edaa_ctx* ctx, int n_images, edaa_image_desc* images,
                            const edaa_params* params);

/* Abundance estimation with the endmembers given: minimise
 * 1/2 ||X - E A||_F^2 over A [p][N] with every column on the simplex (the
 * non-negativity and sum-to-one constraints of abundance estimation once the
 * endmembers are known, as the paper's Introduction states it) by the
 * entropic A-steps of eq. update_A with E in place of X B: params->T outer
 * iterations of params->K1 steps (K2 is ignored), step eta1 = gamma /
 * sigma_max^2(E) (the rule of eq. eta0A applied to E) unless params->eta1 > 0.
 *   X          [L][N], dtype params->x_dtype (device)
 *   E          [L][p] float32 (device), the given endmembers
 *   A0         [p][N] start (device) or NULL for eq. initA0 (1/p)
 *   A          out [p][N] float32 (device)
 *   loss_trace out, host, T+1 objectives (loss[0] at A0), may be NULL
 *   eta_out    out, host, 2 values (eta1 and sqrt(p/N) eta1), may be NULL
 * Errors as edaa_fit. */
edaa_status edaa_abundances(edaa_ctx* ctx, const void* X, int L, int N, int p,
                            const edaa_params* params, const float* E, const float* A0,
                            float* A, double* loss_trace, double* eta_out);

/* Objective 1/2||X - X B A||_F^2 (eq. AA) for X [L][N] float32, A [p][N],
 * B [N][p] (all device); the float32 result is written to loss_dev (device,
 * one float). */
edaa_status edaa_loss_fwd(edaa_ctx* ctx, const float* X, const float* A, const float* B,
                          int L, int N, int p, float* loss_dev);

/* Gradients of grad_out * 1/2||X - X B A||^2 (the derivatives that eq. update_A
 * and eq. update_B step along, with the opposite sign):
 *   gA = grad_out * (X B)^T (X B A - X)          [p][N] (device)
 *   gB = grad_out * X^T (X B A - X) A^T          [N][p] (device)
 * grad_out is a device float (the incoming gradient of the loss). */
edaa_status edaa_loss_bwd(edaa_ctx* ctx, const float* X, const float* A, const float* B,
                          int L, int N, int p, const float* grad_out,
                          float* gA, float* gB);

/* Mirror step of eq. update_softmax on every column of A [p][N] (device, in
 * place): a <- softmax(log a - eta gA) over the p entries of the column. */
edaa_status edaa_mirror_step_A(edaa_ctx* ctx, float* A, const float* gA, int p, int N, float eta);

/* Mirror step on every column of B [N][p] (device, in place):
 * b_j <- softmax(log b_j - eta gB_j) over the N entries of column j. */
edaa_status edaa_mirror_step_B(edaa_ctx* ctx, float* B, const float* gB, int N, int p, float eta);

/* Algorithm 2 selection on host arrays of M values: fit_min over finite fits,
 * I = {m : fit[m] <= threshold * fit_min}, returns argmin over I of mu (lowest
 * index on ties, a finite mu beats NaN), or -1 if no fit is finite.  Pure host
 * function, needs no context. */
int edaa_select(const double* fit, const double* mu, int M, double threshold);

#ifdef __cplusplus
}
#endif

#endif /* EDAA_H */
