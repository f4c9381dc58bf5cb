/*
 * ginimds.h -- C ABI of the Gini MDS library for AMD MI355X (gfx950).
 *
 * The library computes, on one GPU, the data-parallel hot path of Gini
 * multidimensional scaling (arXiv 2605.25124):
 *   - the doubled midranks of the coordinates of a vector (Definition 1 with
 *     the tie rule of Section III-A),
 *   - the matrix of generalised Gini pseudo-distances between all pairs of
 *     rows of a data matrix (Section III-B; the distance-matrix step of
 *     Algorithm 1),
 *   - the raw stress of a latent configuration against that matrix and its
 *     gradient (the SMACOF loss of Section IV-B with unit weights), with the
 *     latent coordinates re-ranked at every evaluation,
 *   - fixed-step gradient-descent fits of many such problems, including a
 *     sweep over nu (Algorithm 1), in one persistent launch.
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers on the context's device unless the
 *     comment says "host".  Matrices are row-major with an explicit leading
 *     dimension (elements between the starts of consecutive rows).
 *   - Calls are asynchronous on the given stream and return once the work is
 *     enqueued, except where the comment says that they synchronise it (the
 *     calls that return host results, gini_autotune, and gini_mds_solve in
 *     its persistent mode or with CHECK_FINITE).  A NULL stream is the null
 *     stream.
 *   - Inputs must be finite.  Ranks compare FP32 values with IEEE < and ==, so
 *     -0 and +0 tie.
 *   - The caller owns every array it passes.  The context owns its scratch
 *     memory and weight tables; it grows scratch on demand, outside any
 *     kernel, and frees everything in gini_destroy.
 *   - Errors: arguments are validated on the host before any GPU work is
 *     enqueued; a failed check returns GINI_EINVAL (or GINI_EUNSUPPORTED) and
 *     enqueues nothing.  gini_last_error(ctx) then describes the failure.
 *     Array arguments must be device memory of the context's GPU (or managed
 *     memory): hipPointerGetAttributes is asked about each, and host memory
 *     or a pointer HIP does not know is refused with GINI_EINVAL.
 *     A HIP runtime failure returns GINI_EDEVICE.
 *   - One context serves one host thread at a time.  Calls on two streams of
 *     one context share its scratch and must not overlap.
 *   - Tracing: every compute entry point opens a ROCTx range named after
 *     itself for the length of the call (host time), which rocprofv3
 *     --marker-trace records beside the kernel trace.
 */
#ifndef GINIMDS_H
#define GINIMDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque HIP stream handle (the same pointer type as hipStream_t). */
typedef struct ihipStream_t* gini_stream_t;

typedef enum {
    GINI_OK = 0,
    GINI_EINVAL = 1,        /* an argument failed validation                 */
    GINI_ENOMEM = 2,        /* device or host allocation failed              */
    GINI_EDEVICE = 3,       /* HIP runtime error, or a device-side failure   */
    GINI_ENOTFINITE = 4,    /* a result was not finite (checked solves only) */
    GINI_EUNSUPPORTED = 5   /* valid but outside what the library supports  */
} gini_status;

/* Distance used between latent points.  GINI: the generalised Gini
 * pseudo-distance of Section III-B over the p latent coordinates (the latent
 * space is a Gini metric space, Section IV-B).  EUCLID: the Euclidean norm
 * used by Algorithm 1 to evaluate the Kruskal stress. */
typedef enum { GINI_LATENT_GINI = 0, GINI_LATENT_EUCLID = 1 } gini_latent;

/* Loss minimised by the descent (Section IV-B lists both).  RAW: the raw
 * stress sum_{i<j} (delta_ij - Delta_ij)^2, the SMACOF loss with unit weights.
 * SAMMON: Sammon's stress sum_{i<j} (delta_ij - Delta_ij)^2 / Delta_ij divided
 * by sum_{i<j} Delta_ij; a pair with Delta_ij = 0 carries no weight. */
typedef enum { GINI_LOSS_RAW = 0, GINI_LOSS_SAMMON = 1 } gini_loss;

typedef struct gini_ctx gini_ctx;

/* Create a context bound to HIP device `device` (>= 0).  No HIP call is made
 * until the first entry point that enqueues work. */
gini_status gini_create(gini_ctx** ctx, int device);
/* Free the context and everything it owns; NULL is a no-op.  Waits for the
 * context's device to finish its outstanding work first. */
void gini_destroy(gini_ctx* ctx);
/* Description of the last failure on this context ("" if none).  The string
 * stays valid until the next call on the context. */
const char* gini_last_error(const gini_ctx* ctx);
/* Static name of a status code. */
const char* gini_status_string(gini_status s);
/* Library version, major*10000 + minor*100 + patch. */
int gini_version(void);

/*
 * gini_weight_table -- host-side table used by every kernel: the weight a
 * coordinate of doubled midrank t receives in the symmetrised generalised
 * Gini pseudo-distance of d-vectors (Section III-B, with the survival function
 * of a coordinate taken as 1 - R/d):
 *     W[t-2] = ((t-2)/(2d))^(nu-1) - ((2d-t)/(2d))^(nu-1),  t = 2 .. 2d,
 * computed in FP64 and rounded once to FP32; exactly antisymmetric,
 * W[2d+2-t] == -W[t].  W: HOST array of 2d-1 floats.  1 <= d <= 65536,
 * nu finite and > 1.  Makes no HIP call; ctx is not needed.
 */
gini_status gini_weight_table(int32_t d, double nu, float* W);

/*
 * gini_rank -- doubled midranks of every row of V (Definition 1; ties share
 * the mean of the ranks they occupy, the rule of Section III-A, so that the zero
 * vector has R = (d+1)/2 everywhere):
 *     twoR[r*ldr + c] = 2*#{c' : V[r,c'] < V[r,c]} + #{c' : V[r,c'] == V[r,c]} + 1
 * V: rows x d FP32, leading dimension ldv >= d.  twoR: rows x d int32,
 * leading dimension ldr >= d.  rows == 0 is a no-op.  1 <= d <= 2^20.
 * Rows of up to 256 coordinates are counted directly (O(d^2) compares, in
 * LDS); longer rows are cut into chunks of 4096 that are sorted on the GPU,
 * and every coordinate's counts come from binary searches in the sorted
 * chunks (O(d log d) per pair of chunks).  The sorted chunks live in the
 * context's scratch (at most 64 MiB; rows are processed in batches).
 * Bit-exact: integer result of FP32 comparisons.
 */
gini_status gini_rank(gini_ctx* ctx, const float* V, int64_t rows, int32_t d, int64_t ldv,
                      int32_t* twoR, int64_t ldr, gini_stream_t stream);

/*
 * gini_dissim -- generalised Gini pseudo-distance between every pair of rows
 * of X (Section III-B, symmetrised form), for each nu in a list, from one
 * ranking of each pair's difference vector:
 *     Delta_k[i, j] = (m/2) * sum_c z_c * W_{m,nu_k}[t_c],   z = fl32(X_i - X_j),
 *     t = doubled midranks of z,
 *     W_{m,nu}[t] = ((t-2)/(2m))^(nu-1) - ((2m-t)/(2m))^(nu-1)
 * which is half the distance from x to y plus half the distance from y to x
 * with the survival function of a coordinate of z taken as 1 - R/m.
 * X: n x m FP32 (ldx >= m).  nu: HOST array of n_nu values, each finite and
 * > 1 (1 <= n_nu <= 64).  Delta: n_nu matrices n x n FP32 (ldd >= n), matrix
 * k starting at Delta + k*stride_nu (stride_nu >= n*ldd when n_nu > 1).
 * The full symmetric matrices are written, with an exact zero diagonal;
 * Delta[j,i] is bitwise equal to Delta[i,j].  n >= 1, 1 <= m <= 4096.
 * FP32 arithmetic with per-lane partial sums; error against an FP64
 * evaluation on the same FP32 differences is below 1e-5 of
 * (m/2)*sum_c |z_c W[t_c]|.
 */
gini_status gini_dissim(gini_ctx* ctx, const float* X, int64_t n, int32_t m, int64_t ldx,
                        const double* nu, int32_t n_nu, float* Delta, int64_t ldd,
                        int64_t stride_nu, gini_stream_t stream);

/*
 * gini_sumsq -- the normaliser of the Kruskal stress (the stress formula that
 * Algorithm 1 evaluates, Section IV-B):
 *     out[2k] + out[2k+1] = sum_{i<j} Delta_k[i, j]^2,   k = 0 .. n_mat-1
 * Delta: n_mat matrices n x n FP32 (ldd >= n), matrix k at Delta + k*stride
 * (stride >= n*ldd when n_mat > 1); only the strict upper triangle is read.
 * out: device float[2*n_mat], (hi, lo) per matrix; n = 1 gives 0.  Each
 * square is split exactly into two FP32 terms and summed with compensation
 * in a fixed order: deterministic.  n >= 1, 1 <= n_mat <= 65535.
 */
gini_status gini_sumsq(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, int32_t n_mat,
                       int64_t stride, float* out, gini_stream_t stream);

/*
 * gini_sum -- the normaliser of the Sammon stress (Section IV-B),
 *     out[2k] + out[2k+1] = sum_{i<j} Delta_k[i, j],
 * with the arguments, layout and ordering of gini_sumsq.
 */
gini_status gini_sum(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, int32_t n_mat, int64_t stride,
                     float* out, gini_stream_t stream);

/*
 * gini_stress_fwd -- raw stress of the configuration Z against Delta (the
 * SMACOF loss of Section IV-B with unit weights, pairs i < j):
 *     sigma = sum_{i<j} (delta(Z_i - Z_j) - Delta[i,j])^2
 * where delta is the latent distance (gini_latent): for GINI the Gini
 * pseudo-distance of the p latent coordinates at the given nu, re-ranked for
 * every pair; for EUCLID the Euclidean norm.  Only the strict upper triangle
 * of Delta is read.
 * Delta: n x n FP32 (ldd >= n).  Z: n x p FP32 (ldz >= p), 1 <= p <= 8
 * (GINI needs p >= 2: the distance of a 1-vector is identically zero).
 * out_sigma: device float[2] receiving (hi, lo), sigma = hi + lo.  n >= 2.
 */
gini_status gini_stress_fwd(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                            float* out_sigma, gini_stream_t stream);

/*
 * gini_stress_bwd -- the same stress and its gradient in ONE pass over Delta:
 *     gradZ[i,:] = scale * d sigma / d Z_i
 *                = scale * sum_{j != i} 2 (delta_ij - Delta_ij) * d delta(Z_i - Z_j) / d Z_i
 * with the latent ranks held fixed (the distance is piecewise linear, so this
 * is its gradient almost everywhere and a subgradient at ties).
 * grad_out: device float scalar multiplying the gradient, or NULL for 1.
 * gradZ: n x p FP32 (ldg >= p), fully overwritten.  out_sigma: as in
 * gini_stress_fwd, or NULL.  Deterministic: fixed reduction order, no
 * floating-point atomics, so repeated calls are bitwise identical.
 */
gini_status gini_stress_bwd(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                            const float* grad_out, float* gradZ, int64_t ldg, float* out_sigma,
                            gini_stream_t stream);

/*
 * gini_stress_bwd_static -- gini_stress_bwd for callers that cannot allocate
 * device memory: work recorded under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, kernels and bitwise
 * results as gini_stress_bwd, but the call allocates nothing (no hipMalloc,
 * hipFree or allocating library call): the tile partials, the descriptor and
 * the stress-slice counter live in one static device array of
 * GINI_STATIC_SCRATCH_BYTES that every GPU the library runs on holds until
 * the process ends; its address is looked up at the first call on a device.
 * That bounds the size: n up to about 36 000 at p = 2 with the Gini latent
 * (one stored gradient component), 26 000 at p = 3 or at p = 2 with the
 * Euclidean latent; a larger problem returns GINI_EUNSUPPORTED with the bytes
 * it needs, before anything is launched.  Every call on one GPU shares that GPU's
 * array, and each call clears what must start at zero: calls that overlap
 * on one GPU (other streams, other host threads) race on it and must be
 * serialised by the caller.  Profiling (gini_profile_enable) does not time it.
 */
#define GINI_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
gini_status gini_stress_bwd_static(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd,
                                   const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                                   const float* grad_out, float* gradZ, int64_t ldg, float* out_sigma,
                                   gini_stream_t stream);

/*
 * gini_sammon_fwd / gini_sammon_bwd -- as gini_stress_fwd / gini_stress_bwd
 * for Sammon's stress (Section IV-B):
 *     sigma = (1 / S) sum_{i<j} (delta_ij - Delta_ij)^2 / Delta_ij,
 *     S = sum_{i<j} Delta_ij = delta_sum[0] + delta_sum[1] (device, gini_sum),
 * pairs with Delta_ij = 0 carry no weight; the gradient holds the latent ranks
 * fixed.  out_sigma receives sigma as (hi, lo).  1 / Delta_ij is the hardware
 * reciprocal (1 ulp).
 */
gini_status gini_sammon_fwd(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, const float* delta_sum,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                            float* out_sigma, gini_stream_t stream);
gini_status gini_sammon_bwd(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, const float* delta_sum,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                            const float* grad_out, float* gradZ, int64_t ldg, float* out_sigma,
                            gini_stream_t stream);

/*
 * gini_sammon_step -- a fixed descent step for the Sammon stress under which
 * it does not increase (Euclidean latent distance, or the p = 2 Gini one):
 *     eta = S / (4 c max_i sum_{j != i, Delta_ij > 0} 1 / Delta_ij),
 * S = sum_{i<j} Delta_ij and c = |d delta / d u|^2 at a tie-free u (as in
 * gini_mds_solve's default step).  2 max_i sum_j w_ij bounds the largest
 * eigenvalue of the weighted Laplacian (Gershgorin), w_ij = 1 / (S Delta_ij),
 * so the step stays inside the quadratic that majorises the stress.  Reads
 * both triangles of Delta (n x n FP32, ldd >= n).  *eta: host.  Synchronises
 * `stream`.
 */
gini_status gini_sammon_step(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, int32_t p, double nu,
                             gini_latent latent, double* eta, gini_stream_t stream);

/* One MDS instance for gini_mds_solve (all pointers are device pointers). */
typedef struct {
    int64_t n;             /* points, >= 2                                     */
    int32_t p;             /* latent dimension, 1..8 (>= 2 for GINI)           */
    int32_t loss;          /* gini_loss; RAW or SAMMON (shared by one call)   */
    const float* Delta;    /* n x n dissimilarities (upper triangle read)      */
    int64_t ldd;           /* >= n                                             */
    float* Z;              /* n x p configuration, updated in place            */
    int64_t ldz;           /* >= p                                             */
    double nu;             /* > 1, used by the GINI latent distance            */
    gini_latent latent;
    float eta;             /* step; <= 0 selects 1 / (2 n c) (see below); the
                              SAMMON loss needs eta > 0 (gini_sammon_step)    */
    float* sigma_hist;     /* iters floats: sigma(Z_t) before step t; or NULL  */
    const float* delta_sumsq; /* (hi, lo) from gini_sumsq of this Delta, or
                                 NULL; needed only by ks_hist                 */
    float* ks_hist;        /* iters floats: Kruskal stress
                              sqrt(sigma(Z_t) / sum_{i<j} Delta_ij^2); or NULL
                              (RAW loss only)                                 */
    const float* delta_sum;   /* (hi, lo) from gini_sum of this Delta; needed
                                 by the SAMMON loss, else ignored              */
} gini_instance;

enum {
    GINI_SOLVE_PERSISTENT = 1,   /* all instances, all iterations, one launch   */
    GINI_SOLVE_PLAIN = 2,        /* per instance, per iteration: 2 launches     */
    GINI_SOLVE_BATCHED = 4,      /* per iteration: 2 launches for all instances */
    GINI_SOLVE_AUTOTUNE = 8,     /* choose tile, grid and mode by measurement   */
    GINI_SOLVE_CHECK_FINITE = 16, /* return GINI_ENOTFINITE if a sigma is not   */
    GINI_SOLVE_SPLIT = 32,       /* with BATCHED: two groups on two streams     */
    GINI_SOLVE_CALLER_ORDER = 64 /* queue the instances in the caller's order,
                                    not largest first                          */
};

typedef struct {
    int32_t iters;     /* >= 0                                                  */
    int32_t flags;     /* one of PERSISTENT / PLAIN / BATCHED, or AUTOTUNE;
                          plus CHECK_FINITE; SPLIT only together with BATCHED   */
    int32_t tile;      /* 0 = library choice, else 64, 128 or 256               */
    int32_t grid;      /* PERSISTENT: workgroups of the launch; PLAIN and
                          BATCHED: threads of a reduction workgroup, 256 or
                          1024 (results do not depend on it); 0 = library
                          choice                                                */
} gini_solve_opts;

/*
 * gini_mds_solve -- the MDS fit of Algorithm 1: for every instance, iters
 * fixed steps of gradient descent on the raw stress,
 *     sigma_hist[t] = sigma(Z_t),   Z_{t+1} = Z_t - eta * grad sigma(Z_t),
 * with default eta = 1 / (2 n c), c = |d delta / d u|^2 at a tie-free u
 * (c = 1 for EUCLID, where the step is the Guttman transform of SMACOF plus
 * a translation; c = 2 * 4^(1-nu) for GINI at p = 2).
 * inst: HOST array of n_inst descriptors (1 <= n_inst <= 65536).  Instances
 * must not share Z, sigma_hist or ks_hist; an instance with ks_hist needs
 * delta_sumsq, and ks_hist[t] = sqrt(sigma_hist[t] / (delta_sumsq[0] +
 * delta_sumsq[1])) is formed in FP64 from the compensated sigma (0 when the
 * normaliser is 0).  BATCHED | SPLIT deals the instances (largest first) into
 * two groups of about equal work and issues each group's launches on its own
 * stream (`stream`, and a stream the context owns, made to wait for each
 * other at the start and the end of the call), so that the reduction of one
 * group runs beside the stress units of the other; with one instance it is
 * plain BATCHED.  Work units and reduction blocks are queued instance by
 * instance, largest n first (CALLER_ORDER: in the order of `inst`).  All modes
 * and orders give bitwise identical results for the same tile size (every
 * instance's sums have a fixed shape).  PLAIN and BATCHED return
 * once their work is enqueued on `stream` (Z and the histories are complete
 * when `stream` reaches that point); PERSISTENT, and any call with
 * CHECK_FINITE, synchronise `stream` before returning, to report device-side
 * failures: a persistent launch that stops making progress aborts and returns
 * GINI_EDEVICE.  A context's calls must be ordered: on one stream, or the
 * caller orders the streams (they share the context's scratch).
 */
gini_status gini_mds_solve(gini_ctx* ctx, const gini_instance* inst, int32_t n_inst,
                           const gini_solve_opts* opts, gini_stream_t stream);

/*
 * gini_autotune -- time candidate (mode, tile, grid) choices for this batch of
 * instances over `probe_iters` iterations each, on copies of the
 * configurations (the caller's Z and histories are not modified), and write
 * the fastest into *best (flags keep the caller's CHECK_FINITE bit).  The
 * candidates are the batched mode at every tile size (when there are several
 * instances also with SPLIT and with CALLER_ORDER; each with reduction
 * workgroups of 256 and 1024 threads), and the persistent mode at several
 * grid sizes only where one iteration has no more work units than the GPU has
 * compute units (elsewhere its per-unit release costs more than two launches
 * per iteration).  The
 * result is cached in the context, keyed by the batch's shape, and used by
 * gini_mds_solve with GINI_SOLVE_AUTOTUNE.  Synchronises `stream`.
 */
gini_status gini_autotune(gini_ctx* ctx, const gini_instance* inst, int32_t n_inst,
                          int32_t probe_iters, gini_solve_opts* best, gini_stream_t stream);

/* Options of gini_select_nu. */
typedef struct {
    int32_t iters;         /* descent steps of every (nu, fold) fit, >= 1    */
    int32_t p;             /* latent dimension, as in gini_instance          */
    gini_latent latent;    /* latent distance of the fit (GINI: Section IV-B) */
    int32_t folds;         /* K >= 1; fold f holds rows [f*n/K, (f+1)*n/K)   */
    int32_t flags;         /* launch mode, as gini_solve_opts.flags          */
    int32_t tile;          /* 0 = library choice, else 64, 128 or 256        */
} gini_select_opts;

/*
 * gini_select_nu -- Algorithm 1 (optimised Gini MDS) in one call.  For every
 * nu of the list and every fold: the Gini dissimilarities of the fold's rows
 * (gini_dissim; one ranking per pair serves every nu), `iters` descent steps
 * from the fold's rows of Z0 (gini_mds_solve, all nu x folds fits batched
 * together), then the Kruskal stress of the fitted configuration with the
 * Euclidean latent distance, the statistic Algorithm 1 compares:
 *     KS = sqrt( sum_{i<j} (|Z_i - Z_j|_2 - Delta_ij)^2 / sum_{i<j} Delta_ij^2 ).
 * The mean KS over the folds picks nu* = argmin (the first on ties).
 * X: n x m FP32 (ldx >= m), 1 <= m <= 4096.  nu: HOST array of n_nu values
 * (1 <= n_nu <= 64), each finite and > 1.  Z0: n x p FP32 (ldz0 >= p).
 * Z_out: n_nu configurations n x p (ldzo >= p), configuration k at
 * Z_out + k*stride_z (stride_z >= n*ldzo when n_nu > 1); the rows of fold f
 * are fitted against fold f only.  ks_mean: HOST double[n_nu]; ks_fold: HOST
 * double[n_nu*folds] (nu-major) or NULL; best: HOST int32, the index of nu*.
 * Every fold needs at least two rows (n >= 2*folds).  The dissimilarities
 * live in a context-owned device workspace of
 * sum_f n_nu * n_f * ceil64(n_f) floats, grown on demand.  Synchronises
 * `stream`.
 */
gini_status gini_select_nu(gini_ctx* ctx, const float* X, int64_t n, int32_t m, int64_t ldx, const double* nu,
                           int32_t n_nu, const float* Z0, int64_t ldz0, const gini_select_opts* opts,
                           float* Z_out, int64_t ldzo, int64_t stride_z, double* ks_mean, double* ks_fold,
                           int32_t* best, gini_stream_t stream);

/* Options of gini_alternate_nu. */
typedef struct {
    int32_t iters;         /* Sammon descent steps per round, >= 1           */
    int32_t p;             /* latent dimension                               */
    gini_latent latent;    /* latent distance of the fit                     */
    int32_t rounds;        /* alternations T >= 1                            */
    int32_t init;          /* index in the nu list of the first nu fitted    */
    int32_t flags;         /* launch mode, as gini_solve_opts.flags          */
    int32_t tile;          /* 0 = library choice, else 64, 128 or 256        */
} gini_alternate_opts;

/*
 * gini_alternate_nu -- the alternation of Algorithm 2 (Section V-C): starting
 * from nu = nu[init] and the configuration Z0, every round
 *   1. takes `iters` descent steps on the Sammon stress at the current nu,
 *      from the configuration the previous round left (gini_sammon_step's
 *      step for that nu's dissimilarities);
 *   2. scores the configuration against every nu of the list by the Kruskal
 *      stress with the Euclidean latent distance (no refit), and
 *   3. moves to the nu with the smallest score.
 * The dissimilarities of every nu come from one gini_dissim call (one
 * ranking per pair) into the context's workspace (n_nu * n * ceil64(n)
 * floats).  X: n x m FP32 (ldx >= m), n >= 2.  nu: HOST array of n_nu values
 * (1 <= n_nu <= 64).  Z0, Z_out: n x p FP32 (ldz0, ldzo >= p); Z_out holds the
 * last round's fit.  nu_hist: HOST int32[rounds], the index fitted in each
 * round; ks: HOST double[rounds * n_nu] (round-major), the scores after each
 * round's fit, or NULL; best: HOST int32, the argmin after the last round.
 * Synchronises `stream`.
 */
gini_status gini_alternate_nu(gini_ctx* ctx, const float* X, int64_t n, int32_t m, int64_t ldx, const double* nu,
                              int32_t n_nu, const float* Z0, int64_t ldz0, const gini_alternate_opts* opts,
                              float* Z_out, int64_t ldzo, int32_t* nu_hist, double* ks, int32_t* best,
                              gini_stream_t stream);

/*
 * gini_classical_mds -- classical MDS (Section IV-A) of a dissimilarity
 * matrix, e.g. as the starting configuration of the descent: the p
 * eigenpairs of B = -1/2 H D^2 H (D^2 the entrywise squares of Delta,
 * H = I - 11^T/n) with the largest eigenvalues, Z = V_p diag(sqrt(max(lam, 0))).
 * B is never formed: subspace iteration on a block of q = min(8, p + 4, n - 1)
 * centred vectors applies it as one pass over the rows of Delta (both
 * triangles read, diagonal skipped), with a Rayleigh-Ritz step per iteration;
 * it stops when the p largest Ritz values move by at most tol of the largest
 * (or after max_iters).  The start block is fixed, so results repeat.
 * Delta: n x n FP32 (ldd >= n), n >= 2.  1 <= p <= min(8, n - 1).  Z: n x p
 * FP32 (ldz >= p), device.  eigvals: HOST double[p] (decreasing) or NULL;
 * iters_done: HOST int32 or NULL.  The columns of Z are determined up to sign.
 * Uses the context's workspace; synchronises `stream`.
 */
gini_status gini_classical_mds(gini_ctx* ctx, const float* Delta, int64_t n, int64_t ldd, int32_t p,
                               int32_t max_iters, double tol, float* Z, int64_t ldz, double* eigvals,
                               int32_t* iters_done, gini_stream_t stream);

/*
 * gini_standardize -- the preprocessing of the simulations of Section V-C:
 * every column of X is centred to zero median and scaled to unit variance,
 *     Y[i, c] = (X[i, c] - median_c) / sd_c,
 * median_c the middle order statistic (the mean of the two middle ones for
 * even n, found exactly), sd_c the population standard deviation about the
 * mean (a constant column is only centred).  The dissimilarities depend on
 * differences of rows only, so only the scaling changes them.  X, Y: n x m
 * FP32 (ldx, ldy >= m); Y may be X (then ldy == ldx).  stats: device
 * float[2m], (median, sd) per column, or NULL.  n >= 1, m >= 1.
 */
gini_status gini_standardize(gini_ctx* ctx, const float* X, int64_t n, int32_t m, int64_t ldx, float* Y,
                             int64_t ldy, float* stats, gini_stream_t stream);

/* Kernel timing collected by the context while profiling is enabled: HIP
 * events recorded on the launching stream around each stress-tile launch,
 * each reduction launch and each persistent launch. */
typedef struct {
    int64_t tile_launches;
    double tile_ms;          /* summed durations of the stress-tile kernels */
    int64_t reduce_launches;
    double reduce_ms;
    int64_t persistent_launches;
    double persistent_ms;
    int64_t dissim_launches;
    double dissim_ms;
} gini_profile;

/* Start (enable != 0) or stop recording kernel timings; clears the totals. */
gini_status gini_profile_enable(gini_ctx* ctx, int enable);
/* Wait for the recorded events, return the totals and clear them. */
gini_status gini_profile_read(gini_ctx* ctx, gini_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* GINIMDS_H */
