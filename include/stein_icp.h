/*
 * stein_icp.h -- C ABI of the MI355X (gfx950) Stein-ICP library.
 *
 * Stein ICP (Afzal Maken, Ramos, Ott, arXiv:2106.03287) approximates the
 * posterior over a six-DoF pose theta = (x, y, z, roll, pitch, yaw) that maps
 * a source cloud S onto a reference cloud R by K particles. One iteration
 * (the procedure closing Sec. IV):
 *   1. every particle transforms the same minibatch of m source points
 *      (SGD-ICP minibatch, Sec. III-B),
 *   2. each transformed point is matched to its nearest reference point by
 *      brute force (Eq. 1),
 *   3. each particle takes the mean point-to-point gradient (Eqs. 4-5),
 *   4. the particles are coupled by the Stein direction of Eq. 16 with an
 *      RBF translation kernel and the wrapped-angle rotation kernel of
 *      Eq. 17, bandwidths by the median heuristic (Sec. V),
 *   5. every particle is moved along it (Eq. 12) by Adam (Sec. V).
 *
 * Conventions shared by every entry point:
 *  - Points are FP32 metres, row-major n x 3 (x, y, z), in DEVICE memory.
 *  - Particles are FP64, row-major K x 6 (x, y, z in m; roll, pitch, yaw in
 *    rad), DEVICE memory. Particle theta maps a source point s to
 *    Rz(yaw) Ry(pitch) Rx(roll) s + (x, y, z).
 *  - A minibatch schedule is int32 rows x m in DEVICE memory; the iteration
 *    whose step count (completed updates) is t uses row t mod rows.
 *  - `hip_stream` is a hipStream_t (NULL = the default stream). Calls that
 *    are not marked blocking only enqueue work on it.
 *  - Every function returns STEIN_ICP_OK or a negative status. On failure
 *    the context is left as it was (all validation precedes any enqueue) and
 *    stein_icp_last_error() describes the cause.
 *  - The caller owns every pointer it passes; the library copies what it
 *    keeps. The context owns its device buffers until stein_icp_destroy.
 *  - Contexts are not thread-safe: one thread (or stream) drives a context.
 */
#ifndef STEIN_ICP_H
#define STEIN_ICP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STEIN_ICP_OK 0
#define STEIN_ICP_E_INVALID (-1) /* bad argument, non-finite input, bad schedule */
#define STEIN_ICP_E_NOMEM (-2)   /* device allocation failed */
#define STEIN_ICP_E_DEVICE (-3)  /* a HIP call failed (message has the HIP error) */
#define STEIN_ICP_E_STATE (-4)   /* call not valid in the context's state */

/* Nearest-neighbour search (Eq. 1). FP32: exact squared distances in FP32
 * (dx, dy, dz in FP32, d = fma(dz,dz, fma(dy,dy, dx*dx))), lowest index on
 * ties. BF16_RERANK: the same answer, found faster: candidates screened by
 * |a|^2 + |b|^2 - 2 a.b on BF16 matrix cores with FP32 accumulation (centred
 * coordinates split into three BF16 parts), the best re-ranked with the FP32
 * distance above, and every answer certified against a bound on the screen's
 * error; a query whose certificate fails is searched again in FP32. Far from
 * the centroid the bound widens and more queries take the FP32 path.
 * F16_RERANK: the same certified screen with the centred coordinates scaled
 * by a power of two and split into two FP16 parts (FP16's 11-bit significand
 * carries in two parts what BF16 needs three for): one matrix product per
 * block of references instead of two, with an error bound of the same size.
 * All three modes return the same answers. */
enum { STEIN_ICP_NN_FP32 = 0, STEIN_ICP_NN_BF16_RERANK = 1, STEIN_ICP_NN_F16_RERANK = 2 };
/* Update rule: Adam on -phi (Sec. V), or theta += lr * phi (Eq. 12). */
enum { STEIN_ICP_OPT_ADAM = 0, STEIN_ICP_OPT_SGD = 1 };
/* Kernel bandwidth: median heuristic h = med^2 / ln K over the K(K-1)/2
 * distances between distinct particles (mean of the two middle values for an
 * even count; h = 1 when K = 1 or med = 0), or fixed values. */
enum { STEIN_ICP_BW_MEDIAN = 0, STEIN_ICP_BW_FIXED = 1 };
/* Prior: uniform (zero gradient, as in the paper's experiments), or Gaussian
 * translation (Eq. 14, variance prior_var_trans) and von Mises rotation
 * (Eq. 15, concentration prior_kappa_rot) around prior_mu. */
enum { STEIN_ICP_PRIOR_UNIFORM = 0, STEIN_ICP_PRIOR_GAUSS_VONMISES = 1 };
/* ICP error metric of the gradient. POINT: Eqs. 4-5, e = R s + u - r.
 * PLANE: point-to-plane (the metric of the paper's quantitative results,
 * Sec. V; cited to Chen and Medioni in Sec. II): matches still by Eq. 1,
 * e replaced by its projection rho n on the unit normal n of the matched
 * reference (rho = n^T e), i.e. the gradient of (1/2m) sum rho^2. Normals
 * are computed at init: the eigenvector of the smallest eigenvalue of the
 * FP64 covariance of each reference point's normal_k nearest references
 * (itself included, FP32 distances as in Eq. 1, ties to the lower index);
 * zero where the smallest and middle eigenvalues lie within 1e-10 of the
 * trace of each other (no unique plane). The sign of a normal is not
 * defined; the gradient does not depend on it. */
enum { STEIN_ICP_METRIC_POINT = 0, STEIN_ICP_METRIC_PLANE = 1 };

typedef struct stein_icp_config {
    uint32_t struct_size;    /* sizeof(stein_icp_config): ABI version check */
    int32_t num_particles;   /* K, 1 <= K <= 1024 */
    int32_t batch_size;      /* m, 1 <= m <= every source size */
    int32_t schedule_rows;   /* rows of the minibatch schedule, >= 1 */
    double lr;               /* step size (> 0) */
    double beta1, beta2;     /* Adam, in [0, 1) */
    double eps;              /* Adam, > 0 */
    uint64_t seed;           /* library-drawn initial particles / schedule */
    double init_half_trans;  /* library-drawn init: centre +- half (m) */
    double init_half_rot;    /* ... (rad) */
    double init_centre[6];
    int32_t nn_mode;         /* STEIN_ICP_NN_* */
    int32_t optimizer;       /* STEIN_ICP_OPT_* */
    int32_t bandwidth_mode;  /* STEIN_ICP_BW_* */
    int32_t prior_mode;      /* STEIN_ICP_PRIOR_* */
    double fixed_h_trans;    /* used when bandwidth_mode == FIXED (> 0) */
    double fixed_h_rot;
    double prior_mu[6];
    double prior_var_trans[3];  /* > 0 */
    double prior_kappa_rot[3];  /* >= 0 */
    int64_t n_scale;         /* N multiplying the mean gradient (Eq. 16); 0 = source size */
    int32_t use_graph;       /* 1: stein_icp_step replays captured hipGraphs */
    int32_t autotune;        /* 1: time candidate NN tile shapes at init and keep the best */
    int32_t metric;          /* STEIN_ICP_METRIC_* */
    int32_t normal_k;        /* neighbours per normal (PLANE), 3 <= normal_k <= 32 */
} stein_icp_config;

typedef struct stein_icp_ctx stein_icp_ctx;

/* Fill `cfg` with the defaults: K 100, m 300, schedule_rows 1, lr 0.01,
 * beta1 0.9, beta2 0.999, eps 1e-8, seed 0, init +-0.2 m / +-pi/4 around 0,
 * FP32 search, Adam, median bandwidth, uniform prior, n_scale 0, graphs on,
 * autotune off, point-to-point metric, normal_k 10. */
void stein_icp_default_config(stein_icp_config *cfg);

/* Create a context for one cloud pair. Blocking: packs the clouds into the
 * library's layout, checks them (finite, |coordinate| <= 1e9), checks the
 * schedule (indices in [0, n_src)), computes the initial rotations, and
 * synchronises `hip_stream` before returning.
 *   src_xyz, n_src: device FP32 n_src x 3 source cloud S.
 *   ref_xyz, n_ref: device FP32 n_ref x 3 reference cloud R (n_ref < 2^31 - 64).
 *   init_particles: device FP64 K x 6, or NULL to draw them from cfg->seed
 *                   (uniform in init_centre +- half widths).
 *   schedule:       device int32 cfg->schedule_rows x m, or NULL to draw rows
 *                   from cfg->seed (m distinct indices per row).
 * On success *out owns the context. */
int stein_icp_init(stein_icp_ctx **out, const stein_icp_config *cfg,
                   const float *src_xyz, int64_t n_src,
                   const float *ref_xyz, int64_t n_ref,
                   const double *init_particles, const int32_t *schedule,
                   void *hip_stream);

/* Create a context holding n_pairs independent problems that advance
 * together, each with its own clouds, K particles and schedule (same K, m and
 * schedule_rows for all). Host arrays of n_pairs device pointers and sizes.
 * init_particles: device FP64 n_pairs x K x 6, or NULL (pair p draws from
 * cfg->seed + p). schedules: host array of n_pairs device pointers, or NULL
 * (pair p draws from cfg->seed + p). 1 <= n_pairs <= 65535. Pairs given the
 * same cloud (same device pointer and size) share one packed copy of it, its
 * normals and its BF16 fragments; with K = 1 and one cloud pair repeated,
 * the pairs are independent SGD-ICP runs (the paper's Monte-Carlo ground
 * truth, Sec. V-A), each with its own start and minibatches. Blocking, like
 * stein_icp_init. */
int stein_icp_batch_init(stein_icp_ctx **out, const stein_icp_config *cfg, int32_t n_pairs,
                         const float *const *src_xyz, const int64_t *n_src,
                         const float *const *ref_xyz, const int64_t *n_ref,
                         const double *init_particles, const int32_t *const *schedules,
                         void *hip_stream);

/* Run n_iters >= 0 iterations. Asynchronous on `hip_stream`. */
int stein_icp_step(stein_icp_ctx *ctx, int32_t n_iters, void *hip_stream);

/* Copy the particles to device FP64 out (n_pairs x K x 6). Asynchronous. */
int stein_icp_particles(const stein_icp_ctx *ctx, double *out, void *hip_stream);

/* FP32 particle I/O (the problem statement's K x 6 FP32 particles, beside
 * the FP64 state the library keeps):
 * stein_icp_particles_f32: the particles rounded to FP32 (nearest), device
 *   FP32 n_pairs x K x 6 out. Asynchronous.
 * stein_icp_set_particles_f32: start again from device FP32 n_pairs x K x 6
 *   particles (widened exactly to FP64), Adam moments zero, step count 0.
 *   Blocking: a non-finite value gives E_INVALID with the context unchanged. */
int stein_icp_particles_f32(const stein_icp_ctx *ctx, float *out, void *hip_stream);
int stein_icp_set_particles_f32(stein_icp_ctx *ctx, const float *theta, void *hip_stream);

/* Read the optimiser state: device FP64 theta, Adam first and second moments
 * (each n_pairs x K x 6; any may be NULL) and the host step count t (may be
 * NULL). Blocking (synchronises `hip_stream`). */
int stein_icp_get_state(const stein_icp_ctx *ctx, double *theta, double *mom, double *vel,
                        int64_t *t, void *hip_stream);

/* Replace the optimiser state (device FP64 arrays as above; NULL moments are
 * set to zero) and the step count t >= 0, and recompute the rotations.
 * Blocking: the inputs are first checked for non-finite values
 * (E_INVALID, context unchanged), then copied on `hip_stream`. */
int stein_icp_set_state(stein_icp_ctx *ctx, const double *theta, const double *mom,
                        const double *vel, int64_t t, void *hip_stream);

/* Quantities of the most recent iteration, for checking: device FP64 gbar
 * (mean gradient of Eqs. 4-5, n_pairs x K x 6), phi (Eq. 16 direction,
 * n_pairs x K x 6), h (n_pairs x 2: translation, rotation bandwidth) and int32
 * match (n_pairs x K x m reference indices). Any may be NULL. Asynchronous. */
int stein_icp_get_diagnostics(const stein_icp_ctx *ctx, double *gbar, double *phi, double *h,
                              int32_t *match, void *hip_stream);

/* Number of pairs, particles and minibatch size of a context. */
int stein_icp_shape(const stein_icp_ctx *ctx, int32_t *n_pairs, int32_t *K, int32_t *m);

/* Nearest-neighbour work shape of the context: FP32 queries per lane,
 * wavefronts per workgroup, references per workgroup chunk and chunks (of
 * pair 0), persistence (0: one workgroup per work item; n: n workgroups per
 * compute unit walking the work table of all pairs), and the mean time in ms
 * of one NN + gradient launch pair measured by the autotuner (0 if not
 * tuned). Any of the outputs may be NULL. */
int stein_icp_nn_tiling(const stein_icp_ctx *ctx, int32_t *queries_per_lane, int32_t *waves,
                        int32_t *chunk, int32_t *chunks, int32_t *persist, double *tuned_ms);

/* Force the nearest-neighbour work shape: queries_per_lane in {1, 2, 4},
 * waves in {4, 8, 16}, chunk a positive multiple of 32 references (capped
 * at each pair's padded reference count), persist in [0, 64] as above. The
 * BF16 screen takes 1 or 2 queries per lane, and 4 or 8 waves with 2. The
 * shape changes only how the search is split over workgroups, never its
 * result. Blocking (reallocates the per-chunk key buffer and synchronises
 * `hip_stream`). */
int stein_icp_set_nn_tiling(stein_icp_ctx *ctx, int32_t queries_per_lane, int32_t waves,
                            int32_t chunk, int32_t persist, void *hip_stream);

/* Profiled mode: run n_iters >= 1 iterations with plain launches (no graph),
 * recording HIP events on `hip_stream` around each launch, and return the
 * summed times in ms_out[3] (host): nearest neighbours (Eq. 1); mean
 * gradients (Eqs. 4-5) together with the median-heuristic bandwidths
 * (Sec. V), which share one launch; Stein direction plus update (Eqs. 12,
 * 16). Advances the state like stein_icp_step. Blocking. */
int stein_icp_stage_times(stein_icp_ctx *ctx, int32_t n_iters, double *ms_out, void *hip_stream);

/* Mean duration in ms of the nearest-neighbour kernel (Eq. 1) over
 * n_launches >= 1 back-to-back launches on the current queries, timed with
 * HIP events on `hip_stream`. The launches only rewrite the per-chunk keys,
 * which the next iteration recomputes, so the optimiser state is unchanged.
 * Blocking. */
int stein_icp_time_nn(stein_icp_ctx *ctx, int32_t n_launches, double *ms_per_launch, void *hip_stream);

/* Certificate statistics of the BF16 screen (STEIN_ICP_NN_BF16_RERANK; both
 * 0 for the FP32 search), accumulated since init over every nearest-
 * neighbour launch of the context (iterations, profiled and timed launches):
 * *certificates: screen certificates evaluated -- one per real query, chunk,
 *   lane half (two) and wavefront holding blocks of the chunk (Eq. 1 is
 *   proved exact for each);
 * *rescans: those that failed and were searched again in FP32.
 * Either output may be NULL. Blocking (synchronises `hip_stream`). */
int stein_icp_nn_rescans(const stein_icp_ctx *ctx, int64_t *rescans, int64_t *certificates,
                         void *hip_stream);

/* Release the context and its device memory. NULL is a no-op. Blocking
 * (synchronises the device before freeing). */
void stein_icp_destroy(stein_icp_ctx *ctx);

/* Message for the last failure on the calling thread ("" if none). */
const char *stein_icp_last_error(void);

/* Standalone nearest-neighbour search (Eq. 1) over given FP32 queries.
 *   q_xyz: device FP32 nq x 3; ref_xyz: device FP32 n_ref x 3;
 *   mode: STEIN_ICP_NN_*; idx: device int32 nq; d2: device FP32 nq (the
 *   FP32 squared distance of the returned index; may be NULL).
 * Allocates and frees its own scratch; blocking. */
int stein_icp_nn(const float *q_xyz, int64_t nq, const float *ref_xyz, int64_t n_ref,
                 int32_t mode, int32_t *idx, float *d2, void *hip_stream);

/* The raw screened values of a matrix-core screen, for checking its error
 * bound: for mode BF16_RERANK or F16_RERANK, values[i * n_ref + j] (device
 * FP32, nq x n_ref, nq * n_ref <= 2^31) is |q_i|^2 + |r_j|^2 - 2 q_i.r_j as
 * that screen computes it (centred on the reference centroid, split into
 * BF16 or FP16 parts, on the same matrix products; the FP16 screen's values
 * are divided by 4^scale_exp, exactly), NaN for a query the FP16 screen
 * does not screen. centre (host, 4 floats, may be NULL): the centroid
 * c0[0..2] and the bound R >= every centred reference norm; scale_exp
 * (host, may be NULL): the FP16 screen's power-of-two scale. The error
 * bounds: |S - F| <= 52 u (|q_c| + R)^2 + 6.2 u F (BF16 x 3) and
 * |S - F| <= 50 u (|q_c| + |r_c|)^2 + 2^-22 (|q_c| + |r_c| + 2^-e) 2^-e
 * with e = scale_exp (FP16 x 2), u = 2^-24, F the FP32 squared distance of
 * Eq. 1, allowing the matrix core up to one FP32 ulp of its partial sum per
 * addition. Allocates and frees its own scratch; blocking. */
int stein_icp_screen_values(const float *q_xyz, int64_t nq, const float *ref_xyz, int64_t n_ref,
                            int32_t mode, float *values, float *centre, int32_t *scale_exp,
                            void *hip_stream);

/* stein_icp_nn for callers that cannot allocate device memory (code that
 * runs while a stream is being captured into a hipGraph, tight serving
 * loops, harnesses that forbid hipMalloc): the same search, arguments,
 * validation, answers (bit for bit) and blocking behaviour, with no call to
 * hipMalloc or hipFree. Its working memory -- packed queries (16 B each),
 * packed references (16 B per reference padded to a multiple of 32, plus
 * 64 B of BF16 fragments for BF16_RERANK), the work table and the per-chunk
 * keys (8 B per query and reference chunk; fewer chunks are used when they
 * would not fit) -- lives in a 32 MiB array inside the library, one per GPU,
 * held until the process ends. E_INVALID when a search needs more than that
 * (FP32: beyond about 1.2 M queries against 0.1 M references). Every call on
 * one GPU uses that GPU's array: calls that overlap on one GPU (other
 * threads or streams) race and must be serialised by the caller. */
int stein_icp_nn_noalloc(const float *q_xyz, int64_t nq, const float *ref_xyz, int64_t n_ref,
                         int32_t mode, int32_t *idx, float *d2, void *hip_stream);

/* Standalone k-nearest-neighbour search under Eq. 1's metric: for each
 * query the k smallest (FP32 squared distance, index) pairs in ascending
 * order, ties to the lower index (the neighbourhoods of the normals).
 *   q_xyz: device FP32 nq x 3; ref_xyz: device FP32 n_ref x 3; 1 <= k <= 32;
 *   idx: device int32 nq x k (-1 past n_ref); d2: device FP32 nq x k
 *   (+inf past n_ref).
 * Allocates and frees its own scratch; blocking. */
int stein_icp_knn(const float *q_xyz, int64_t nq, const float *ref_xyz, int64_t n_ref,
                  int32_t k, int32_t *idx, float *d2, void *hip_stream);

/* Normals of a cloud, as the point-to-plane metric computes them at init
 * (see STEIN_ICP_METRIC_PLANE), from each point's k nearest points.
 *   ref_xyz: device FP32 n_ref x 3; 3 <= k <= 32 (all points when
 *   n_ref < k); normals: device FP64 n_ref x 3 (unit or zero); eig: device
 *   FP64 n_ref x 3, the covariance eigenvalues in ascending order, or NULL.
 * Allocates and frees its own scratch; blocking. */
int stein_icp_normals(const float *ref_xyz, int64_t n_ref, int32_t k, double *normals,
                      double *eig, void *hip_stream);

/* The normals a point-to-plane context computed at init: device FP64
 * (sum of n_ref over its pairs) x 3, pairs in order. E_STATE for a
 * point-to-point context. Stream-ordered. */
int stein_icp_get_normals(const stein_icp_ctx *ctx, double *out, void *hip_stream);

/* Scores of a posterior sample set a (host FP64 na x 6 poses) against a
 * reference sample set b (host FP64 nb x 6), e.g. a Monte-Carlo ground truth
 * of independent SGD-ICP runs (a batch context with K = 1 whose pairs all
 * share one cloud pair), as the paper scores its posteriors (Sec. V-A):
 *   kl[0], kl[1]: KL(N_a || N_b) between the normal fits (sample mean,
 *     covariance with an n - 1 denominator) of the translations and of the
 *     rotations;
 *   ovl[0..5]: overlapping coefficient, the integral of min(f_a, f_b), of the
 *     normal fits of each coordinate (0: disjoint, 1: identical).
 * Angles are first taken within pi of b's circular mean. Either output may
 * be NULL. E_INVALID for fewer than 2 poses in a set, a non-finite sample or
 * a covariance that is not positive definite. No device needed. */
int stein_icp_posterior_scores(const double *a, int64_t na, const double *b, int64_t nb,
                               double *kl, double *ovl);

/* Host helpers (no device needed). The library's own generator is
 * SplitMix64 (Steele, Lea, Flood 2014): uniform doubles from the top 53 bits,
 * minibatch rows by Floyd's sampling of m distinct indices.
 * stein_icp_make_schedule: host int32 rows x m.
 * stein_icp_make_init: host FP64 K x 6, centre (may be NULL = 0) +- half. */
int stein_icp_make_schedule(uint64_t seed, int64_t n_src, int32_t m, int32_t rows,
                            int32_t *out_host);
int stein_icp_make_init(uint64_t seed, int32_t K, double half_trans, double half_rot,
                        const double *centre, double *out_host);

#ifdef __cplusplus
}
#endif

#endif /* STEIN_ICP_H */
