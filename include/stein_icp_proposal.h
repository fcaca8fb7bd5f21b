/*
 * stein_icp_proposal.h -- C ABI of the learned initial-particle proposal.
 *
 * Stein ICP (arXiv:2106.03287) starts its K particles from a uniform draw
 * over a box of poses (Sec. V) and then needs many iterations before they
 * settle on the posterior. This library adds a learned proposal: a point-set
 * network reads the (source, reference) pair and emits K particles that seed
 * Stein ICP instead (`init_particles` of stein_icp_init / stein_icp_batch_init);
 * a pair whose network output is not finite falls back to the uniform draw.
 * The network is not part of the paper.
 *
 * Network (every cloud is first resampled to P points, see
 * stein_icp_proposal_prepare):
 *   per point:   h1 = relu(x W1 + b1)    3 -> 64
 *                h2 = relu(h1 W2 + b2)  64 -> 128
 *                h3 = relu(h2 W3 + b3) 128 -> 256
 *   per cloud:   f = max over points of h3 (first maximum on ties)
 *   per pair:    z = relu([f_src, f_ref] W4 + b4)  512 -> 256
 *                y = z W5 + b5                     256 -> 6K
 * y is read as K row-major particles (x, y, z, roll, pitch, yaw).
 * Every matrix product rounds both operands to BF16 (round to nearest even)
 * and accumulates in FP32 on the matrix cores; weights, activations and
 * gradients are stored in FP32.
 *
 * Parameter vector (FP32, in this order; weights row-major in x out):
 *   W1 3x64, b1 64, W2 64x128, b2 128, W3 128x256, b3 256, W4 512x256, b4 256,
 *   W5 256x6K, b5 6K  -- stein_icp_proposal_param_count gives the total.
 *
 * Training loss per pair b (targets are K particles of a converged Stein-ICP
 * run): the biased MMD^2 estimate between the network's particles X and the
 * target particles Y,
 *   L_b = (1/K^2) sum_{i,j} [k(x_i,x_j) + k(y_i,y_j) - 2 k(x_i,y_j)],
 *   k(u,v) = sum_s exp(-1/2 sum_c ((u_c - v_c) / sigma_{s,c})^2),
 * angle differences wrapped to [-pi, pi]; the batch loss is the mean of L_b.
 *
 * Conventions are those of stein_icp.h: device pointers unless stated, the
 * caller owns what it passes, NULL stream = default stream, status codes
 * STEIN_ICP_*, stein_icp_last_error() describes a failure, and a model is
 * driven by one thread.
 */
#ifndef STEIN_ICP_PROPOSAL_H
#define STEIN_ICP_PROPOSAL_H

#include <stdint.h>

#include "stein_icp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define STEIN_ICP_PROPOSAL_MAX_POINTS 4096
#define STEIN_ICP_PROPOSAL_MAX_PARTICLES 1024
#define STEIN_ICP_PROPOSAL_MAX_SCALES 4

typedef struct stein_icp_proposal stein_icp_proposal;

typedef struct stein_icp_proposal_config {
    uint64_t struct_size;    /* sizeof(stein_icp_proposal_config) */
    int32_t num_particles;   /* K, 1..1024: the head emits 6K values */
    int32_t points;          /* P, 1..4096: network input points per cloud */
    int32_t max_batch;       /* most pairs per forward / loss call, >= 1 */
    int32_t n_loss_scales;   /* 1..4 kernel widths of the training loss */
    double loss_sigma[STEIN_ICP_PROPOSAL_MAX_SCALES][6]; /* > 0; m for x,y,z, rad for angles */
} stein_icp_proposal_config;

/* Defaults: K 100, P 4096, max_batch 32, four loss widths
 * (0.01, 0.04, 0.16, 0.64) m and (0.02, 0.08, 0.32, 1.28) rad, from below a
 * converged posterior's spread to that of the initial draw. Host only. */
int stein_icp_proposal_default_config(stein_icp_proposal_config *cfg);

/* Number of FP32 parameters of a network with K particles. Host only. */
int stein_icp_proposal_param_count(int32_t num_particles, int64_t *count);

/* Allocate a model for `cfg` (parameters zero, Adam moments zero, step 0).
 * Blocking. Fails with STEIN_ICP_E_INVALID on a bad config before any
 * device call, STEIN_ICP_E_NOMEM when the buffers do not fit (about 1 MiB
 * per pair of max_batch; when P is not a multiple of 64 the per-point
 * activations are kept too, 1792 bytes for each of 2 max_batch P points). */
int stein_icp_proposal_create(stein_icp_proposal **out, const stein_icp_proposal_config *cfg);
int stein_icp_proposal_destroy(stein_icp_proposal *model);

/* Weight file: the NumPy .npy format (magic "\x93NUMPY", version 1.0, 2.0 or
 * 3.0, a little-endian header length, an ASCII dict header) holding one
 * one-dimensional little-endian float32 array ('<f4', fortran_order False)
 * of the parameter vector in the order above; its length, 172,928 + 1,542 K,
 * fixes K (`np.save(path, params)` writes such a file).
 * stein_icp_proposal_read_weights (host only) checks the file and reports
 * *count values (may be NULL) for *num_particles = K (may be NULL); with
 * params != NULL it also reads them into params (host, capacity values) and
 * checks they are finite. E_INVALID for an unreadable or malformed file. */
int stein_icp_proposal_read_weights(const char *path, float *params, int64_t capacity, int64_t *count,
                                    int32_t *num_particles);

/* Create a model (stein_icp_proposal_default_config, with the file's K) and
 * load the parameters of a weight file into it. Blocking. On failure *out is
 * NULL and nothing stays allocated. */
int stein_icp_proposal_load(stein_icp_proposal **out, const char *weights_path);

/* Copy `param_count` FP32 parameters in (resets the Adam moments and step
 * count) or out. Device pointers; enqueued on `hip_stream`. */
int stein_icp_proposal_set_params(stein_icp_proposal *model, const float *params, void *hip_stream);
int stein_icp_proposal_get_params(const stein_icp_proposal *model, float *params, void *hip_stream);

/* Network input of one cloud: out (P x 3) point p = xyz point floor(p n / P),
 * n >= 1 (each point once when n = P, evenly repeated when n < P; the cloud
 * is expected in random order, as a strided pick then is a uniform subset).
 * Enqueued. */
int stein_icp_proposal_prepare(const stein_icp_proposal *model, const float *xyz, int64_t n, float *out,
                               void *hip_stream);

/* Forward pass over `batch` pairs (1..max_batch). clouds: batch x 2 x P x 3
 * FP32 (pair b: source then reference). particles: batch x K x 6 FP64 out.
 * nonfinite (may be NULL): batch int32 out, 1 where a pair's output holds a
 * non-finite value (that pair should use the uniform draw). Enqueued. */
int stein_icp_proposal_forward(stein_icp_proposal *model, const float *clouds, int32_t batch, double *particles,
                               int32_t *nonfinite, void *hip_stream);

/* Training loss and gradient: forward over `batch` pairs, then per-pair loss
 * L_b (FP64, `loss`: batch values out) and the gradient of mean_b L_b with
 * respect to every parameter, kept in the model for stein_icp_proposal_adam
 * and copied to `grad` (param_count FP32, may be NULL). targets: batch x K x
 * 6 FP64. Enqueued. */
int stein_icp_proposal_loss(stein_icp_proposal *model, const float *clouds, const double *targets, int32_t batch,
                            double *loss, float *grad, void *hip_stream);

/* One Adam step on the gradient of the last stein_icp_proposal_loss call:
 * t += 1; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). Enqueued. */
int stein_icp_proposal_adam(stein_icp_proposal *model, double lr, double beta1, double beta2, double eps,
                            void *hip_stream);

/* Set distance between particle sets (the same MMD^2 as the training loss,
 * FP64): out[b] for X[b], Y[b] (batch x K x 6 each, device). sigma: host
 * n_scales x 6 widths. Enqueued; needs no model. */
int stein_icp_proposal_mmd(const double *X, const double *Y, int32_t batch, int32_t K, int32_t n_scales,
                           const double *sigma, double *out, void *hip_stream);

/* Proposal for one pair: prepare both clouds, run the network, write K x 6
 * FP64 particles to `particles` and set *used_fallback (host) to 1 when the
 * output was not finite -- then pass NULL init_particles to stein_icp_init for
 * the uniform draw. Blocking (reads the finiteness flag). */
int stein_icp_propose(stein_icp_proposal *model, const float *src_xyz, int64_t n_src, const float *ref_xyz,
                      int64_t n_ref, double *particles, int32_t *used_fallback, void *hip_stream);

/* The network's matrix product as a primitive:
 *   C = op(A) op(B) [+ bias] [relu] [+ C]   (M x N, FP32, row-major, ldc)
 * op(A) = A (A: M x K, lda) or A^T (ta = 1, A: K x M, lda); op(B) = B (B: K x N,
 * ldb) or B^T (tb = 1, B: N x K, ldb); bias: N values or NULL. Operands are
 * rounded to BF16, products accumulate in FP32. splits > 1 divides K among
 * that many workgroup slices whose partial products go to `workspace`
 * (splits x M x N FP32, caller-owned) and are summed in slice order.
 * K = 0 gives C = bias (relu) (+ C). An operand with no elements may be NULL.
 * Enqueued. */
int stein_icp_gemm_bf16(int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const float *A, int64_t lda,
                        const float *B, int64_t ldb, float *C, int64_t ldc, const float *bias, int32_t relu,
                        int32_t accumulate, int32_t splits, float *workspace, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* STEIN_ICP_PROPOSAL_H */
