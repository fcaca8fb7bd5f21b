// Host side of the learned initial-particle proposal: model buffers, the
// forward and backward passes as sequences of matrix-core GEMMs and small
// kernels, Adam, the set distance and the C ABI of
// include/stein_icp_proposal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "stein_icp_proposal.h"

#include "proposal.hpp"

namespace sicp {
int report_error(int code, const std::string& msg);
}

using namespace sicp::prop;

namespace {

int fail(int code, const std::string& msg) { return sicp::report_error(code, msg); }

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(STEIN_ICP_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

inline int64_t ceil_div(int64_t v, int64_t a) { return (v + a - 1) / a; }

constexpr int kF1 = 64, kF2 = 128, kF3 = 256, kFcat = 512, kFz = 256;
constexpr int64_t kPoolChunk = 256;     // points per max-pool partial
constexpr int64_t kColChunk = 64;       // rows per column-sum partial
constexpr int kMaxSplits = 64;

// offsets of the parameter blocks in the flat vector
struct Layout {
    int64_t W1, b1, W2, b2, W3, b3, W4, b4, W5, b5, total;
    explicit Layout(int64_t K)
    {
        int64_t o = 0;
        W1 = o; o += 3 * kF1;
        b1 = o; o += kF1;
        W2 = o; o += (int64_t)kF1 * kF2;
        b2 = o; o += kF2;
        W3 = o; o += (int64_t)kF2 * kF3;
        b3 = o; o += kF3;
        W4 = o; o += (int64_t)kFcat * kFz;
        b4 = o; o += kFz;
        W5 = o; o += (int64_t)kFz * 6 * K;
        b5 = o; o += 6 * K;
        total = o;
    }
};

int validate(const stein_icp_proposal_config* c)
{
    if (!c) return fail(STEIN_ICP_E_INVALID, "config is NULL");
    if (c->struct_size != sizeof(stein_icp_proposal_config))
        return fail(STEIN_ICP_E_INVALID, "struct_size does not match this library's stein_icp_proposal_config");
    if (c->num_particles < 1 || c->num_particles > STEIN_ICP_PROPOSAL_MAX_PARTICLES)
        return fail(STEIN_ICP_E_INVALID, "num_particles must be in [1, 1024]");
    if (c->points < 1 || c->points > STEIN_ICP_PROPOSAL_MAX_POINTS)
        return fail(STEIN_ICP_E_INVALID, "points must be in [1, 4096]");
    if (c->max_batch < 1 || (int64_t)c->max_batch * c->points > (int64_t)1 << 24)
        return fail(STEIN_ICP_E_INVALID, "max_batch must be >= 1 with max_batch * points <= 2^24");
    if (c->n_loss_scales < 1 || c->n_loss_scales > STEIN_ICP_PROPOSAL_MAX_SCALES)
        return fail(STEIN_ICP_E_INVALID, "n_loss_scales must be in [1, 4]");
    for (int s = 0; s < c->n_loss_scales; ++s)
        for (int d = 0; d < 6; ++d)
            if (!(std::isfinite(c->loss_sigma[s][d]) && c->loss_sigma[s][d] > 0.0))
                return fail(STEIN_ICP_E_INVALID, "loss_sigma must be finite and > 0");
    return STEIN_ICP_OK;
}

int make_scales(int32_t ns, const double* sigma, MmdScales& sc)
{
    if (ns < 1 || ns > kMaxLossScales || !sigma) return fail(STEIN_ICP_E_INVALID, "n_scales must be in [1, 4]");
    std::memset(&sc, 0, sizeof(sc));
    sc.ns = ns;
    for (int s = 0; s < ns; ++s)
        for (int d = 0; d < 6; ++d) {
            const double v = sigma[6 * s + d];
            if (!(std::isfinite(v) && v > 0.0)) return fail(STEIN_ICP_E_INVALID, "sigma must be finite and > 0");
            sc.inv[s][d] = 1.0 / v;
        }
    return STEIN_ICP_OK;
}

int launch_gemm(hipStream_t s, int ta, int tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                const float* B, int64_t ldb, float* C, int64_t ldc, const float* bias, int relu, int acc,
                int32_t splits, float* ws, unsigned long long* pool_keys = nullptr, int64_t pool_P = 0)
{
    if (M <= 0 || N <= 0) return STEIN_ICP_OK;
    if (splits < 1) splits = 1;
    const int64_t ksteps = std::max<int64_t>(ceil_div(K, kGK), 1);
    int64_t kper = ceil_div(ksteps, splits) * kGK;
    splits = (int32_t)std::max<int64_t>(ceil_div(std::max<int64_t>(K, 1), kper), 1);
    GemmArgs g{};
    g.A = A;
    g.B = B;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda;
    g.ldb = ldb;
    g.kper = kper;
    g.ta = ta;
    g.tb = tb;
    g.pool_keys = pool_keys;
    g.pool_P = pool_P;
    if (pool_keys) splits = 1;
    const int64_t Mt = ceil_div(M, kGT), Nt = ceil_div(N, kGT);
    const dim3 grid((unsigned)(ceil_div(Mt, kXcds) * kXcds * Nt), 1, (unsigned)splits);
    if (splits == 1) {
        g.C = C;
        g.ldc = ldc;
        g.bias = bias;
        g.relu = relu;
        g.accumulate = acc;
        g.c_split = 0;
        gemm_bf16_kernel<<<grid, 256, 0, s>>>(g);
    } else {
        g.C = ws;
        g.ldc = N;
        g.bias = nullptr;
        g.relu = 0;
        g.accumulate = 0;
        g.c_split = M * N;
        gemm_bf16_kernel<<<grid, 256, 0, s>>>(g);
        splitk_reduce_kernel<<<(unsigned)ceil_div(M * N, 256), 256, 0, s>>>(ws, splits, M, N, C, ldc, bias, relu,
                                                                            acc);
    }
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

}  // namespace

struct stein_icp_proposal {
    stein_icp_proposal_config cfg;
    int64_t K, P, Bmax, n_params;
    MmdScales scales;
    void* arena = nullptr;
    float *params, *grad, *adam_m, *adam_v;
    bool fused_pool;       // P % 64 == 0: the fused per-point kernel, no per-point activations in HBM
    float *H1, *H2, *H3;   // per-point activations, only without the fused kernel
    float *pool_v, *F, *Z, *Y, *dY, *dZ, *dF;
    int32_t *pool_i, *arg, *flags;
    unsigned long long* pool_keys;
    float *G0, *G1, *G2, *dA3, *dA2, *dA1;   // winner rows of the sparse backward (F3 per cloud)
    float *ws, *colpart, *prep;
    int64_t ws_floats, colpart_floats;
    int64_t step = 0;
    int32_t last_batch = 0;   // batch of the last loss call (0: no gradient yet)
    int32_t num_cus = 256;
};

namespace {

using Model = stein_icp_proposal;

int gemm(const Model* m, hipStream_t s, int ta, int tb, int64_t M, int64_t N, int64_t K, const float* A,
         int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc, const float* bias, int relu)
{
    // split K when the output tiles alone cannot fill the chip and K is long
    const int64_t tiles = ceil_div(M, kGT) * ceil_div(N, kGT);
    int32_t splits = 1;
    if (tiles < 512 && K >= 4 * kGK * 2) {
        const int64_t want = ceil_div(1024, tiles);
        const int64_t by_k = K / (4 * kGK);   // keep >= 4 K steps per slice
        splits = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, by_k, kMaxSplits,
                                                                  m->ws_floats / std::max<int64_t>(M * N, 1)}));
    }
    return launch_gemm(s, ta, tb, M, N, K, A, lda, B, ldb, C, ldc, bias, relu, 0, splits, m->ws);
}

int colsum(const Model* m, hipStream_t s, const float* X, int64_t rows, int64_t N, float* out)
{
    const int64_t nch = std::max<int64_t>(ceil_div(rows, kColChunk), 1);
    if (nch * N > m->colpart_floats) return fail(STEIN_ICP_E_INVALID, "column-sum workspace too small");
    colsum_partial_kernel<<<dim3((unsigned)ceil_div(N, 256), (unsigned)nch), 256, 0, s>>>(X, rows, N, kColChunk,
                                                                                          m->colpart);
    colsum_merge_kernel<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(m->colpart, nch, N, out);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

#define CHECK(expr)                   \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != STEIN_ICP_OK) return rc_; \
    } while (0)

// Forward pass: H1..H3, pooled F, arg, Z, Y (all FP32) for `B` pairs.
int forward(Model* m, hipStream_t s, const float* X, int64_t B)
{
    const Layout L(m->K);
    const float* w = m->params;
    const int64_t rows = 2 * B * m->P, K6 = 6 * m->K;
    if (m->fused_pool) {
        fill_u64_kernel<<<(unsigned)ceil_div(2 * B * kF3, 256), 256, 0, s>>>(m->pool_keys, 2 * B * kF3, 0ull);
        MlpArgs ma{};
        ma.X = X;
        ma.W1 = w + L.W1;
        ma.b1 = w + L.b1;
        ma.W2 = w + L.W2;
        ma.b2 = w + L.b2;
        ma.W3 = w + L.W3;
        ma.b3 = w + L.b3;
        ma.keys = m->pool_keys;
        ma.rows = rows;
        ma.P = m->P;
        // one workgroup per CU holds the staged weights (LDS bound) and works
        // on two tiles at a time; tiles are strided over the workgroups
        const int64_t tiles = rows / kMT;
        mlp_pool_kernel<<<(unsigned)std::min<int64_t>(ceil_div(tiles, 2), m->num_cus), kMlpThreads, kMlpLdsBytes, s>>>(ma);
        pool_keys_finish_kernel<<<(unsigned)ceil_div(2 * B * kF3, 256), 256, 0, s>>>(m->pool_keys, 2 * B, kF3, m->F,
                                                                                    kFcat, m->arg);
    } else {
        CHECK(gemm(m, s, 0, 0, rows, kF1, 3, X, 3, w + L.W1, kF1, m->H1, kF1, w + L.b1, 1));
        CHECK(gemm(m, s, 0, 0, rows, kF2, kF1, m->H1, kF1, w + L.W2, kF2, m->H2, kF2, w + L.b2, 1));
        CHECK(gemm(m, s, 0, 0, rows, kF3, kF2, m->H2, kF2, w + L.W3, kF3, m->H3, kF3, w + L.b3, 1));
        const int64_t nch = ceil_div(m->P, kPoolChunk);
        maxpool_partial_kernel<<<dim3((unsigned)(2 * B), (unsigned)nch), kF3, 0, s>>>(m->H3, m->P, kF3, kPoolChunk,
                                                                                      m->pool_v, m->pool_i);
        maxpool_merge_kernel<<<(unsigned)ceil_div(2 * B * kF3, 256), 256, 0, s>>>(m->pool_v, m->pool_i, 2 * B, nch,
                                                                                 kF3, m->F, kFcat, m->arg);
    }
    HIP_TRY(hipGetLastError());
    CHECK(gemm(m, s, 0, 0, B, kFz, kFcat, m->F, kFcat, w + L.W4, kFz, m->Z, kFz, w + L.b4, 1));
    CHECK(gemm(m, s, 0, 0, B, K6, kFz, m->Z, kFz, w + L.W5, K6, m->Y, K6, w + L.b5, 0));
    return STEIN_ICP_OK;
}

// Backward pass of mean_b L_b from dY (already scaled by 1/B) into m->grad.
// The head is dense. Below the max-pool only the points that won a pooled
// feature receive gradient: the per-point layers are differentiated on F3
// rows per cloud (its distinct winners, then zero rows) instead of all P
// points, with the dense chain rule's products (BF16 operands, FP32 sums).
int backward(Model* m, hipStream_t s, const float* X, int64_t B)
{
    const Layout L(m->K);
    const float* w = m->params;
    float* g = m->grad;
    const int64_t K6 = 6 * m->K, rows = 2 * B * kF3;
    // head: y = z W5 + b5, z = relu(f W4 + b4)
    CHECK(gemm(m, s, 1, 0, kFz, K6, B, m->Z, kFz, m->dY, K6, g + L.W5, K6, nullptr, 0));
    CHECK(colsum(m, s, m->dY, B, K6, g + L.b5));
    CHECK(gemm(m, s, 0, 1, B, kFz, K6, m->dY, K6, w + L.W5, K6, m->dZ, kFz, nullptr, 0));
    relu_backward_kernel<<<(unsigned)ceil_div(B * kFz, 256), 256, 0, s>>>(m->Z, m->dZ, B * kFz);
    CHECK(gemm(m, s, 1, 0, kFcat, kFz, B, m->F, kFcat, m->dZ, kFz, g + L.W4, kFz, nullptr, 0));
    CHECK(colsum(m, s, m->dZ, B, kFz, g + L.b4));
    CHECK(gemm(m, s, 0, 1, B, kFcat, kFz, m->dZ, kFz, w + L.W4, kFz, m->dF, kFcat, nullptr, 0));
    // winner rows: the winning points' inputs and the pooled gradients they
    // carry; their first two layers are recomputed with the forward's
    // products (one K slice each, the same MFMA order, bias and ReLU: the
    // same bits)
    winner_rows_kernel<kF3><<<(unsigned)(2 * B), kF3, 0, s>>>(X, m->arg, m->F, m->dF, kFcat, m->P, m->G0, m->dA3);
    HIP_TRY(hipGetLastError());
    CHECK(launch_gemm(s, 0, 0, rows, kF1, 3, m->G0, 3, w + L.W1, kF1, m->G1, kF1, w + L.b1, 1, 0, 1, nullptr));
    CHECK(launch_gemm(s, 0, 0, rows, kF2, kF1, m->G1, kF1, w + L.W2, kF2, m->G2, kF2, w + L.b2, 1, 0, 1, nullptr));
    CHECK(gemm(m, s, 1, 0, kF2, kF3, rows, m->G2, kF2, m->dA3, kF3, g + L.W3, kF3, nullptr, 0));
    CHECK(colsum(m, s, m->dA3, rows, kF3, g + L.b3));
    CHECK(gemm(m, s, 0, 1, rows, kF2, kF3, m->dA3, kF3, w + L.W3, kF3, m->dA2, kF2, nullptr, 0));
    relu_backward_kernel<<<(unsigned)ceil_div(rows * kF2, 256), 256, 0, s>>>(m->G2, m->dA2, rows * kF2);
    CHECK(gemm(m, s, 1, 0, kF1, kF2, rows, m->G1, kF1, m->dA2, kF2, g + L.W2, kF2, nullptr, 0));
    CHECK(colsum(m, s, m->dA2, rows, kF2, g + L.b2));
    CHECK(gemm(m, s, 0, 1, rows, kF1, kF2, m->dA2, kF2, w + L.W2, kF2, m->dA1, kF1, nullptr, 0));
    relu_backward_kernel<<<(unsigned)ceil_div(rows * kF1, 256), 256, 0, s>>>(m->G1, m->dA1, rows * kF1);
    CHECK(gemm(m, s, 1, 0, 3, kF1, rows, m->G0, 3, m->dA1, kF1, g + L.W1, kF1, nullptr, 0));
    CHECK(colsum(m, s, m->dA1, rows, kF1, g + L.b1));
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

int launch_mmd(hipStream_t s, const float* Xf, const double* Xd, const double* Y, int64_t B, int32_t K,
               const MmdScales& sc, double gscale, float* dX, double* loss)
{
    // X and Y sets plus the gradient partials of max(1, 256 / K) row groups
    // (K <= 1024 keeps it within 144 KiB)
    const size_t lds = sizeof(double) * (12 * (size_t)K + 6 * (size_t)std::max(1, 256 / K) * K);
    if (lds > 65536)
        HIP_TRY(hipFuncSetAttribute((const void*)mmd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    mmd_kernel<<<(unsigned)B, 256, lds, s>>>(Xf, Xd, Y, K, sc, gscale, dX, loss);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

void free_model(Model* m)
{
    if (!m) return;
    if (m->arena) (void)hipFree(m->arena);
    delete m;
}

}  // namespace

extern "C" {

int stein_icp_proposal_default_config(stein_icp_proposal_config* c)
{
    if (!c) return fail(STEIN_ICP_E_INVALID, "config is NULL");
    std::memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(*c);
    c->num_particles = 100;
    c->points = 4096;
    c->max_batch = 32;
    c->n_loss_scales = 4;
    const double t[4] = {0.01, 0.04, 0.16, 0.64}, r[4] = {0.02, 0.08, 0.32, 1.28};
    for (int s = 0; s < 4; ++s)
        for (int d = 0; d < 6; ++d) c->loss_sigma[s][d] = d < 3 ? t[s] : r[s];
    return STEIN_ICP_OK;
}

int stein_icp_proposal_param_count(int32_t K, int64_t* count)
{
    if (!count) return fail(STEIN_ICP_E_INVALID, "count is NULL");
    if (K < 1 || K > STEIN_ICP_PROPOSAL_MAX_PARTICLES) return fail(STEIN_ICP_E_INVALID, "K must be in [1, 1024]");
    *count = Layout(K).total;
    return STEIN_ICP_OK;
}

int stein_icp_proposal_create(stein_icp_proposal** out, const stein_icp_proposal_config* cfg)
{
    if (!out) return fail(STEIN_ICP_E_INVALID, "out is NULL");
    *out = nullptr;
    CHECK(validate(cfg));
    MmdScales scales;
    CHECK(make_scales(cfg->n_loss_scales, &cfg->loss_sigma[0][0], scales));
    Model* m = new Model();
    m->scales = scales;
    m->cfg = *cfg;
    m->K = cfg->num_particles;
    m->P = cfg->points;
    m->Bmax = cfg->max_batch;
    const Layout L(m->K);
    m->n_params = L.total;
    const int64_t rows = 2 * m->Bmax * m->P, K6 = 6 * m->K, nch = ceil_div(m->P, kPoolChunk);
    const int64_t slots = 2 * m->Bmax * kF3;
    m->fused_pool = (m->P % kGT) == 0;
    // split-K partials: the largest weight gradient product is W5 (256 x 6K)
    // or W4 (512 x 256); the per-point weights are smaller
    m->ws_floats = (int64_t)kMaxSplits * std::max<int64_t>({(int64_t)kFz * K6, (int64_t)kFcat * kFz, kF2 * kF3});
    m->colpart_floats = std::max<int64_t>(ceil_div(std::max(slots, m->Bmax), kColChunk), 1) * std::max<int64_t>(K6, kF3);
    // arena layout (256-byte aligned blocks)
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_params = take(4 * L.total), o_grad = take(4 * L.total), o_m = take(4 * L.total),
                 o_v = take(4 * L.total);
    const size_t o_H1 = take(m->fused_pool ? 0 : 4 * rows * kF1), o_H2 = take(m->fused_pool ? 0 : 4 * rows * kF2);
    const size_t o_H3 = take(m->fused_pool ? 0 : 4 * rows * kF3);
    const size_t o_keys = take(8 * slots);
    const size_t o_G0 = take(4 * slots * 3), o_G1 = take(4 * slots * kF1), o_G2 = take(4 * slots * kF2);
    const size_t o_dA3 = take(4 * slots * kF3), o_dA2 = take(4 * slots * kF2), o_dA1 = take(4 * slots * kF1);
    const size_t o_pv = take(m->fused_pool ? 0 : 4 * 2 * m->Bmax * nch * kF3);
    const size_t o_pi = take(m->fused_pool ? 0 : 4 * 2 * m->Bmax * nch * kF3);
    const size_t o_arg = take(4 * 2 * m->Bmax * kF3);
    const size_t o_F = take(4 * m->Bmax * kFcat), o_Z = take(4 * m->Bmax * kFz), o_Y = take(4 * m->Bmax * K6);
    const size_t o_dY = take(4 * m->Bmax * K6), o_dZ = take(4 * m->Bmax * kFz), o_dF = take(4 * m->Bmax * kFcat);
    const size_t o_flags = take(4 * m->Bmax);
    const size_t o_ws = take(4 * m->ws_floats), o_cp = take(4 * m->colpart_floats);
    const size_t o_prep = take(4 * 2 * 3 * m->P);
    if (hipMalloc(&m->arena, off) != hipSuccess) {
        (void)hipGetLastError();
        m->arena = nullptr;
        free_model(m);
        return fail(STEIN_ICP_E_NOMEM, "device allocation of the proposal model failed");
    }
    char* a = (char*)m->arena;
    m->params = (float*)(a + o_params);
    m->grad = (float*)(a + o_grad);
    m->adam_m = (float*)(a + o_m);
    m->adam_v = (float*)(a + o_v);
    m->H1 = m->fused_pool ? nullptr : (float*)(a + o_H1);
    m->H2 = m->fused_pool ? nullptr : (float*)(a + o_H2);
    m->H3 = m->fused_pool ? nullptr : (float*)(a + o_H3);
    m->pool_keys = (unsigned long long*)(a + o_keys);
    m->G0 = (float*)(a + o_G0);
    m->G1 = (float*)(a + o_G1);
    m->G2 = (float*)(a + o_G2);
    m->dA3 = (float*)(a + o_dA3);
    m->dA2 = (float*)(a + o_dA2);
    m->dA1 = (float*)(a + o_dA1);
    m->pool_v = (float*)(a + o_pv);
    m->pool_i = (int32_t*)(a + o_pi);
    m->arg = (int32_t*)(a + o_arg);
    m->F = (float*)(a + o_F);
    m->Z = (float*)(a + o_Z);
    m->Y = (float*)(a + o_Y);
    m->dY = (float*)(a + o_dY);
    m->dZ = (float*)(a + o_dZ);
    m->dF = (float*)(a + o_dF);
    m->flags = (int32_t*)(a + o_flags);
    m->ws = (float*)(a + o_ws);
    m->colpart = (float*)(a + o_cp);
    m->prep = (float*)(a + o_prep);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&m->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (m->num_cus < 1) m->num_cus = 256;
    if (hipFuncSetAttribute((const void*)mlp_pool_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMlpLdsBytes) != hipSuccess) {
        (void)hipGetLastError();
        free_model(m);
        return fail(STEIN_ICP_E_DEVICE, "cannot give the fused per-point kernel its LDS");
    }
    if (hipMemset(m->arena, 0, off) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        const hipError_t e = hipGetLastError();
        free_model(m);
        return fail(STEIN_ICP_E_DEVICE, std::string("clearing the proposal model failed: ") + hipGetErrorString(e));
    }
    *out = m;
    return STEIN_ICP_OK;
}

int stein_icp_proposal_destroy(stein_icp_proposal* m)
{
    if (!m) return STEIN_ICP_OK;
    if (hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
    free_model(m);
    return STEIN_ICP_OK;
}

int stein_icp_proposal_set_params(stein_icp_proposal* m, const float* params, void* stream)
{
    if (!m || !params) return fail(STEIN_ICP_E_INVALID, "model or params is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(m->params, params, 4 * m->n_params, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemsetAsync(m->adam_m, 0, 4 * m->n_params, s));
    HIP_TRY(hipMemsetAsync(m->adam_v, 0, 4 * m->n_params, s));
    m->step = 0;
    m->last_batch = 0;
    return STEIN_ICP_OK;
}

int stein_icp_proposal_read_weights(const char* path, float* params, int64_t capacity, int64_t* count,
                                    int32_t* num_particles)
{
    if (!path) return fail(STEIN_ICP_E_INVALID, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(STEIN_ICP_E_INVALID, std::string("cannot open ") + path);
    const auto bad = [&](const std::string& why) {
        std::fclose(f);
        return fail(STEIN_ICP_E_INVALID, std::string(path) + ": " + why);
    };
    // NumPy .npy: magic, version, little-endian header length (2 bytes in
    // version 1, 4 in versions 2 and 3), an ASCII dict literal, the data
    unsigned char pre[10];
    if (std::fread(pre, 1, 8, f) != 8 || std::memcmp(pre, "\x93NUMPY", 6) != 0) return bad("not a .npy file");
    const int major = pre[6];
    uint32_t hlen = 0;
    if (major == 1) {
        if (std::fread(pre + 8, 1, 2, f) != 2) return bad("truncated header");
        hlen = (uint32_t)pre[8] | ((uint32_t)pre[9] << 8);
    } else if (major == 2 || major == 3) {
        unsigned char b[4];
        if (std::fread(b, 1, 4, f) != 4) return bad("truncated header");
        hlen = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
    } else {
        return bad("unsupported .npy version");
    }
    if (hlen > 65536) return bad("header too long");
    std::string h(hlen, '\0');
    if (std::fread(&h[0], 1, hlen, f) != hlen) return bad("truncated header");
    const auto value_of = [&](const char* key) -> std::string {
        const size_t k = h.find(key);
        if (k == std::string::npos) return "";
        size_t v = h.find(':', k);
        if (v == std::string::npos) return "";
        ++v;
        while (v < h.size() && h[v] == ' ') ++v;
        if (v >= h.size()) return "";
        size_t e = v;
        if (h[v] == '(') {
            e = h.find(')', v);
            if (e == std::string::npos) return "";
            ++e;
        } else {
            while (e < h.size() && h[e] != ',' && h[e] != '}') ++e;
        }
        return h.substr(v, e - v);
    };
    if (value_of("'descr'") != "'<f4'") return bad("data must be little-endian float32 ('<f4')");
    if (value_of("'fortran_order'") != "False") return bad("fortran_order must be False");
    const std::string shp = value_of("'shape'");
    long long n = -1;
    char tail[8] = {0};
    if (std::sscanf(shp.c_str(), "(%lld%7[,)]", &n, tail) != 2 || n < 1 || (std::strcmp(tail, ",)") != 0 &&
                                                                              std::strcmp(tail, ")") != 0))
        return bad("shape must be one-dimensional");
    // the count fixes K: total = (fixed part) + 1542 K
    const int64_t fixed = Layout(1).total - 6 * ((int64_t)kFz + 1);
    const int64_t per_k = 6 * ((int64_t)kFz + 1);
    if ((n - fixed) % per_k != 0 || (n - fixed) / per_k < 1 || (n - fixed) / per_k > STEIN_ICP_PROPOSAL_MAX_PARTICLES)
        return bad("parameter count matches no particle count K in [1, 1024]");
    const int32_t K = (int32_t)((n - fixed) / per_k);
    if (count) *count = n;
    if (num_particles) *num_particles = K;
    if (params) {
        if (capacity < n) return bad("params holds fewer than the file's values");
        if (std::fread(params, 4, (size_t)n, f) != (size_t)n) return bad("truncated data");
        for (long long i = 0; i < n; ++i)
            if (!std::isfinite(params[i])) return bad("a parameter is not finite");
    }
    std::fclose(f);
    return STEIN_ICP_OK;
}

int stein_icp_proposal_load(stein_icp_proposal** out, const char* path)
{
    if (!out) return fail(STEIN_ICP_E_INVALID, "out is NULL");
    *out = nullptr;
    int64_t n = 0;
    int32_t K = 0;
    CHECK(stein_icp_proposal_read_weights(path, nullptr, 0, &n, &K));
    std::vector<float> host((size_t)n);
    CHECK(stein_icp_proposal_read_weights(path, host.data(), n, &n, &K));
    stein_icp_proposal_config cfg;
    CHECK(stein_icp_proposal_default_config(&cfg));
    cfg.num_particles = K;
    stein_icp_proposal* m = nullptr;
    CHECK(stein_icp_proposal_create(&m, &cfg));
    if (hipMemcpy(m->params, host.data(), 4 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        free_model(m);
        return fail(STEIN_ICP_E_DEVICE, std::string("uploading the weights failed: ") + hipGetErrorString(e));
    }
    *out = m;
    return STEIN_ICP_OK;
}

int stein_icp_proposal_get_params(const stein_icp_proposal* m, float* params, void* stream)
{
    if (!m || !params) return fail(STEIN_ICP_E_INVALID, "model or params is NULL");
    HIP_TRY(hipMemcpyAsync(params, m->params, 4 * m->n_params, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return STEIN_ICP_OK;
}

int stein_icp_proposal_prepare(const stein_icp_proposal* m, const float* xyz, int64_t n, float* out, void* stream)
{
    if (!m || !xyz || !out) return fail(STEIN_ICP_E_INVALID, "model, xyz or out is NULL");
    if (n < 1 || n > ((int64_t)1 << 40) / m->P) return fail(STEIN_ICP_E_INVALID, "cloud size out of range");
    subsample_kernel<<<(unsigned)ceil_div(m->P, 256), 256, 0, (hipStream_t)stream>>>(xyz, n, m->P, out);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

int stein_icp_proposal_forward(stein_icp_proposal* m, const float* clouds, int32_t B, double* particles,
                               int32_t* nonfinite, void* stream)
{
    if (!m || !clouds || !particles) return fail(STEIN_ICP_E_INVALID, "model, clouds or particles is NULL");
    if (B < 1 || B > m->Bmax) return fail(STEIN_ICP_E_INVALID, "batch must be in [1, max_batch]");
    hipStream_t s = (hipStream_t)stream;
    CHECK(forward(m, s, clouds, B));
    const int64_t n = (int64_t)B * 6 * m->K;
    int32_t* flags = nonfinite ? nonfinite : m->flags;
    fill_i32_kernel<<<(unsigned)ceil_div(B, 256), 256, 0, s>>>(flags, B, 0);
    output_particles_kernel<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(m->Y, n, 6 * m->K, particles, flags);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

int stein_icp_proposal_loss(stein_icp_proposal* m, const float* clouds, const double* targets, int32_t B,
                            double* loss, float* grad, void* stream)
{
    if (!m || !clouds || !targets || !loss) return fail(STEIN_ICP_E_INVALID, "model, clouds, targets or loss is NULL");
    if (B < 1 || B > m->Bmax) return fail(STEIN_ICP_E_INVALID, "batch must be in [1, max_batch]");
    hipStream_t s = (hipStream_t)stream;
    CHECK(forward(m, s, clouds, B));
    CHECK(launch_mmd(s, m->Y, nullptr, targets, B, (int32_t)m->K, m->scales, 1.0 / B, m->dY, loss));
    CHECK(backward(m, s, clouds, B));
    if (grad) HIP_TRY(hipMemcpyAsync(grad, m->grad, 4 * m->n_params, hipMemcpyDeviceToDevice, s));
    m->last_batch = B;
    return STEIN_ICP_OK;
}

int stein_icp_proposal_adam(stein_icp_proposal* m, double lr, double b1, double b2, double eps, void* stream)
{
    if (!m) return fail(STEIN_ICP_E_INVALID, "model is NULL");
    if (m->last_batch == 0) return fail(STEIN_ICP_E_STATE, "no gradient: call stein_icp_proposal_loss first");
    if (!(std::isfinite(lr) && lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && std::isfinite(eps) && eps > 0))
        return fail(STEIN_ICP_E_INVALID, "need lr > 0, 0 <= beta < 1, eps > 0");
    m->step += 1;
    const double bc1 = 1.0 - std::pow(b1, (double)m->step), bc2 = 1.0 - std::pow(b2, (double)m->step);
    adam_kernel<<<(unsigned)ceil_div(m->n_params, 256), 256, 0, (hipStream_t)stream>>>(
        m->params, m->grad, m->adam_m, m->adam_v, m->n_params, lr, b1, b2, eps, bc1, bc2);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

int stein_icp_proposal_mmd(const double* X, const double* Y, int32_t B, int32_t K, int32_t ns, const double* sigma,
                           double* out, void* stream)
{
    if (!X || !Y || !out) return fail(STEIN_ICP_E_INVALID, "X, Y or out is NULL");
    if (B < 1 || K < 1 || K > STEIN_ICP_PROPOSAL_MAX_PARTICLES)
        return fail(STEIN_ICP_E_INVALID, "need batch >= 1 and K in [1, 1024]");
    MmdScales sc;
    CHECK(make_scales(ns, sigma, sc));
    return launch_mmd((hipStream_t)stream, nullptr, X, Y, B, K, sc, 0.0, nullptr, out);
}

int stein_icp_propose(stein_icp_proposal* m, const float* src, int64_t n_src, const float* ref, int64_t n_ref,
                      double* particles, int32_t* used_fallback, void* stream)
{
    if (!m || !src || !ref || !particles || !used_fallback)
        return fail(STEIN_ICP_E_INVALID, "model, clouds, particles or used_fallback is NULL");
    hipStream_t s = (hipStream_t)stream;
    CHECK(stein_icp_proposal_prepare(m, src, n_src, m->prep, stream));
    CHECK(stein_icp_proposal_prepare(m, ref, n_ref, m->prep + 3 * m->P, stream));
    CHECK(stein_icp_proposal_forward(m, m->prep, 1, particles, m->flags, stream));
    int32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, m->flags, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *used_fallback = bad ? 1 : 0;
    return STEIN_ICP_OK;
}

int stein_icp_gemm_bf16(int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                        const float* B, int64_t ldb, float* C, int64_t ldc, const float* bias, int32_t relu,
                        int32_t accumulate, int32_t splits, float* workspace, void* stream)
{
    if (M < 0 || N < 0 || K < 0 || (ta != 0 && ta != 1) || (tb != 0 && tb != 1))
        return fail(STEIN_ICP_E_INVALID, "need M, N, K >= 0 and ta, tb in {0, 1}");
    // empty operands may be NULL: nothing is read from them
    if ((M > 0 && N > 0 && !C) || (M > 0 && K > 0 && !A) || (N > 0 && K > 0 && !B))
        return fail(STEIN_ICP_E_INVALID, "A, B or C is NULL");
    if ((ceil_div(M, kGT) + kXcds) * ceil_div(N, kGT) * kXcds >= ((int64_t)1 << 31))
        return fail(STEIN_ICP_E_INVALID, "M x N too large for one launch");
    if (lda < (ta ? M : K) || ldb < (tb ? K : N) || ldc < N)
        return fail(STEIN_ICP_E_INVALID, "leading dimension smaller than the row length");
    if (splits < 1 || splits > kMaxSplits) return fail(STEIN_ICP_E_INVALID, "splits must be in [1, 64]");
    if (splits > 1 && !workspace) return fail(STEIN_ICP_E_INVALID, "splits > 1 needs a workspace");
    return launch_gemm((hipStream_t)stream, ta, tb, M, N, K, A, lda, B, ldb, C, ldc, bias, relu, accumulate, splits,
                       workspace);
}

}  // extern "C"
