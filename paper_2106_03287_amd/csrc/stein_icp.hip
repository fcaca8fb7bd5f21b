// Host side of the Stein-ICP library: validation, device layout, tiling,
// hipGraph capture and the C ABI declared in include/stein_icp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "stein_icp.h"

#include "common.hpp"
#include "grad_bw.hpp"
#include "nn.hpp"
#include "nn_bf16_launch.h"
#include "normals.hpp"
#include "prep.hpp"
#include "svgd.hpp"

using namespace sicp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(STEIN_ICP_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Centre of the BF16 screen (the reference centroid, rounded to FP32) in
// c0[0..2] and, in c0[3], an upper bound of the norms of the centred
// references as the kernels form them (FP32 differences), which sizes the
// screen's error bound.
void bf16_centre(const float* xyz, int64_t n, PairDesc& pd)
{
    double acc[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) acc[d] += xyz[3 * i + d];
    for (int d = 0; d < 3; ++d) pd.c0[d] = std::isfinite(acc[d]) ? (float)(acc[d] / n) : 0.0f;
    double r2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double q = 0.0;
        for (int d = 0; d < 3; ++d) {
            const float c = xyz[3 * i + d] - pd.c0[d];   // FP32, as in the kernels
            q += (double)c * c;
        }
        r2 = std::max(r2, q);
    }
    pd.c0[3] = std::nextafter((float)(std::sqrt(r2) * (1.0 + 0x1.0p-20)), INFINITY);
    pd.sexp = f16_screen_exponent_host(pd.c0[3]);
}
inline int64_t ceil_div(int64_t v, int64_t a) { return (v + a - 1) / a; }
// The two certified matrix-core screens (BF16 x 3, FP16 x 2) against the
// plain FP32 search.
inline bool is_screen(int32_t mode) { return mode == STEIN_ICP_NN_BF16_RERANK || mode == STEIN_ICP_NN_F16_RERANK; }
inline int screen_fmt(int32_t mode) { return mode == STEIN_ICP_NN_F16_RERANK ? kFmtF16x2 : kFmtBf16x3; }
inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ------------------------------------------------------------------ host RNG
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).
struct SplitMix64 {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }  // [0, 1)
};

void make_schedule(uint64_t seed, int64_t n, int32_t m, int32_t rows, int32_t* out)
{
    SplitMix64 g{seed ^ 0x5DEECE66Dull};
    std::vector<uint8_t> used((size_t)n, 0);
    for (int32_t r = 0; r < rows; ++r) {
        int32_t* row = out + (int64_t)r * m;
        int32_t c = 0;
        // Floyd's algorithm: m distinct values from [0, n)
        for (int64_t j = n - m; j < n; ++j) {
            const int64_t t = (int64_t)(g.next() % (uint64_t)(j + 1));
            const int64_t v = used[(size_t)t] ? j : t;
            used[(size_t)v] = 1;
            row[c++] = (int32_t)v;
        }
        for (int32_t i = 0; i < m; ++i) used[(size_t)row[i]] = 0;
    }
}

void make_init(uint64_t seed, int32_t K, double ht, double hr, const double* centre, double* out)
{
    SplitMix64 g{seed ^ 0xA0761D6478BD642Full};
    for (int32_t k = 0; k < K; ++k)
        for (int d = 0; d < 6; ++d) {
            const double c = centre ? centre[d] : 0.0;
            const double h = d < 3 ? ht : hr;
            out[6 * k + d] = c + (2.0 * g.uniform() - 1.0) * h;
        }
}

// ------------------------------------------------------------------ tiling
struct Tiling {
    int q = 2;                   // queries per lane
    int w = 4;                   // wavefronts per workgroup
    int persist = 0;             // 0: one workgroup per item; n: n workgroups per CU, grid-stride
    std::vector<int32_t> chunk;  // per pair, references per chunk
};

// Default shape: enough workgroups to give every SIMD several waves, with at
// least 64 references (4 tiles) per wave; the autotuner refines it.
int default_queries_per_lane(int64_t nq) { return nq >= 65536 ? 4 : (nq >= 8192 ? 2 : 1); }

// References per chunk for a pair of n_ref_pad references when `pairs` pairs
// of nq queries each (q per lane) share the launch.
int32_t default_chunk(int64_t n_ref_pad, int64_t nq, int q, int64_t pairs)
{
    const int64_t qb = ceil_div(nq, (int64_t)kWave * q);
    const int64_t target_wg = 4096;  // x4 waves = 16k waves over 1024 SIMDs
    const int64_t per_pair = std::max<int64_t>(1, ceil_div(target_wg, pairs * qb));
    const int64_t max_chunks = std::max<int64_t>(1, n_ref_pad / (4 * 64));
    const int64_t c = std::min(per_pair, max_chunks);
    return (int32_t)round_up(ceil_div(n_ref_pad, c), 4 * kTile);
}

Tiling default_tiling(const std::vector<PairDesc>& pd, int64_t nq)
{
    Tiling t;
    t.q = default_queries_per_lane(nq);
    for (const auto& p : pd) t.chunk.push_back(default_chunk(p.n_ref_pad, nq, t.q, (int64_t)pd.size()));
    return t;
}

// Tuned shapes by (pairs, queries per pair, total padded references),
// shared by every context of the process.
struct TuneKey {
    int32_t P;
    int64_t nq, refs;
    bool operator<(const TuneKey& o) const
    {
        return P != o.P ? P < o.P : (nq != o.nq ? nq < o.nq : refs < o.refs);
    }
};
std::map<TuneKey, std::pair<Tiling, double>> g_tuned;

}  // namespace

// ------------------------------------------------------------------ context
struct stein_icp_ctx {
    stein_icp_config cfg{};
    int device = 0;
    int32_t P = 0, K = 0, m = 0, rows = 0;
    int64_t nq = 0;  // K * m per pair
    std::vector<PairDesc> pairs;
    Tiling tiling;
    std::vector<WorkItem> work;
    double tuned_ms = 0.0;

    char* arena = nullptr;
    PairDesc* d_pairs = nullptr;
    std::vector<PairDesc> groups;   // NN groups (runs of consecutive pairs on one packed reference)
    PairDesc* d_groups = nullptr;
    float4* src4 = nullptr;
    float4* ref4 = nullptr;
    int32_t* sched = nullptr;
    // theta / step are the current particles and step counts, theta_next /
    // step_next what the coming update writes; the two swap after every
    // iteration (parity 0: the first of each pair of buffers is current)
    double *theta = nullptr, *theta_next = nullptr, *mom = nullptr, *vel = nullptr, *gbar = nullptr, *phi = nullptr;
    double* h = nullptr;
    int64_t *step = nullptr, *step_next = nullptr;
    int parity = 0;
    Pose* pose = nullptr;
    float4* queries = nullptr;   // FP32 queries of the coming iteration, K*m per pair
    uint4* apack = nullptr;      // BF16 reference fragments (BF16 screen only)
    int32_t* match = nullptr;
    double* nrm = nullptr;       // point-to-plane: (n, 0) per packed reference, FP64
    double* dscr = nullptr;
    int* flag = nullptr;
    unsigned long long* rescans = nullptr;   // failed screen certificates (BF16 search), accumulated
    int64_t certificates = 0;                // screen certificates enqueued so far (host count)

    WorkItem* d_work = nullptr;  // separate allocations: resized by the tuner
    uint64_t* partial = nullptr;

    hipStream_t cap_stream = nullptr;   // graph capture
    std::map<int, hipGraphExec_t> graphs;   // key 2 * iterations + starting parity
};

namespace {

// The bandwidths do not depend on the particles: a fixed bandwidth, or one
// particle (h = 1 then, as the median heuristic's guard gives).
bool const_bandwidth(const stein_icp_config& c)
{
    return c.bandwidth_mode == STEIN_ICP_BW_FIXED || c.num_particles < 2;
}

// With a matrix-core screen, dynamic LDS up to this and at most two
// particles per compute unit (the gradient launch then holds few
// workgroups, and the bandwidth selection beside them took longer than the
// gradients), the median bandwidths run as extra workgroups of the
// nearest-neighbour launch, beside the search: with the pair keys in LDS up
// to K of about 128, with the distances in global memory up to K of about
// 490. With many pairs the gradients take longer than the selection, and the
// extra workgroups would only delay the search. (The FP32 search keeps them
// in the gradient launch: the selection's registers would cost it
// occupancy.) Every workgroup of the launch takes the dynamic LDS, so the
// bound keeps two search workgroups per compute unit.
constexpr size_t kFusedBandwidthLds = 48 * 1024;
int g_num_cus = 256;   // compute units of the device, read at the first init

// Where the fused bandwidth workgroups keep the pair distances: keys in LDS
// where they fit, else keys in global memory (the keyed selection reads a
// quarter of the bytes of FP64 distances, in fewer passes), else FP64.
int fused_bandwidth_form(int K)
{
    if (!bandwidth_keyable(K)) return kDistancesInGlobal;
    return bandwidth_role_lds_bytes(K, kKeysInLds) <= kFusedBandwidthLds ? kKeysInLds : kKeysInGlobal;
}

bool fused_bandwidth(const stein_icp_config& c, int64_t pairs)
{
    const int K = c.num_particles;
    return is_screen(c.nn_mode) && !const_bandwidth(c) &&
           bandwidth_role_lds_bytes(K, fused_bandwidth_form(K)) <= kFusedBandwidthLds &&
           pairs * K <= 2 * (int64_t)g_num_cus;
}

SvgdParams svgd_params(const stein_icp_config& c)
{
    SvgdParams p{};
    p.lr = c.lr;
    p.beta1 = c.beta1;
    p.beta2 = c.beta2;
    p.eps = c.eps;
    p.h_fixed_t = c.fixed_h_trans;
    p.h_fixed_r = c.fixed_h_rot;
    for (int i = 0; i < 6; ++i) p.prior_mu[i] = c.prior_mu[i];
    for (int i = 0; i < 3; ++i) {
        p.prior_var[i] = c.prior_var_trans[i];
        p.prior_kappa[i] = c.prior_kappa_rot[i];
    }
    p.optimizer = c.optimizer;
    p.bandwidth = c.bandwidth_mode;
    p.prior = c.prior_mode;
    return p;
}

int validate_config(const stein_icp_config* c)
{
    if (!c) return fail(STEIN_ICP_E_INVALID, "cfg is NULL");
    if (c->struct_size != sizeof(stein_icp_config))
        return fail(STEIN_ICP_E_INVALID, "cfg->struct_size does not match this library's stein_icp_config");
    if (c->num_particles < 1 || c->num_particles > kMaxK)
        return fail(STEIN_ICP_E_INVALID, "num_particles must be in [1, 1024]");
    if (c->batch_size < 1) return fail(STEIN_ICP_E_INVALID, "batch_size must be >= 1");
    if (c->schedule_rows < 1) return fail(STEIN_ICP_E_INVALID, "schedule_rows must be >= 1");
    if ((int64_t)c->schedule_rows * c->batch_size > (int64_t)1 << 31)
        return fail(STEIN_ICP_E_INVALID, "schedule_rows * batch_size too large");
    if (!finite_pos(c->lr)) return fail(STEIN_ICP_E_INVALID, "lr must be finite and > 0");
    if (!(c->beta1 >= 0.0 && c->beta1 < 1.0) || !(c->beta2 >= 0.0 && c->beta2 < 1.0))
        return fail(STEIN_ICP_E_INVALID, "beta1 and beta2 must be in [0, 1)");
    if (!finite_pos(c->eps)) return fail(STEIN_ICP_E_INVALID, "eps must be finite and > 0");
    if (!(std::isfinite(c->init_half_trans) && c->init_half_trans >= 0.0) ||
        !(std::isfinite(c->init_half_rot) && c->init_half_rot >= 0.0))
        return fail(STEIN_ICP_E_INVALID, "init half widths must be finite and >= 0");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(c->init_centre[i])) return fail(STEIN_ICP_E_INVALID, "init_centre must be finite");
    if (c->nn_mode != STEIN_ICP_NN_FP32 && !is_screen(c->nn_mode))
        return fail(STEIN_ICP_E_INVALID, "unknown nn_mode");
    if (c->optimizer != STEIN_ICP_OPT_ADAM && c->optimizer != STEIN_ICP_OPT_SGD)
        return fail(STEIN_ICP_E_INVALID, "unknown optimizer");
    if (c->bandwidth_mode != STEIN_ICP_BW_MEDIAN && c->bandwidth_mode != STEIN_ICP_BW_FIXED)
        return fail(STEIN_ICP_E_INVALID, "unknown bandwidth_mode");
    if (c->bandwidth_mode == STEIN_ICP_BW_FIXED && (!finite_pos(c->fixed_h_trans) || !finite_pos(c->fixed_h_rot)))
        return fail(STEIN_ICP_E_INVALID, "fixed bandwidths must be finite and > 0");
    if (c->prior_mode != STEIN_ICP_PRIOR_UNIFORM && c->prior_mode != STEIN_ICP_PRIOR_GAUSS_VONMISES)
        return fail(STEIN_ICP_E_INVALID, "unknown prior_mode");
    if (c->prior_mode == STEIN_ICP_PRIOR_GAUSS_VONMISES) {
        for (int i = 0; i < 6; ++i)
            if (!std::isfinite(c->prior_mu[i])) return fail(STEIN_ICP_E_INVALID, "prior_mu must be finite");
        for (int i = 0; i < 3; ++i) {
            if (!finite_pos(c->prior_var_trans[i]))
                return fail(STEIN_ICP_E_INVALID, "prior_var_trans must be finite and > 0");
            if (!(std::isfinite(c->prior_kappa_rot[i]) && c->prior_kappa_rot[i] >= 0.0))
                return fail(STEIN_ICP_E_INVALID, "prior_kappa_rot must be finite and >= 0");
        }
    }
    if (c->n_scale < 0) return fail(STEIN_ICP_E_INVALID, "n_scale must be >= 0");
    if (c->use_graph != 0 && c->use_graph != 1) return fail(STEIN_ICP_E_INVALID, "use_graph must be 0 or 1");
    if (c->autotune != 0 && c->autotune != 1) return fail(STEIN_ICP_E_INVALID, "autotune must be 0 or 1");
    if (c->metric != STEIN_ICP_METRIC_POINT && c->metric != STEIN_ICP_METRIC_PLANE)
        return fail(STEIN_ICP_E_INVALID, "unknown metric");
    if (c->normal_k < 3 || c->normal_k > kKnnMax) return fail(STEIN_ICP_E_INVALID, "normal_k must be in [3, 32]");
    return STEIN_ICP_OK;
}

constexpr int64_t kMaxRef = ((int64_t)1 << 31) - 64;

dim3 grid1d(int64_t n, int threads) { return dim3((unsigned)ceil_div(std::max<int64_t>(n, 1), threads)); }


// Launch the NN kernel with q queries per lane and w wavefronts per workgroup.
template <int Q>
void launch_nn_q(int w, unsigned nwork, const NNArgs& a, hipStream_t s)
{
    switch (w) {
    case 4: hipLaunchKernelGGL((nn_fp32_kernel<Q, 4>), dim3(nwork), dim3(kWave * 4), 0, s, a); break;
    case 8: hipLaunchKernelGGL((nn_fp32_kernel<Q, 8>), dim3(nwork), dim3(kWave * 8), 0, s, a); break;
    default: hipLaunchKernelGGL((nn_fp32_kernel<Q, 16>), dim3(nwork), dim3(kWave * 16), 0, s, a); break;
    }
}

// BF16 screen + FP32 rerank with the same work table and key format.
hipError_t launch_nn_bf16(const Tiling& t, unsigned nwork, NNBf16Args a, int fmt, hipStream_t s)
{
    if (nwork == 0) return hipSuccess;
    if (t.w != 4 && t.w != 8 && t.w != 16) return hipErrorInvalidValue;
    a.nwork = nwork;
    const unsigned grid = t.persist > 0 ? std::min<unsigned>(nwork, (unsigned)(t.persist * g_num_cus)) : nwork;
    int64_t min_chunk = t.chunk.empty() ? 0 : INT64_MAX;
    for (const int32_t c : t.chunk) min_chunk = std::min<int64_t>(min_chunk, c);
    return launch_nn_bf16_kernel(t.q, t.w, fmt, nn_bf16_key_span(t.q, t.w, min_chunk), grid, a, s);
}

hipError_t launch_nn(const Tiling& t, unsigned nwork, NNArgs a, hipStream_t s)
{
    if (nwork == 0) return hipSuccess;
    if (t.w != 4 && t.w != 8 && t.w != 16) return hipErrorInvalidValue;
    a.nwork = nwork;
    const unsigned grid = t.persist > 0 ? std::min<unsigned>(nwork, (unsigned)(t.persist * g_num_cus)) : nwork;
    switch (t.q) {
    case 1: launch_nn_q<1>(t.w, grid, a, s); break;
    case 2: launch_nn_q<2>(t.w, grid, a, s); break;
    case 4: launch_nn_q<4>(t.w, grid, a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// NN groups and the work table. Consecutive pairs on the same packed
// reference with the same chunking form one group: their queries are
// contiguous, so the search runs them as one query set (full query blocks
// where each pair alone would leave a ragged one). A group's chunk keys are
// chunk-major over all its queries; pair l of the group finds its keys at
// part_off + l K m with stride part_stride.
void build_work(stein_icp_ctx* c)
{
    c->work.clear();
    c->groups.clear();
    for (int32_t p = 0; p < c->P; ++p) {
        PairDesc& pd = c->pairs[p];
        pd.chunk = c->tiling.chunk[p];
        pd.chunks = (int32_t)ceil_div(pd.n_ref_pad, pd.chunk);
    }
    int64_t part = 0;
    for (int32_t p0 = 0; p0 < c->P;) {
        int32_t p1 = p0 + 1;
        while (p1 < c->P && c->pairs[p1].ref_off == c->pairs[p0].ref_off &&
               c->pairs[p1].n_ref_pad == c->pairs[p0].n_ref_pad && c->pairs[p1].chunk == c->pairs[p0].chunk)
            ++p1;
        PairDesc g = c->pairs[p0];
        g.nq = (int64_t)(p1 - p0) * c->nq;
        g.q_off = c->pairs[p0].q_off;
        g.qblocks = (int32_t)ceil_div(g.nq, (int64_t)kWave * c->tiling.q);
        g.part_off = part;
        g.part_stride = g.nq;
        for (int32_t p = p0; p < p1; ++p) {
            PairDesc& pd = c->pairs[p];
            pd.part_off = part + (int64_t)(p - p0) * c->nq;
            pd.part_stride = g.nq;
            pd.qblocks = g.qblocks;
        }
        part += (int64_t)g.chunks * g.nq;
        c->groups.push_back(g);
        p0 = p1;
    }
    // chunk-major order inside a group so neighbouring workgroups (which the
    // dispatcher spreads round-robin over the eight XCDs) read different
    // chunks of the same queries: with two chunks, XCD x always searches
    // chunk x mod 2. Many pairs' fragments together exceed an XCD's L2
    // (each XCD then fills every pair's once per launch), but the search
    // stays far from the HBM bound there.
    for (int32_t gi = 0; gi < (int32_t)c->groups.size(); ++gi) {
        const PairDesc& g = c->groups[gi];
        for (int32_t b = 0; b < g.qblocks; ++b)
            for (int32_t ch = 0; ch < g.chunks; ++ch) c->work.push_back(WorkItem{gi, b, ch, 0});
    }
}

// Screen certificates one NN launch evaluates: every real query, for every
// chunk, once per lane half (two) and per wavefront that holds blocks of the
// chunk (min(waves, blocks)).
int64_t certificates_per_launch(const stein_icp_ctx* c)
{
    if (!is_screen(c->cfg.nn_mode)) return 0;
    int64_t n = 0;
    for (const auto& g : c->groups)
        for (int32_t ch = 0; ch < g.chunks; ++ch) {
            const int64_t blocks = (std::min<int64_t>((int64_t)(ch + 1) * g.chunk, g.n_ref_pad) -
                                    (int64_t)ch * g.chunk) / kRefPad;
            n += g.nq * 2 * std::min<int64_t>(c->tiling.w, blocks);
        }
    return n;
}

int64_t partial_elems(const stein_icp_ctx* c)
{
    int64_t n = 0;
    for (const auto& g : c->groups) n += (int64_t)g.chunks * g.nq;
    return n;
}

int upload_tiling(stein_icp_ctx* c, hipStream_t s)
{
    build_work(c);
    if (c->d_work) HIP_TRY(hipFree(c->d_work));
    if (c->partial) HIP_TRY(hipFree(c->partial));
    c->d_work = nullptr;
    c->partial = nullptr;
    if (hipMalloc(&c->d_work, sizeof(WorkItem) * std::max<size_t>(c->work.size(), 1)) != hipSuccess ||
        hipMalloc(&c->partial, sizeof(uint64_t) * std::max<int64_t>(partial_elems(c), 1)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STEIN_ICP_E_NOMEM, "device allocation of the NN work table failed");
    }
    HIP_TRY(hipMemcpyAsync(c->d_pairs, c->pairs.data(), sizeof(PairDesc) * c->P, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->d_groups, c->groups.data(), sizeof(PairDesc) * c->groups.size(),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->d_work, c->work.data(), sizeof(WorkItem) * c->work.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    return STEIN_ICP_OK;
}

NNArgs nn_args(const stein_icp_ctx* c)
{
    NNArgs a{};
    a.work = c->d_work;
    a.pairs = c->d_groups;
    a.ref4 = c->ref4;
    a.queries = c->queries;
    a.partial = c->partial;
    return a;
}

SvgdArgs svgd_args(const stein_icp_ctx* c)
{
    SvgdArgs v{};
    v.pairs = c->d_pairs;
    v.theta = c->theta;
    v.theta_next = c->theta_next;
    v.mom = c->mom;
    v.vel = c->vel;
    v.step = c->step;
    v.step_next = c->step_next;
    v.gbar = c->gbar;
    v.phi = c->phi;
    v.h = c->h;
    v.dscr = c->dscr;
    v.pose = c->pose;
    v.src4 = c->src4;
    v.sched = c->sched;
    v.queries = c->queries;
    v.K = c->K;
    v.m = c->m;
    v.rows = c->rows;
    v.prm = svgd_params(c->cfg);
    return v;
}

// Queries of the coming iteration from the current poses and step count.
hipError_t enqueue_queries(const stein_icp_ctx* c, hipStream_t s)
{
    hipLaunchKernelGGL(queries_kernel, dim3((unsigned)ceil_div(c->nq, 256), (unsigned)c->P), dim3(256), 0, s,
                       c->d_pairs, c->src4, c->sched, c->pose, c->step, c->queries, c->K, c->m, c->rows);
    return hipGetLastError();
}

// Stage 0: nearest neighbours, 1: gradients and bandwidths (one launch),
// 2: Stein direction and update (into theta_next / step_next).
hipError_t enqueue_stage(const stein_icp_ctx* c, int stage, hipStream_t s)
{
    if (stage == 0) {
        if (is_screen(c->cfg.nn_mode)) {
            NNBf16Args b{};
            b.work = c->d_work;
            b.pairs = c->d_groups;
            b.ref4 = c->ref4;
            b.apack = c->apack;
            b.queries = c->queries;
            b.partial = c->partial;
            b.rescans = c->rescans;
            if (fused_bandwidth(c->cfg, c->P)) {
                b.bw = svgd_args(c);
                b.bw_blocks = 2 * c->P;
                b.bw_form = fused_bandwidth_form(c->K);
                b.bw_lds = (uint32_t)bandwidth_role_lds_bytes(c->K, b.bw_form);
            }
            return launch_nn_bf16(c->tiling, (unsigned)c->work.size(), b, screen_fmt(c->cfg.nn_mode), s);
        }
        return launch_nn(c->tiling, (unsigned)c->work.size(), nn_args(c), s);
    }
    if (stage == 1) {
    GradArgs g{};
    g.pairs = c->d_pairs;
    g.src4 = c->src4;
    g.ref4 = c->ref4;
    g.queries = c->queries;
    g.sched = c->sched;
    g.pose = c->pose;
    g.step = c->step;
    g.partial = c->partial;
    g.match = c->match;
    g.gbar = c->gbar;
    g.nrm = c->cfg.metric == STEIN_ICP_METRIC_PLANE ? c->nrm : nullptr;
    g.K = c->K;
    g.m = c->m;
    g.rows = c->rows;
    g.index_keys = is_screen(c->cfg.nn_mode) ? 1 : 0;
    const int32_t bw_pairs = const_bandwidth(c->cfg) || fused_bandwidth(c->cfg, c->P) ? 0 : c->P;
    const int64_t blocks = 2 * (int64_t)bw_pairs + ceil_div((int64_t)c->P * c->K, kGradGroups);
    hipLaunchKernelGGL(grad_bandwidth_kernel, dim3((unsigned)blocks), dim3(kSvgdThreads), grad_bw_lds_bytes(c->K), s,
                       g, svgd_args(c), c->P, bw_pairs);
    return hipGetLastError();
    }
    const SvgdArgs v = svgd_args(c);
    hipLaunchKernelGGL(svgd_phi_update_kernel, dim3((unsigned)c->K, (unsigned)c->P), dim3(kPhiThreads), 0, s, v);
    return hipGetLastError();
}

// After n enqueued iterations the buffers the updates wrote are current.
void advance(stein_icp_ctx* c, int64_t n)
{
    if (n & 1) {
        std::swap(c->theta, c->theta_next);
        std::swap(c->step, c->step_next);
        c->parity ^= 1;
    }
}

constexpr int kStages = 3;  // nearest neighbours, gradients + bandwidths, direction + update

// One iteration in stream order on `s`.
hipError_t enqueue_iteration(const stein_icp_ctx* c, hipStream_t s)
{
    for (int st = 0; st < kStages; ++st) {
        const hipError_t e = enqueue_stage(c, st, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Graph of `len` iterations starting from the context's current parity
// (the kernels' buffer arguments are fixed at capture).
int get_graph(stein_icp_ctx* c, int len, hipGraphExec_t* out)
{
    const int key = 2 * len + c->parity;
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return STEIN_ICP_OK;
    }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    // the capture walks the buffers forward; the launch advances them for real
    double* const th0 = c->theta;
    double* const th1 = c->theta_next;
    int64_t* const st0 = c->step;
    int64_t* const st1 = c->step_next;
    const int par = c->parity;
    for (int i = 0; i < len && e == hipSuccess; ++i) {
        e = enqueue_iteration(c, c->cap_stream);
        advance(c, 1);
    }
    c->theta = th0;
    c->theta_next = th1;
    c->step = st0;
    c->step_next = st1;
    c->parity = par;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(STEIN_ICP_E_DEVICE, std::string("graph capture failed: ") +
                                            hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    c->graphs[key] = ex;
    *out = ex;
    return STEIN_ICP_OK;
}

constexpr int kGraphIters = 25;

int run_iters(stein_icp_ctx* c, int32_t n, hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &st));
    c->certificates += (int64_t)n * certificates_per_launch(c);
    if (!c->cfg.use_graph || st != hipStreamCaptureStatusNone) {
        for (int32_t i = 0; i < n; ++i) {
            HIP_TRY(enqueue_iteration(c, s));
            advance(c, 1);
        }
        return STEIN_ICP_OK;
    }
    int32_t left = n;
    while (left > 0) {
        const int len = std::min<int32_t>(left, kGraphIters);
        hipGraphExec_t ex;
        int rc = get_graph(c, len, &ex);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(ex, s));
        advance(c, len);
        left -= len;
    }
    return STEIN_ICP_OK;
}

// Autotuner: time candidate NN shapes (queries per lane, wavefronts per
// workgroup, references per wavefront) on the context's own data with the
// real nearest-neighbour and gradient kernels (the chunk count trades NN
// parallelism against the gradient kernel's reduction over chunks) and keep
// the fastest. Shapes change only the work decomposition, never the
// arithmetic, so results are identical for every candidate. Results are
// cached per (pairs, queries, references) for the process.
int autotune(stein_icp_ctx* c, hipStream_t s)
{
    int64_t refs = 0;
    for (const auto& pd : c->pairs) refs += pd.n_ref_pad;
    const TuneKey tk{c->P, c->nq, refs};
    auto hit = g_tuned.find(tk);
    if (hit != g_tuned.end()) {
        c->tiling = hit->second.first;
        c->tuned_ms = hit->second.second;
        return upload_tiling(c, s);
    }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e30;
    Tiling best_t = c->tiling;
    std::set<std::vector<int32_t>> seen;
    const bool bf16 = is_screen(c->cfg.nn_mode);
    for (int q : {1, 2, 4})
        for (int w : {4, 8, 16})
            for (int64_t pw : {64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384}) {
                if (bf16 && !nn_bf16_shape_ok(q, w)) continue;
                Tiling t;
                t.q = q;
                t.w = w;
                for (const auto& pd : c->pairs) {
                    const int64_t chunks = std::max<int64_t>(1, ceil_div(pd.n_ref_pad, (int64_t)w * pw));
                    t.chunk.push_back((int32_t)round_up(ceil_div(pd.n_ref_pad, chunks), (int64_t)w * kTile));
                }
                std::vector<int32_t> sig = t.chunk;
                sig.push_back(q);
                sig.push_back(w);
                if (!seen.insert(sig).second) continue;   // same shape as an earlier span
                c->tiling = t;
                int rc = upload_tiling(c, s);
                if (rc) return rc;
                HIP_TRY(enqueue_stage(c, 0, s));  // warm-up
                HIP_TRY(enqueue_stage(c, 1, s));
                const int reps = 10;
                HIP_TRY(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) {
                    HIP_TRY(enqueue_stage(c, 0, s));
                    HIP_TRY(enqueue_stage(c, 1, s));
                }
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms / reps < best) {
                    best = ms / reps;
                    best_t = t;
                }
            }
    // persistent grids on the best shape
    for (int per : {1, 2, 4, 8}) {
        Tiling t = best_t;
        t.persist = per;
        c->tiling = t;
        int rc = upload_tiling(c, s);
        if (rc) return rc;
        HIP_TRY(enqueue_stage(c, 0, s));
        HIP_TRY(enqueue_stage(c, 1, s));
        const int reps = 10;
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) {
            HIP_TRY(enqueue_stage(c, 0, s));
            HIP_TRY(enqueue_stage(c, 1, s));
        }
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best) {
            best = ms / reps;
            best_t = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tiling = best_t;
    c->tuned_ms = best;
    g_tuned[tk] = {best_t, best};
    const int rc = upload_tiling(c, s);
    if (rc) return rc;
    // the tuner's trial launches are not counted
    HIP_TRY(hipMemsetAsync(c->rescans, 0, sizeof(unsigned long long), s));
    HIP_TRY(hipStreamSynchronize(s));
    return STEIN_ICP_OK;
}

// The k nearest of n_ref references for nq queries (device float4 arrays)
// and, if nrm is set, the normals of the neighbourhoods (nrm_stride doubles
// per query; eig: optional eigenvalues). Scratch is allocated here and freed
// after the stream has drained: an init-time call.
int run_knn(const float4* q4, int64_t nq, const float4* ref4, int64_t n_ref, int32_t k, int32_t* idx, float* d2,
            double* nrm, int32_t nrm_stride, double* eig, hipStream_t s)
{
    const int64_t qblocks = ceil_div(nq, kKnnThreads);
    // about eight workgroups per compute unit, by splitting the references
    int64_t chunks = std::max<int64_t>(1, ceil_div(8 * (int64_t)g_num_cus, qblocks));
    chunks = std::min<int64_t>(chunks, ceil_div(n_ref, kKnnTile));
    const int64_t chunk = round_up(ceil_div(n_ref, chunks), kKnnTile);
    chunks = ceil_div(n_ref, chunk);
    uint64_t* part = nullptr;
    if (hipMalloc(&part, 8 * (size_t)chunks * (size_t)nq * (size_t)k) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STEIN_ICP_E_NOMEM, "device allocation for the neighbour lists failed");
    }
    KnnArgs a{};
    a.q4 = q4;
    a.ref4 = ref4;
    a.nq = nq;
    a.n_ref = n_ref;
    a.chunk = chunk;
    a.partial = part;
    a.k = k;
    KnnMergeArgs b{};
    b.partial = part;
    b.ref4 = ref4;
    b.nq = nq;
    b.k = k;
    b.chunks = (int32_t)chunks;
    b.idx = idx;
    b.d2 = d2;
    b.nrm = nrm;
    b.eig = eig;
    b.nrm_stride = nrm_stride;
    const dim3 grid((unsigned)qblocks, (unsigned)chunks);
    if (k <= 16) {
        hipLaunchKernelGGL(knn_partial_kernel<16>, grid, dim3(kKnnThreads), 0, s, a);
        hipLaunchKernelGGL(knn_merge_kernel<16>, grid1d(nq, 256), dim3(256), 0, s, b);
    } else {
        hipLaunchKernelGGL(knn_partial_kernel<kKnnMax>, grid, dim3(kKnnThreads), 0, s, a);
        hipLaunchKernelGGL(knn_merge_kernel<kKnnMax>, grid1d(nq, 256), dim3(256), 0, s, b);
    }
    hipError_t e = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    (void)hipFree(part);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("neighbour search: ") + hipGetErrorString(e));
    return STEIN_ICP_OK;
}

void free_ctx(stein_icp_ctx* c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->arena) (void)hipFree(c->arena);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->partial) (void)hipFree(c->partial);
    delete c;
}

int init_impl(stein_icp_ctx** out, const stein_icp_config* cfg, int32_t P, const float* const* src,
              const int64_t* n_src, const float* const* ref, const int64_t* n_ref, const double* init,
              const int32_t* const* sched, hipStream_t s)
{
    if (!out) return fail(STEIN_ICP_E_INVALID, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc) return rc;
    if (P < 1 || P > 65535) return fail(STEIN_ICP_E_INVALID, "n_pairs must be in [1, 65535]");
    if (!src || !n_src || !ref || !n_ref) return fail(STEIN_ICP_E_INVALID, "cloud arrays are NULL");
    const int32_t K = cfg->num_particles, m = cfg->batch_size, rows = cfg->schedule_rows;
    for (int32_t p = 0; p < P; ++p) {
        if (!src[p] || !ref[p]) return fail(STEIN_ICP_E_INVALID, "a cloud pointer is NULL");
        if (n_src[p] < 1 || n_ref[p] < 1) return fail(STEIN_ICP_E_INVALID, "clouds must hold >= 1 point");
        if (n_ref[p] > kMaxRef || n_src[p] > kMaxRef)
            return fail(STEIN_ICP_E_INVALID, "clouds must hold fewer than 2^31 - 64 points");
        if (m > n_src[p]) return fail(STEIN_ICP_E_INVALID, "batch_size exceeds a source cloud size");
        if (sched && !sched[p]) return fail(STEIN_ICP_E_INVALID, "a schedule pointer is NULL");
    }
    const int64_t nq = (int64_t)K * m;
    if (nq > ((int64_t)1 << 31)) return fail(STEIN_ICP_E_INVALID, "K * batch_size too large");

    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    HIP_TRY(hipDeviceGetAttribute(&g_num_cus, hipDeviceAttributeMultiprocessorCount, device));
    auto* c = new stein_icp_ctx();
    c->device = device;
    c->cfg = *cfg;
    c->P = P;
    c->K = K;
    c->m = m;
    c->rows = rows;
    c->nq = nq;

    // layout. Pairs given the same device cloud (pointer and size) share one
    // packed copy of it (and of its normals and BF16 fragments): many
    // independent runs on one pair read one cached reference.
    int64_t so = 0, ro = 0;
    std::map<std::pair<const float*, int64_t>, int32_t> src_owner, ref_owner;
    std::vector<int32_t> own_src(P), own_ref(P);   // pair that packed the cloud
    for (int32_t p = 0; p < P; ++p) {
        PairDesc pd{};
        const auto ks = std::make_pair(src[p], n_src[p]);
        const auto kr = std::make_pair(ref[p], n_ref[p]);
        const auto is = src_owner.find(ks);
        const auto ir = ref_owner.find(kr);
        own_src[p] = is == src_owner.end() ? p : is->second;
        own_ref[p] = ir == ref_owner.end() ? p : ir->second;
        if (own_src[p] == p) src_owner[ks] = p;
        if (own_ref[p] == p) ref_owner[kr] = p;
        pd.src_off = own_src[p] == p ? so : c->pairs[own_src[p]].src_off;
        pd.ref_off = own_ref[p] == p ? ro : c->pairs[own_ref[p]].ref_off;
        pd.n_src = n_src[p];
        pd.n_ref = n_ref[p];
        pd.n_ref_pad = round_up(n_ref[p], kRefPad);
        pd.sched_off = (int64_t)p * rows * m;
        pd.n_scale = cfg->n_scale > 0 ? cfg->n_scale : n_src[p];
        pd.q_off = (int64_t)p * nq;
        pd.nq = nq;
        if (own_src[p] == p) so += pd.n_src;
        if (own_ref[p] == p) ro += pd.n_ref_pad;
        c->pairs.push_back(pd);
    }
    c->tiling = default_tiling(c->pairs, nq);
    if (is_screen(cfg->nn_mode) && c->tiling.q > 2) c->tiling.q = 2;
    {
        // the attribute is a per-kernel ceiling shared by every context: use
        // the largest any particle count needs (the launch sizes the rest)
        size_t most = 0;
        for (int k = 1; k <= kMaxK; ++k) most = std::max(most, grad_bw_lds_bytes(k));
        HIP_TRY(hipFuncSetAttribute((const void*)grad_bandwidth_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)most));
    }
    const bool bf16 = is_screen(cfg->nn_mode);
    int64_t apack_n = 0;
    if (bf16) {
        std::vector<float> h;
        for (int32_t p = 0; p < P; ++p) {
            PairDesc& pd = c->pairs[p];
            if (own_ref[p] != p) {
                const PairDesc& o = c->pairs[own_ref[p]];
                for (int i = 0; i < 4; ++i) pd.c0[i] = o.c0[i];
                pd.sexp = o.sexp;
                pd.apack_off = o.apack_off;
                continue;
            }
            h.resize((size_t)pd.n_ref * 3);
            if (hipMemcpy(h.data(), ref[p], 12 * (size_t)pd.n_ref, hipMemcpyDeviceToHost) != hipSuccess) {
                delete c;
                return fail(STEIN_ICP_E_DEVICE, "reading the reference cloud for its centroid failed");
            }
            bf16_centre(h.data(), pd.n_ref, pd);
            pd.apack_off = apack_n;
            apack_n += 4 * pd.n_ref_pad;
        }
    }
    const int64_t PK6 = (int64_t)P * K * 6;
    const int64_t npairs2 = K >= 2 ? (int64_t)K * (K - 1) : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (size_t)round_up((int64_t)(off + bytes), 256);
        return o;
    };
    const size_t o_pairs = take(sizeof(PairDesc) * P);
    const size_t o_upairs = take(sizeof(PairDesc) * P);   // the pairs that own their reference
    const size_t o_groups = take(sizeof(PairDesc) * P);
    const size_t o_src = take(sizeof(float4) * so);
    const size_t o_ref = take(sizeof(float4) * ro);
    const size_t o_sched = take(sizeof(int32_t) * (size_t)P * rows * m);
    const size_t o_theta = take(8 * PK6), o_thn = take(8 * PK6), o_mom = take(8 * PK6), o_vel = take(8 * PK6);
    const size_t o_gbar = take(8 * PK6), o_phi = take(8 * PK6);
    const size_t o_h = take(8 * 2 * (size_t)P);
    const size_t o_step = take(8 * (size_t)P), o_stepn = take(8 * (size_t)P);
    const size_t o_pose = take(sizeof(Pose) * (size_t)P * K);
    const size_t o_queries = take(sizeof(float4) * (size_t)P * nq);
    const size_t o_apack = take(sizeof(uint4) * (size_t)std::max<int64_t>(apack_n, 1));
    const size_t o_match = take(4 * (size_t)P * nq);
    const bool plane = cfg->metric == STEIN_ICP_METRIC_PLANE;
    const size_t o_nrm = take(plane ? 32 * (size_t)ro : 32);
    const size_t o_dscr = take(8 * (size_t)P * npairs2);
    const size_t o_flag = take(64);
    const size_t o_rescans = take(64);
    if (hipMalloc(&c->arena, off) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(STEIN_ICP_E_NOMEM, "device allocation of " + std::to_string(off) + " bytes failed");
    }
    c->d_pairs = (PairDesc*)(c->arena + o_pairs);
    c->d_groups = (PairDesc*)(c->arena + o_groups);
    c->src4 = (float4*)(c->arena + o_src);
    c->ref4 = (float4*)(c->arena + o_ref);
    c->sched = (int32_t*)(c->arena + o_sched);
    c->theta = (double*)(c->arena + o_theta);
    c->theta_next = (double*)(c->arena + o_thn);
    c->mom = (double*)(c->arena + o_mom);
    c->vel = (double*)(c->arena + o_vel);
    c->gbar = (double*)(c->arena + o_gbar);
    c->phi = (double*)(c->arena + o_phi);
    c->h = (double*)(c->arena + o_h);
    c->step = (int64_t*)(c->arena + o_step);
    c->step_next = (int64_t*)(c->arena + o_stepn);
    c->parity = 0;
    c->pose = (Pose*)(c->arena + o_pose);
    c->queries = (float4*)(c->arena + o_queries);
    c->apack = (uint4*)(c->arena + o_apack);
    c->match = (int32_t*)(c->arena + o_match);
    c->nrm = (double*)(c->arena + o_nrm);
    c->dscr = (double*)(c->arena + o_dscr);
    c->flag = (int*)(c->arena + o_flag);
    c->rescans = (unsigned long long*)(c->arena + o_rescans);

    auto bail = [&](int code) {
        free_ctx(c);
        return code;
    };
    if (hipMemsetAsync(c->arena, 0, off, s) != hipSuccess) return bail(fail(STEIN_ICP_E_DEVICE, "hipMemsetAsync failed"));

    std::vector<int32_t> hsched;
    std::vector<double> hinit;
    for (int32_t p = 0; p < P; ++p) {
        const PairDesc& pd = c->pairs[p];
        if (own_src[p] == p)
            hipLaunchKernelGGL(pack_points_kernel, grid1d(pd.n_src, 256), dim3(256), 0, s, src[p], pd.n_src, pd.n_src,
                               c->src4 + pd.src_off, c->flag);
        if (own_ref[p] == p)
            hipLaunchKernelGGL(pack_points_kernel, grid1d(pd.n_ref_pad, 256), dim3(256), 0, s, ref[p], pd.n_ref,
                               pd.n_ref_pad, c->ref4 + pd.ref_off, c->flag);
        const int64_t ns = (int64_t)rows * m;
        if (sched) {
            hipLaunchKernelGGL(copy_schedule_kernel, grid1d(ns, 256), dim3(256), 0, s, sched[p], ns, pd.n_src,
                               c->sched + pd.sched_off, c->flag);
        } else {
            const size_t o = hsched.size();
            hsched.resize(o + (size_t)ns);
            make_schedule(cfg->seed + (uint64_t)p, pd.n_src, m, rows, hsched.data() + o);
        }
    }
    if (!sched && hipMemcpyAsync(c->sched, hsched.data(), 4 * hsched.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(STEIN_ICP_E_DEVICE, "schedule upload failed"));
    if (init) {
        hipLaunchKernelGGL(copy_finite_kernel, grid1d(PK6, 256), dim3(256), 0, s, init, PK6, c->theta, c->flag);
    } else {
        hinit.resize((size_t)PK6);
        for (int32_t p = 0; p < P; ++p)
            make_init(cfg->seed + (uint64_t)p, K, cfg->init_half_trans, cfg->init_half_rot, cfg->init_centre,
                      hinit.data() + (size_t)p * K * 6);
        if (hipMemcpyAsync(c->theta, hinit.data(), 8 * hinit.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return bail(fail(STEIN_ICP_E_DEVICE, "particle upload failed"));
    }
    std::vector<double> hconst;
    if (const_bandwidth(*cfg)) {
        const bool fixed = cfg->bandwidth_mode == STEIN_ICP_BW_FIXED;
        for (int32_t p = 0; p < P; ++p) {
            hconst.push_back(fixed ? cfg->fixed_h_trans : 1.0);
            hconst.push_back(fixed ? cfg->fixed_h_rot : 1.0);
        }
        if (hipMemcpyAsync(c->h, hconst.data(), 8 * hconst.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return bail(fail(STEIN_ICP_E_DEVICE, "bandwidth upload failed"));
    }
    hipLaunchKernelGGL(pose_kernel, grid1d((int64_t)P * K, 256), dim3(256), 0, s, c->theta, c->pose, (int64_t)P * K);
    if (hipGetLastError() != hipSuccess) return bail(fail(STEIN_ICP_E_DEVICE, "init kernel launch failed"));
    if (hipMemcpyAsync(c->d_pairs, c->pairs.data(), sizeof(PairDesc) * P, hipMemcpyHostToDevice, s) != hipSuccess)
        return bail(fail(STEIN_ICP_E_DEVICE, "pair table upload failed"));
    if (enqueue_queries(c, s) != hipSuccess) return bail(fail(STEIN_ICP_E_DEVICE, "query kernel launch failed"));
    std::vector<PairDesc> uref;   // one descriptor per packed reference
    for (int32_t p = 0; p < P; ++p)
        if (own_ref[p] == p) uref.push_back(c->pairs[p]);
    if (bf16) {
        int64_t maxblk = 0;
        for (const auto& pd : uref) maxblk = std::max<int64_t>(maxblk, pd.n_ref_pad / kRefPad);
        PairDesc* d_upairs = (PairDesc*)(c->arena + o_upairs);
        if (hipMemcpyAsync(d_upairs, uref.data(), sizeof(PairDesc) * uref.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            launch_pack_bf16(d_upairs, (int32_t)uref.size(), maxblk, c->ref4, c->apack, screen_fmt(cfg->nn_mode), s) !=
                hipSuccess)
            return bail(fail(STEIN_ICP_E_DEVICE, "BF16 packing launch failed"));
    }
    int flag = 0;
    if (hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(STEIN_ICP_E_DEVICE, "init synchronisation failed"));
    if (flag & 1) return bail(fail(STEIN_ICP_E_INVALID, "a cloud holds a non-finite coordinate or one above 1e9"));
    if (flag & 2) return bail(fail(STEIN_ICP_E_INVALID, "a schedule index lies outside [0, n_src)"));
    if (flag & 4) return bail(fail(STEIN_ICP_E_INVALID, "an initial particle is non-finite"));
    if (plane) {
        for (const auto& pd : uref) {
            rc = run_knn(c->ref4 + pd.ref_off, pd.n_ref, c->ref4 + pd.ref_off, pd.n_ref, cfg->normal_k, nullptr,
                         nullptr, c->nrm + 4 * pd.ref_off, 4, nullptr, s);
            if (rc) return bail(rc);
        }
    }
    rc = upload_tiling(c, s);
    if (rc) return bail(rc);
    if (cfg->autotune) {
        rc = autotune(c, s);
        if (rc) return bail(rc);
        // the tuner ran real iterations' NN stage only; the state is untouched
    }
    *out = c;
    g_err.clear();
    return STEIN_ICP_OK;
}

}  // namespace

// ====================================================================== ABI

namespace sicp {
// Error reporting shared with the other translation units of the library.
__attribute__((visibility("hidden"))) int report_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace sicp

extern "C" {

void stein_icp_default_config(stein_icp_config* c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->struct_size = sizeof(stein_icp_config);
    c->num_particles = 100;
    c->batch_size = 300;
    c->schedule_rows = 1;
    c->lr = 0.01;
    c->beta1 = 0.9;
    c->beta2 = 0.999;
    c->eps = 1e-8;
    c->init_half_trans = 0.2;
    c->init_half_rot = M_PI / 4;
    c->nn_mode = STEIN_ICP_NN_FP32;
    c->optimizer = STEIN_ICP_OPT_ADAM;
    c->bandwidth_mode = STEIN_ICP_BW_MEDIAN;
    c->prior_mode = STEIN_ICP_PRIOR_UNIFORM;
    c->fixed_h_trans = 1.0;
    c->fixed_h_rot = 1.0;
    for (int i = 0; i < 3; ++i) {
        c->prior_var_trans[i] = 1.0;
        c->prior_kappa_rot[i] = 0.0;
    }
    c->use_graph = 1;
    c->metric = STEIN_ICP_METRIC_POINT;
    c->normal_k = 10;
}

const char* stein_icp_last_error(void) { return g_err.c_str(); }

int stein_icp_init(stein_icp_ctx** out, const stein_icp_config* cfg, const float* src_xyz, int64_t n_src,
                   const float* ref_xyz, int64_t n_ref, const double* init_particles, const int32_t* schedule,
                   void* hip_stream)
{
    const float* s[1] = {src_xyz};
    const float* r[1] = {ref_xyz};
    const int32_t* sc[1] = {schedule};
    return init_impl(out, cfg, 1, s, &n_src, r, &n_ref, init_particles, schedule ? sc : nullptr,
                     (hipStream_t)hip_stream);
}

int stein_icp_batch_init(stein_icp_ctx** out, const stein_icp_config* cfg, int32_t n_pairs,
                         const float* const* src_xyz, const int64_t* n_src, const float* const* ref_xyz,
                         const int64_t* n_ref, const double* init_particles, const int32_t* const* schedules,
                         void* hip_stream)
{
    return init_impl(out, cfg, n_pairs, src_xyz, n_src, ref_xyz, n_ref, init_particles, schedules,
                     (hipStream_t)hip_stream);
}

int stein_icp_step(stein_icp_ctx* ctx, int32_t n_iters, void* hip_stream)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    if (n_iters < 0) return fail(STEIN_ICP_E_INVALID, "n_iters must be >= 0");
    return run_iters(ctx, n_iters, (hipStream_t)hip_stream);
}

int stein_icp_particles(const stein_icp_ctx* ctx, double* out, void* hip_stream)
{
    if (!ctx || !out) return fail(STEIN_ICP_E_INVALID, "ctx or out is NULL");
    HIP_TRY(hipMemcpyAsync(out, ctx->theta, 8 * (size_t)ctx->P * ctx->K * 6, hipMemcpyDeviceToDevice,
                           (hipStream_t)hip_stream));
    return STEIN_ICP_OK;
}

int stein_icp_get_state(const stein_icp_ctx* ctx, double* theta, double* mom, double* vel, int64_t* t,
                        void* hip_stream)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t bytes = 8 * (size_t)ctx->P * ctx->K * 6;
    if (theta) HIP_TRY(hipMemcpyAsync(theta, ctx->theta, bytes, hipMemcpyDeviceToDevice, s));
    if (mom) HIP_TRY(hipMemcpyAsync(mom, ctx->mom, bytes, hipMemcpyDeviceToDevice, s));
    if (vel) HIP_TRY(hipMemcpyAsync(vel, ctx->vel, bytes, hipMemcpyDeviceToDevice, s));
    int64_t tt = 0;
    HIP_TRY(hipMemcpyAsync(&tt, ctx->step, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (t) *t = tt;
    return STEIN_ICP_OK;
}

int stein_icp_set_state(stein_icp_ctx* ctx, const double* theta, const double* mom, const double* vel, int64_t t,
                        void* hip_stream)
{
    if (!ctx || !theta) return fail(STEIN_ICP_E_INVALID, "ctx or theta is NULL");
    if (t < 0) return fail(STEIN_ICP_E_INVALID, "t must be >= 0");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = (int64_t)ctx->P * ctx->K * 6;
    // every input is checked before anything of the context changes
    {
        int bad = 0;
        hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, ctx->flag, (int64_t)1, 0);
        hipLaunchKernelGGL(check_finite_kernel, grid1d(n, 256), dim3(256), 0, s, theta, n, ctx->flag);
        if (mom) hipLaunchKernelGGL(check_finite_kernel, grid1d(n, 256), dim3(256), 0, s, mom, n, ctx->flag);
        if (vel) hipLaunchKernelGGL(check_finite_kernel, grid1d(n, 256), dim3(256), 0, s, vel, n, ctx->flag);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return fail(STEIN_ICP_E_INVALID, "a particle or moment is non-finite");
    }
    HIP_TRY(hipMemcpyAsync(ctx->theta, theta, 8 * n, hipMemcpyDeviceToDevice, s));
    if (mom) HIP_TRY(hipMemcpyAsync(ctx->mom, mom, 8 * n, hipMemcpyDeviceToDevice, s));
    else hipLaunchKernelGGL(fill_f64_kernel, grid1d(n, 256), dim3(256), 0, s, ctx->mom, n, 0.0);
    if (vel) HIP_TRY(hipMemcpyAsync(ctx->vel, vel, 8 * n, hipMemcpyDeviceToDevice, s));
    else hipLaunchKernelGGL(fill_f64_kernel, grid1d(n, 256), dim3(256), 0, s, ctx->vel, n, 0.0);
    hipLaunchKernelGGL(fill_i64_kernel, grid1d(ctx->P, 256), dim3(256), 0, s, ctx->step, (int64_t)ctx->P, t);
    hipLaunchKernelGGL(pose_kernel, grid1d((int64_t)ctx->P * ctx->K, 256), dim3(256), 0, s, ctx->theta, ctx->pose,
                       (int64_t)ctx->P * ctx->K);
    HIP_TRY(hipGetLastError());
    HIP_TRY(enqueue_queries(ctx, s));
    return STEIN_ICP_OK;
}

int stein_icp_particles_f32(const stein_icp_ctx* ctx, float* out, void* hip_stream)
{
    if (!ctx || !out) return fail(STEIN_ICP_E_INVALID, "ctx or out is NULL");
    const int64_t n = (int64_t)ctx->P * ctx->K * 6;
    hipLaunchKernelGGL(narrow_f64_kernel, grid1d(n, 256), dim3(256), 0, (hipStream_t)hip_stream, ctx->theta, n, out);
    HIP_TRY(hipGetLastError());
    return STEIN_ICP_OK;
}

int stein_icp_set_particles_f32(stein_icp_ctx* ctx, const float* theta, void* hip_stream)
{
    if (!ctx || !theta) return fail(STEIN_ICP_E_INVALID, "ctx or theta is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = (int64_t)ctx->P * ctx->K * 6;
    int bad = 0;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, ctx->flag, (int64_t)1, 0);
    hipLaunchKernelGGL(check_finite_f32_kernel, grid1d(n, 256), dim3(256), 0, s, theta, n, ctx->flag);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&bad, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return fail(STEIN_ICP_E_INVALID, "a particle is non-finite");
    hipLaunchKernelGGL(widen_f32_kernel, grid1d(n, 256), dim3(256), 0, s, theta, n, ctx->theta);
    hipLaunchKernelGGL(fill_f64_kernel, grid1d(n, 256), dim3(256), 0, s, ctx->mom, n, 0.0);
    hipLaunchKernelGGL(fill_f64_kernel, grid1d(n, 256), dim3(256), 0, s, ctx->vel, n, 0.0);
    hipLaunchKernelGGL(fill_i64_kernel, grid1d(ctx->P, 256), dim3(256), 0, s, ctx->step, (int64_t)ctx->P, (int64_t)0);
    hipLaunchKernelGGL(pose_kernel, grid1d((int64_t)ctx->P * ctx->K, 256), dim3(256), 0, s, ctx->theta, ctx->pose,
                       (int64_t)ctx->P * ctx->K);
    HIP_TRY(hipGetLastError());
    HIP_TRY(enqueue_queries(ctx, s));
    return STEIN_ICP_OK;
}

int stein_icp_get_diagnostics(const stein_icp_ctx* ctx, double* gbar, double* phi, double* h, int32_t* match,
                              void* hip_stream)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t b6 = 8 * (size_t)ctx->P * ctx->K * 6;
    if (gbar) HIP_TRY(hipMemcpyAsync(gbar, ctx->gbar, b6, hipMemcpyDeviceToDevice, s));
    if (phi) HIP_TRY(hipMemcpyAsync(phi, ctx->phi, b6, hipMemcpyDeviceToDevice, s));
    if (h) HIP_TRY(hipMemcpyAsync(h, ctx->h, 16 * (size_t)ctx->P, hipMemcpyDeviceToDevice, s));
    if (match) HIP_TRY(hipMemcpyAsync(match, ctx->match, 4 * (size_t)ctx->P * ctx->nq, hipMemcpyDeviceToDevice, s));
    return STEIN_ICP_OK;
}

int stein_icp_shape(const stein_icp_ctx* ctx, int32_t* n_pairs, int32_t* K, int32_t* m)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    if (n_pairs) *n_pairs = ctx->P;
    if (K) *K = ctx->K;
    if (m) *m = ctx->m;
    return STEIN_ICP_OK;
}

int stein_icp_nn_tiling(const stein_icp_ctx* ctx, int32_t* qpl, int32_t* waves, int32_t* chunk, int32_t* chunks,
                        int32_t* persist, double* tuned_ms)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    if (qpl) *qpl = ctx->tiling.q;
    if (persist) *persist = ctx->tiling.persist;
    if (waves) *waves = ctx->tiling.w;
    if (chunk) *chunk = ctx->pairs[0].chunk;
    if (chunks) *chunks = ctx->pairs[0].chunks;
    if (tuned_ms) *tuned_ms = ctx->tuned_ms;
    return STEIN_ICP_OK;
}

int stein_icp_set_nn_tiling(stein_icp_ctx* ctx, int32_t qpl, int32_t waves, int32_t chunk, int32_t persist,
                            void* hip_stream)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    if (persist < 0 || persist > 64) return fail(STEIN_ICP_E_INVALID, "persist must be in [0, 64]");
    if (qpl != 1 && qpl != 2 && qpl != 4) return fail(STEIN_ICP_E_INVALID, "queries_per_lane must be 1, 2 or 4");
    if (waves != 4 && waves != 8 && waves != 16) return fail(STEIN_ICP_E_INVALID, "waves must be 4, 8 or 16");
    if (chunk < kRefPad || chunk % kRefPad != 0)
        return fail(STEIN_ICP_E_INVALID, "chunk must be a positive multiple of 32");
    if (is_screen(ctx->cfg.nn_mode) && !nn_bf16_shape_ok(qpl, waves))
        return fail(STEIN_ICP_E_INVALID, "the matrix-core screens take 1 or 2 queries per lane, and 4 or 8 waves with 2");
    Tiling t;
    t.q = qpl;
    t.w = waves;
    t.persist = persist;
    for (const auto& pd : ctx->pairs) t.chunk.push_back((int32_t)std::min<int64_t>(chunk, pd.n_ref_pad));
    const Tiling old = ctx->tiling;
    ctx->tiling = t;
    const int rc = upload_tiling(ctx, (hipStream_t)hip_stream);
    if (rc) ctx->tiling = old;
    return rc;
}

int stein_icp_stage_times(stein_icp_ctx* ctx, int32_t n_iters, double* ms_out, void* hip_stream)
{
    if (!ctx || !ms_out) return fail(STEIN_ICP_E_INVALID, "ctx or ms_out is NULL");
    if (n_iters < 1) return fail(STEIN_ICP_E_INVALID, "n_iters must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &st));
    if (st != hipStreamCaptureStatusNone) return fail(STEIN_ICP_E_STATE, "stream is capturing");
    std::vector<hipEvent_t> ev((size_t)n_iters * (kStages + 1), nullptr);
    int rc = STEIN_ICP_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(STEIN_ICP_E_DEVICE, "hipEventCreate failed");
    const size_t W = kStages + 1;
    for (int32_t i = 0; i < n_iters && rc == STEIN_ICP_OK; ++i) {
        hipEvent_t* e = ev.data() + W * (size_t)i;
        hipError_t err = hipEventRecord(e[0], s);
        for (int st = 0; st < kStages && err == hipSuccess; ++st) {
            err = enqueue_stage(ctx, st, s);
            if (err == hipSuccess) err = hipEventRecord(e[st + 1], s);
        }
        if (err != hipSuccess) rc = fail(STEIN_ICP_E_DEVICE, std::string("profiled step: ") + hipGetErrorString(err));
        else {
            advance(ctx, 1);
            ctx->certificates += certificates_per_launch(ctx);
        }
    }
    if (rc == STEIN_ICP_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(STEIN_ICP_E_DEVICE, "sync failed");
    double t[kStages] = {0, 0, 0};
    for (int32_t i = 0; i < n_iters && rc == STEIN_ICP_OK; ++i)
        for (int k = 0; k < kStages; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[W * (size_t)i + k], ev[W * (size_t)i + k + 1]) != hipSuccess)
                rc = fail(STEIN_ICP_E_DEVICE, "hipEventElapsedTime failed");
            t[k] += ms;
        }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc == STEIN_ICP_OK)
        for (int k = 0; k < kStages; ++k) ms_out[k] = t[k];
    return rc;
}

int stein_icp_time_nn(stein_icp_ctx* ctx, int32_t n_launches, double* ms_per_launch, void* hip_stream)
{
    if (!ctx || !ms_per_launch) return fail(STEIN_ICP_E_INVALID, "ctx or ms_per_launch is NULL");
    if (n_launches < 1) return fail(STEIN_ICP_E_INVALID, "n_launches must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t e = enqueue_stage(ctx, 0, s);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int32_t i = 0; i < n_launches && e == hipSuccess; ++i) e = enqueue_stage(ctx, 0, s);
    ctx->certificates += (int64_t)(n_launches + 1) * certificates_per_launch(ctx);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("stein_icp_time_nn: ") + hipGetErrorString(e));
    *ms_per_launch = (double)ms / n_launches;
    return STEIN_ICP_OK;
}

int stein_icp_nn_rescans(const stein_icp_ctx* ctx, int64_t* rescans, int64_t* certificates, void* hip_stream)
{
    if (!ctx) return fail(STEIN_ICP_E_INVALID, "ctx is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    unsigned long long n = 0;
    HIP_TRY(hipMemcpyAsync(&n, ctx->rescans, sizeof(n), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (rescans) *rescans = (int64_t)n;
    if (certificates) *certificates = ctx->certificates;
    return STEIN_ICP_OK;
}

void stein_icp_destroy(stein_icp_ctx* ctx) { free_ctx(ctx); }

int stein_icp_nn(const float* q_xyz, int64_t nq, const float* ref_xyz, int64_t n_ref, int32_t mode, int32_t* idx,
                 float* d2, void* hip_stream)
{
    if (nq < 0 || n_ref < 1) return fail(STEIN_ICP_E_INVALID, "need nq >= 0 and n_ref >= 1");
    if (nq > kMaxRef || n_ref > kMaxRef) return fail(STEIN_ICP_E_INVALID, "sizes must be below 2^31 - 64");
    if (mode != STEIN_ICP_NN_FP32 && !is_screen(mode)) return fail(STEIN_ICP_E_INVALID, "unknown nn mode");
    if (nq == 0) return STEIN_ICP_OK;
    if (!q_xyz || !ref_xyz || !idx) return fail(STEIN_ICP_E_INVALID, "a pointer is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    PairDesc pd{};
    pd.q_off = 0;
    pd.nq = nq;
    pd.part_stride = nq;
    pd.n_ref = n_ref;
    pd.n_ref_pad = round_up(n_ref, kRefPad);
    const bool bf16 = is_screen(mode);
    if (bf16) {
        std::vector<float> h((size_t)n_ref * 3);
        if (hipMemcpy(h.data(), ref_xyz, 12 * (size_t)n_ref, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(STEIN_ICP_E_DEVICE, "reading the reference cloud for its centroid failed");
        bf16_centre(h.data(), n_ref, pd);
        pd.apack_off = 0;
    }
    std::vector<PairDesc> v{pd};
    Tiling t = default_tiling(v, nq);
    if (bf16 && t.q > 2) t.q = 2;
    pd.chunk = t.chunk[0];
    pd.chunks = (int32_t)ceil_div(pd.n_ref_pad, pd.chunk);
    pd.qblocks = (int32_t)ceil_div(nq, (int64_t)kWave * t.q);
    std::vector<WorkItem> work;
    for (int32_t b = 0; b < pd.qblocks; ++b)
        for (int32_t ch = 0; ch < pd.chunks; ++ch) work.push_back(WorkItem{0, b, ch, 0});
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (size_t)round_up((int64_t)(off + bytes), 256);
        return o;
    };
    const size_t o_q = take(16 * (size_t)nq), o_r = take(16 * (size_t)pd.n_ref_pad);
    const size_t o_p = take(8 * (size_t)pd.chunks * nq), o_w = take(sizeof(WorkItem) * work.size());
    const size_t o_d = take(sizeof(PairDesc)), o_f = take(64);
    const size_t o_ap = take(bf16 ? sizeof(uint4) * (size_t)(4 * pd.n_ref_pad) : 16);
    char* mem = nullptr;
    if (hipMalloc(&mem, off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STEIN_ICP_E_NOMEM, "device allocation failed");
    }
    int rc = STEIN_ICP_OK;
    int flag = 0;
    NNArgs a{};
    a.work = (WorkItem*)(mem + o_w);
    a.pairs = (PairDesc*)(mem + o_d);
    a.ref4 = (float4*)(mem + o_r);
    a.queries = (float4*)(mem + o_q);
    a.partial = (uint64_t*)(mem + o_p);
    int* fl = (int*)(mem + o_f);
    hipError_t e = hipMemsetAsync(fl, 0, 64, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void*)a.pairs, &pd, sizeof(pd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void*)a.work, work.data(), sizeof(WorkItem) * work.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pack_points_kernel, grid1d(nq, 256), dim3(256), 0, s, q_xyz, nq, nq, (float4*)a.queries, fl);
        hipLaunchKernelGGL(pack_points_kernel, grid1d(pd.n_ref_pad, 256), dim3(256), 0, s, ref_xyz, n_ref,
                           pd.n_ref_pad, (float4*)a.ref4, fl);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, fl, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && flag) rc = fail(STEIN_ICP_E_INVALID, "a coordinate is non-finite or above 1e9");
    if (e == hipSuccess && !rc) {
        if (bf16) {
            e = launch_pack_bf16(a.pairs, 1, pd.n_ref_pad / kRefPad, a.ref4, (uint4*)(mem + o_ap), screen_fmt(mode), s);
            NNBf16Args b{};
            b.work = a.work;
            b.pairs = a.pairs;
            b.ref4 = a.ref4;
            b.apack = (const uint4*)(mem + o_ap);
            b.queries = a.queries;
            b.partial = a.partial;
            if (e == hipSuccess) e = launch_nn_bf16(t, (unsigned)work.size(), b, screen_fmt(mode), s);
        } else {
            e = launch_nn(t, (unsigned)work.size(), a, s);
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(nn_finish_kernel, grid1d(nq, 256), dim3(256), 0, s, a.partial, a.queries, a.ref4,
                               pd.n_ref_pad, nq, pd.chunks, bf16 ? 1 : 0, idx, d2);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) rc = fail(STEIN_ICP_E_DEVICE, std::string("stein_icp_nn: ") + hipGetErrorString(e));
    (void)hipFree(mem);
    return rc;
}

int stein_icp_screen_values(const float* q_xyz, int64_t nq, const float* ref_xyz, int64_t n_ref, int32_t mode,
                            float* values, float* centre, int32_t* scale_exp, void* hip_stream)
{
    if (!is_screen(mode)) return fail(STEIN_ICP_E_INVALID, "mode must be one of the matrix-core screens");
    if (nq < 0 || n_ref < 1 || n_ref > kMaxRef) return fail(STEIN_ICP_E_INVALID, "need nq >= 0 and 1 <= n_ref < 2^31 - 64");
    if (nq > ((int64_t)1 << 31) / n_ref) return fail(STEIN_ICP_E_INVALID, "nq * n_ref must be at most 2^31");
    if (!ref_xyz || (nq > 0 && (!q_xyz || !values))) return fail(STEIN_ICP_E_INVALID, "a pointer is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    PairDesc pd{};
    pd.n_ref = n_ref;
    pd.n_ref_pad = round_up(n_ref, kRefPad);
    std::vector<float> h((size_t)n_ref * 3);
    if (hipMemcpy(h.data(), ref_xyz, 12 * (size_t)n_ref, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(STEIN_ICP_E_DEVICE, "reading the reference cloud for its centroid failed");
    bf16_centre(h.data(), n_ref, pd);
    if (centre)
        for (int i = 0; i < 4; ++i) centre[i] = pd.c0[i];
    if (scale_exp) *scale_exp = pd.sexp;
    if (nq == 0) return STEIN_ICP_OK;
    const int64_t nq_pad = round_up(nq, 32);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (size_t)round_up((int64_t)(off + bytes), 256);
        return o;
    };
    const size_t o_q = take(16 * (size_t)nq_pad), o_r = take(16 * (size_t)pd.n_ref_pad);
    const size_t o_ap = take(64 * (size_t)pd.n_ref_pad), o_d = take(sizeof(PairDesc)), o_f = take(64);
    char* mem = nullptr;
    if (hipMalloc(&mem, off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STEIN_ICP_E_NOMEM, "device allocation failed");
    }
    int flag = 0, rc = STEIN_ICP_OK;
    float4* q4 = (float4*)(mem + o_q);
    float4* r4 = (float4*)(mem + o_r);
    PairDesc* d_pd = (PairDesc*)(mem + o_d);
    int* fl = (int*)(mem + o_f);
    hipError_t e = hipMemsetAsync(fl, 0, 64, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pd, &pd, sizeof(pd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pack_points_kernel, grid1d(nq_pad, 256), dim3(256), 0, s, q_xyz, nq, nq_pad, q4, fl);
        hipLaunchKernelGGL(pack_points_kernel, grid1d(pd.n_ref_pad, 256), dim3(256), 0, s, ref_xyz, n_ref,
                           pd.n_ref_pad, r4, fl);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, fl, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && flag) rc = fail(STEIN_ICP_E_INVALID, "a coordinate is non-finite or above 1e9");
    if (e == hipSuccess && !rc) {
        e = launch_pack_bf16(d_pd, 1, pd.n_ref_pad / kRefPad, r4, (uint4*)(mem + o_ap), screen_fmt(mode), s);
        if (e == hipSuccess)
            e = launch_screen_values(d_pd, pd.n_ref_pad, (const uint4*)(mem + o_ap), q4, nq, screen_fmt(mode), values, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) rc = fail(STEIN_ICP_E_DEVICE, std::string("stein_icp_screen_values: ") + hipGetErrorString(e));
    (void)hipFree(mem);
    return rc;
}

namespace {

// Scratch of stein_icp_nn_noalloc: device memory of this library's code
// object, one copy on every GPU the library runs on, held until the process
// ends. Host code addresses it only through the pointer hipGetSymbolAddress
// returns for the current device (the array's name is not a device address
// on the host).
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// The scratch array's device address on the current device, looked up once
// per device.
int scratch_on_device(char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(STEIN_ICP_E_DEVICE, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(STEIN_ICP_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (char*)p;
    }
    *out = g_scratch[dev];
    return STEIN_ICP_OK;
}

// Pair descriptor, cleared flag and work table (query block, chunk) of a
// standalone search, written on the device.
__global__ void nn_setup_kernel(PairDesc pd, PairDesc* __restrict__ pd_out, WorkItem* __restrict__ work,
                                int64_t nwork, int32_t chunks, int* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        *pd_out = pd;
        *flag = 0;
    }
    if (i < nwork) work[i] = WorkItem{0, (int32_t)(i / chunks), (int32_t)(i % chunks), 0};
}

}  // namespace

int stein_icp_nn_noalloc(const float* q_xyz, int64_t nq, const float* ref_xyz, int64_t n_ref, int32_t mode,
                         int32_t* idx, float* d2, void* hip_stream)
{
    if (nq < 0 || n_ref < 1) return fail(STEIN_ICP_E_INVALID, "need nq >= 0 and n_ref >= 1");
    if (nq > kMaxRef || n_ref > kMaxRef) return fail(STEIN_ICP_E_INVALID, "sizes must be below 2^31 - 64");
    if (mode != STEIN_ICP_NN_FP32 && !is_screen(mode)) return fail(STEIN_ICP_E_INVALID, "unknown nn mode");
    if (nq == 0) return STEIN_ICP_OK;
    if (!q_xyz || !ref_xyz || !idx) return fail(STEIN_ICP_E_INVALID, "a pointer is NULL");
    const bool bf16 = is_screen(mode);
    PairDesc pd{};
    pd.nq = nq;
    pd.part_stride = nq;
    pd.n_ref = n_ref;
    pd.n_ref_pad = round_up(n_ref, kRefPad);
    Tiling t;   // the standalone search's shape (stein_icp_nn), fewer chunks if the keys need it
    t.q = default_queries_per_lane(nq);
    int64_t chunk = default_chunk(pd.n_ref_pad, nq, t.q, 1);
    if (bf16 && t.q > 2) t.q = 2;
    t.w = 4;
    // scratch layout: flag, descriptor, work table, queries, references,
    // BF16 fragments, chunk keys (256-byte aligned blocks)
    const int64_t qblocks = ceil_div(nq, (int64_t)kWave * t.q);
    const auto a256 = [](int64_t b) { return round_up(b, 256); };
    const int64_t fixed = 256 + a256(sizeof(PairDesc)) + a256(16 * nq) + a256(16 * pd.n_ref_pad) +
                          (bf16 ? a256(64 * pd.n_ref_pad) : 0);
    int64_t chunks = ceil_div(pd.n_ref_pad, chunk);
    const auto total = [&](int64_t ch) {
        return fixed + a256((int64_t)sizeof(WorkItem) * qblocks * ch) + a256(8 * ch * nq);
    };
    while (chunks > 1 && total(chunks) > (int64_t)kNoAllocScratchBytes) --chunks;
    if (total(chunks) > (int64_t)kNoAllocScratchBytes)
        return fail(STEIN_ICP_E_INVALID, "stein_icp_nn_noalloc: the search needs " + std::to_string(total(chunks)) +
                                             " bytes of scratch, above its 32 MiB");
    chunk = round_up(ceil_div(pd.n_ref_pad, chunks), 4 * kTile);
    chunks = ceil_div(pd.n_ref_pad, chunk);
    pd.chunk = (int32_t)chunk;
    pd.chunks = (int32_t)chunks;
    pd.qblocks = (int32_t)qblocks;
    const int64_t nwork = qblocks * chunks;
    char* base = nullptr;
    int rc = scratch_on_device(&base);
    if (rc) return rc;
    int64_t off = 0;
    const auto take = [&](int64_t bytes) {
        char* p = base + off;
        off += a256(bytes);
        return p;
    };
    int* fl = (int*)take(256);
    PairDesc* d_pd = (PairDesc*)take(sizeof(PairDesc));
    WorkItem* work = (WorkItem*)take((int64_t)sizeof(WorkItem) * nwork);
    float4* q4 = (float4*)take(16 * nq);
    float4* r4 = (float4*)take(16 * pd.n_ref_pad);
    uint4* ap = bf16 ? (uint4*)take(64 * pd.n_ref_pad) : nullptr;
    uint64_t* keys = (uint64_t*)take(8 * chunks * nq);
    hipStream_t s = (hipStream_t)hip_stream;
    int flag = 0;
    hipLaunchKernelGGL(nn_setup_kernel, grid1d(nwork, 256), dim3(256), 0, s, pd, d_pd, work, nwork, (int32_t)chunks,
                       fl);
    hipLaunchKernelGGL(pack_points_kernel, grid1d(nq, 256), dim3(256), 0, s, q_xyz, nq, nq, q4, fl);
    hipLaunchKernelGGL(pack_points_kernel, grid1d(pd.n_ref_pad, 256), dim3(256), 0, s, ref_xyz, n_ref, pd.n_ref_pad,
                       r4, fl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, fl, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("stein_icp_nn_noalloc: ") + hipGetErrorString(e));
    if (flag) return fail(STEIN_ICP_E_INVALID, "a coordinate is non-finite or above 1e9");
    if (bf16) {
        e = launch_bf16_centre(d_pd, r4, n_ref, s);
        if (e == hipSuccess) e = launch_pack_bf16(d_pd, 1, pd.n_ref_pad / kRefPad, r4, ap, screen_fmt(mode), s);
        NNBf16Args b{};
        b.work = work;
        b.pairs = d_pd;
        b.ref4 = r4;
        b.apack = ap;
        b.queries = q4;
        b.partial = keys;
        if (e == hipSuccess) e = launch_nn_bf16(t, (unsigned)nwork, b, screen_fmt(mode), s);
    } else {
        NNArgs a{};
        a.work = work;
        a.pairs = d_pd;
        a.ref4 = r4;
        a.queries = q4;
        a.partial = keys;
        e = launch_nn(t, (unsigned)nwork, a, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(nn_finish_kernel, grid1d(nq, 256), dim3(256), 0, s, keys, q4, r4, pd.n_ref_pad, nq,
                           (int32_t)chunks, bf16 ? 1 : 0, idx, d2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("stein_icp_nn_noalloc: ") + hipGetErrorString(e));
    return STEIN_ICP_OK;
}

namespace {

// Pack device xyz clouds into float4 scratch, check them, and run the
// neighbour search (and normals) over them. q_xyz == NULL: the queries are
// the references themselves.
int knn_entry(const char* fn, const float* q_xyz, int64_t nq, const float* ref_xyz, int64_t n_ref, int32_t k,
              int32_t* idx, float* d2, double* nrm, double* eig, hipStream_t s)
{
    const int64_t nq_pad = round_up(std::max<int64_t>(nq, 1), 64), nr_pad = round_up(n_ref, 64);
    char* mem = nullptr;
    const size_t o_r = 16 * (size_t)nq_pad, bytes = o_r + 16 * (size_t)nr_pad + 256;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STEIN_ICP_E_NOMEM, std::string(fn) + ": device allocation failed");
    }
    float4* q4 = (float4*)mem;
    float4* r4 = (float4*)(mem + o_r);
    int* fl = (int*)(mem + o_r + 16 * (size_t)nr_pad);
    int flag = 0, rc = STEIN_ICP_OK;
    hipError_t e = hipMemsetAsync(fl, 0, sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pack_points_kernel, grid1d(n_ref, 256), dim3(256), 0, s, ref_xyz, n_ref, n_ref, r4, fl);
        if (q_xyz)
            hipLaunchKernelGGL(pack_points_kernel, grid1d(nq, 256), dim3(256), 0, s, q_xyz, nq, nq, q4, fl);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, fl, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        rc = fail(STEIN_ICP_E_DEVICE, std::string(fn) + ": " + hipGetErrorString(e));
    else if (flag)
        rc = fail(STEIN_ICP_E_INVALID, std::string(fn) + ": a coordinate is non-finite or above 1e9");
    else
        rc = run_knn(q_xyz ? q4 : r4, nq, r4, n_ref, k, idx, d2, nrm, 3, eig, s);
    (void)hipFree(mem);
    return rc;
}

}  // namespace

int stein_icp_knn(const float* q_xyz, int64_t nq, const float* ref_xyz, int64_t n_ref, int32_t k, int32_t* idx,
                  float* d2, void* hip_stream)
{
    if (nq < 0 || n_ref < 1) return fail(STEIN_ICP_E_INVALID, "need nq >= 0 and n_ref >= 1");
    if (nq > kMaxRef || n_ref > kMaxRef) return fail(STEIN_ICP_E_INVALID, "sizes must be below 2^31 - 64");
    if (k < 1 || k > kKnnMax) return fail(STEIN_ICP_E_INVALID, "k must be in [1, 32]");
    if (nq == 0) return STEIN_ICP_OK;
    if (!q_xyz || !ref_xyz || !idx || !d2) return fail(STEIN_ICP_E_INVALID, "a pointer is NULL");
    return knn_entry("stein_icp_knn", q_xyz, nq, ref_xyz, n_ref, k, idx, d2, nullptr, nullptr,
                     (hipStream_t)hip_stream);
}

int stein_icp_normals(const float* ref_xyz, int64_t n_ref, int32_t k, double* normals, double* eig, void* hip_stream)
{
    if (n_ref < 1 || n_ref > kMaxRef) return fail(STEIN_ICP_E_INVALID, "n_ref must be in [1, 2^31 - 64)");
    if (k < 3 || k > kKnnMax) return fail(STEIN_ICP_E_INVALID, "k must be in [3, 32]");
    if (!ref_xyz || !normals) return fail(STEIN_ICP_E_INVALID, "a pointer is NULL");
    return knn_entry("stein_icp_normals", nullptr, n_ref, ref_xyz, n_ref, k,
                     nullptr, nullptr, normals, eig, (hipStream_t)hip_stream);
}

int stein_icp_get_normals(const stein_icp_ctx* ctx, double* out, void* hip_stream)
{
    if (!ctx || !out) return fail(STEIN_ICP_E_INVALID, "ctx or out is NULL");
    if (ctx->cfg.metric != STEIN_ICP_METRIC_PLANE)
        return fail(STEIN_ICP_E_STATE, "the context uses the point-to-point metric: it holds no normals");
    hipStream_t s = (hipStream_t)hip_stream;
    int64_t o = 0;
    for (const auto& pd : ctx->pairs) {
        if (hipMemcpy2DAsync(out + 3 * o, 3 * sizeof(double), ctx->nrm + 4 * pd.ref_off, 4 * sizeof(double),
                             3 * sizeof(double), (size_t)pd.n_ref, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(STEIN_ICP_E_DEVICE, "copying the normals failed");
        o += pd.n_ref;
    }
    return STEIN_ICP_OK;
}

namespace {

double wrap_pi(double a) { return std::atan2(std::sin(a), std::cos(a)); }

// Mean and covariance (n - 1 denominator) of columns d0 .. d0 + 2 of the
// n x 6 rows x; with `centre`, each value v is first taken as
// centre + wrap(v - centre) (angles).
void fit3(const double* x, int64_t n, int d0, const double* centre, double mu[3], double S[9])
{
    auto val = [&](int64_t i, int d) {
        const double v = x[6 * i + d0 + d];
        return centre ? centre[d] + wrap_pi(v - centre[d]) : v;
    };
    for (int d = 0; d < 3; ++d) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += val(i, d);
        mu[d] = acc / (double)n;
    }
    for (int e = 0; e < 9; ++e) S[e] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v[3];
        for (int d = 0; d < 3; ++d) v[d] = val(i, d) - mu[d];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) S[3 * r + c] += v[r] * v[c];
    }
    for (int e = 0; e < 9; ++e) S[e] /= (double)(n - 1);
}

// Lower Cholesky factor of a symmetric 3x3 matrix; false unless positive definite.
bool chol3(const double S[9], double L[9])
{
    for (int e = 0; e < 9; ++e) L[e] = 0.0;
    for (int j = 0; j < 3; ++j) {
        double d = S[4 * j];
        for (int k = 0; k < j; ++k) d -= L[3 * j + k] * L[3 * j + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        L[4 * j] = std::sqrt(d);
        for (int i = j + 1; i < 3; ++i) {
            double v = S[3 * i + j];
            for (int k = 0; k < j; ++k) v -= L[3 * i + k] * L[3 * j + k];
            L[3 * i + j] = v / L[4 * j];
        }
    }
    return true;
}

// Solve L y = b in place (forward substitution).
void lsolve3(const double L[9], double b[3])
{
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < i; ++k) b[i] -= L[3 * i + k] * b[k];
        b[i] /= L[4 * i];
    }
}

// KL(N(ma, Sa) || N(mb, Sb)) = (tr(Sb^-1 Sa) + |Lb^-1 (mb - ma)|^2 - 3 + ln det Sb - ln det Sa) / 2,
// with tr(Sb^-1 Sa) = |Lb^-1 La|_F^2 for Cholesky factors La, Lb.
bool kl_gauss3(const double ma[3], const double Sa[9], const double mb[3], const double Sb[9], double* out)
{
    double La[9], Lb[9];
    if (!chol3(Sa, La) || !chol3(Sb, Lb)) return false;
    double tr = 0.0;
    for (int c = 0; c < 3; ++c) {
        double col[3] = {La[c], La[3 + c], La[6 + c]};
        lsolve3(Lb, col);
        tr += (col[0] * col[0] + col[1] * col[1]) + col[2] * col[2];
    }
    double z[3] = {mb[0] - ma[0], mb[1] - ma[1], mb[2] - ma[2]};
    lsolve3(Lb, z);
    const double maha = (z[0] * z[0] + z[1] * z[1]) + z[2] * z[2];
    double ld = 0.0;
    for (int j = 0; j < 3; ++j) ld += 2.0 * (std::log(Lb[4 * j]) - std::log(La[4 * j]));
    *out = 0.5 * (tr + maha - 3.0 + ld);
    return true;
}

// Overlapping coefficient, the integral of min(f1, f2), of two normal
// densities: with s1 < s2 the narrower density is the smaller one outside
// the two crossing points x1 < x2 (roots of ln f1 = ln f2) and the larger
// one between them; equal widths cross once, at the midpoint.
double ovl_normal(double m1, double s1, double m2, double s2)
{
    const double r2 = 1.4142135623730951;   // sqrt(2)
    if (s1 > s2) {
        std::swap(m1, m2);
        std::swap(s1, s2);
    }
    const double a = 1.0 / (s1 * s1) - 1.0 / (s2 * s2);
    if (!(a > 0.0)) return std::erfc(std::fabs(m1 - m2) / (2.0 * r2 * s1));
    const double b = -2.0 * (m1 / (s1 * s1) - m2 / (s2 * s2));
    const double c = (m1 * m1) / (s1 * s1) - (m2 * m2) / (s2 * s2) - 2.0 * std::log(s2 / s1);
    const double disc = std::max(b * b - 4.0 * a * c, 0.0);
    const double q = -0.5 * (b + (b >= 0.0 ? 1.0 : -1.0) * std::sqrt(disc));
    double x1 = q / a, x2 = q != 0.0 ? c / q : x1;
    if (x1 > x2) std::swap(x1, x2);
    // tails of f1 beyond x1 and x2, and the mass of f2 between them
    const double t1 = 0.5 * std::erfc((m1 - x1) / (r2 * s1));
    const double t2 = 0.5 * std::erfc((x2 - m1) / (r2 * s1));
    const double mid = 0.5 * (std::erfc((x1 - m2) / (r2 * s2)) - std::erfc((x2 - m2) / (r2 * s2)));
    return t1 + mid + t2;
}

}  // namespace

int stein_icp_posterior_scores(const double* a, int64_t na, const double* b, int64_t nb, double* kl, double* ovl)
{
    if (!a || !b) return fail(STEIN_ICP_E_INVALID, "a sample array is NULL");
    if (na < 2 || nb < 2) return fail(STEIN_ICP_E_INVALID, "each sample set needs at least 2 poses");
    for (int64_t i = 0; i < 6 * na; ++i)
        if (!std::isfinite(a[i])) return fail(STEIN_ICP_E_INVALID, "a sample is non-finite");
    for (int64_t i = 0; i < 6 * nb; ++i)
        if (!std::isfinite(b[i])) return fail(STEIN_ICP_E_INVALID, "a sample is non-finite");
    // angles around the circular mean of the reference set b
    double centre[3];
    for (int d = 0; d < 3; ++d) {
        double sn = 0.0, cs = 0.0;
        for (int64_t i = 0; i < nb; ++i) {
            sn += std::sin(b[6 * i + 3 + d]);
            cs += std::cos(b[6 * i + 3 + d]);
        }
        centre[d] = std::atan2(sn, cs);
    }
    double mu_a[2][3], S_a[2][9], mu_b[2][3], S_b[2][9];
    for (int g = 0; g < 2; ++g) {
        fit3(a, na, 3 * g, g ? centre : nullptr, mu_a[g], S_a[g]);
        fit3(b, nb, 3 * g, g ? centre : nullptr, mu_b[g], S_b[g]);
    }
    double k[2], o[6];
    for (int g = 0; g < 2; ++g)
        if (!kl_gauss3(mu_a[g], S_a[g], mu_b[g], S_b[g], &k[g]))
            return fail(STEIN_ICP_E_INVALID, "a sample covariance is not positive definite");
    for (int g = 0; g < 2; ++g)
        for (int d = 0; d < 3; ++d)
            o[3 * g + d] = ovl_normal(mu_a[g][d], std::sqrt(S_a[g][4 * d]), mu_b[g][d], std::sqrt(S_b[g][4 * d]));
    if (kl)
        for (int g = 0; g < 2; ++g) kl[g] = k[g];
    if (ovl)
        for (int d = 0; d < 6; ++d) ovl[d] = o[d];
    return STEIN_ICP_OK;
}

int stein_icp_make_schedule(uint64_t seed, int64_t n_src, int32_t m, int32_t rows, int32_t* out_host)
{
    if (!out_host) return fail(STEIN_ICP_E_INVALID, "out_host is NULL");
    if (m < 1 || rows < 1 || n_src < m || n_src > kMaxRef)
        return fail(STEIN_ICP_E_INVALID, "need 1 <= m <= n_src < 2^31 - 64 and rows >= 1");
    make_schedule(seed, n_src, m, rows, out_host);
    return STEIN_ICP_OK;
}

int stein_icp_make_init(uint64_t seed, int32_t K, double half_trans, double half_rot, const double* centre,
                        double* out_host)
{
    if (!out_host) return fail(STEIN_ICP_E_INVALID, "out_host is NULL");
    if (K < 1) return fail(STEIN_ICP_E_INVALID, "K must be >= 1");
    if (!(std::isfinite(half_trans) && half_trans >= 0.0 && std::isfinite(half_rot) && half_rot >= 0.0))
        return fail(STEIN_ICP_E_INVALID, "half widths must be finite and >= 0");
    make_init(seed, K, half_trans, half_rot, centre, out_host);
    return STEIN_ICP_OK;
}

}  // extern "C"
