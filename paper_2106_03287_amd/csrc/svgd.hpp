// Stein direction (Eq. 16) and particle update (Eq. 12 with Adam), one
// workgroup of 1024 threads per pair.
//
//  1. G_k = -N gbar_k + grad log p(theta_k)  (Eq. 10 with Eqs. 14-15).
//  2. Median heuristic: the K(K-1)/2 squared distances between distinct
//     particles (translation, and wrapped rotation of Eq. 17) are written to
//     a scratch array and the middle order statistics are found exactly by a
//     block-wide radix select over their IEEE-754 bit patterns (non-negative
//     doubles order like unsigned integers): 12-bit digits, 4096-bin LDS
//     histogram, early exit once the selected bin holds one value.
//  3. phi_k = (1/K) sum_l [G_l k(l,k) + grad_{theta_l} k(l,k)] for the
//     translation and rotation blocks, one wavefront per particle k, lanes
//     over l, fixed-shape shuffle reduction.
//  4. Adam on -phi (or theta += lr phi), then the next iteration's poses.
#pragma once

#include "common.hpp"
#include "prep.hpp"

namespace sicp {

struct SvgdParams {
    double lr, beta1, beta2, eps;
    double h_fixed_t, h_fixed_r;
    double prior_mu[6];
    double prior_var[3];
    double prior_kappa[3];
    int32_t optimizer, bandwidth, prior, pad_;
};

struct SvgdArgs {
    const PairDesc* pairs;
    double* theta;
    double* mom;
    double* vel;
    int64_t* step;
    const double* gbar;
    double* G;
    double* phi;
    double* h;
    double* dscr;     // 2 * K(K-1)/2 per pair
    Pose* pose;
    int32_t K, pad_;
    SvgdParams prm;
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Wrapped angle difference in (-pi, pi]: x - 2 pi round(x / 2 pi).
__device__ __forceinline__ double wrap_pi(double x)
{
#pragma clang fp contract(off)
    const double k = rint(x * (1.0 / kTwoPi));
    return x - k * kTwoPi;
}

__device__ __forceinline__ double dist2_trans(const double* __restrict__ a, const double* __restrict__ b)
{
#pragma clang fp contract(off)
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return (d0 * d0 + d1 * d1) + d2 * d2;
}

__device__ __forceinline__ double dist2_rot(const double* __restrict__ a, const double* __restrict__ b)
{
#pragma clang fp contract(off)
    const double d0 = wrap_pi(a[3] - b[3]), d1 = wrap_pi(a[4] - b[4]), d2 = wrap_pi(a[5] - b[5]);
    return (d0 * d0 + d1 * d1) + d2 * d2;
}

struct SelectShared {
    uint32_t hist[4096];
    uint32_t wsum[kSvgdThreads / kWave];
    uint64_t u64a, u64b;
    uint32_t bin, before, count, found;
};

// Inclusive scan of one value per thread over the workgroup; returns the
// exclusive prefix.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, SelectShared& sh)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) sh.wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += sh.wsum[w];
    __syncthreads();
    return before + x - v;
}

// Exact rank-r order statistic (0-based) of n non-negative doubles in global
// memory, by radix selection on their bit patterns.
__device__ inline uint64_t block_select(const double* __restrict__ v, int64_t n, int64_t r,
                                        SelectShared& sh)
{
    const int tid = threadIdx.x;
    uint64_t prefix = 0, mask = 0;
    const int shifts[6] = {52, 40, 28, 16, 4, 0};
    const int widths[6] = {12, 12, 12, 12, 12, 4};
    for (int pass = 0; pass < 6; ++pass) {
        const int sft = shifts[pass];
        const uint32_t nb = 1u << widths[pass];
        const uint64_t dmask = (uint64_t)(nb - 1);
        for (uint32_t b = tid; b < 4096; b += kSvgdThreads) sh.hist[b] = 0;
        __syncthreads();
        for (int64_t i = tid; i < n; i += kSvgdThreads) {
            const uint64_t u = (uint64_t)__double_as_longlong(v[i]);
            if ((u & mask) == prefix) atomicAdd(&sh.hist[(u >> sft) & dmask], 1u);
        }
        __syncthreads();
        // four consecutive bins per thread
        uint32_t c[4], loc = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t bin = 4 * tid + b;
            c[b] = bin < nb ? sh.hist[bin] : 0u;
            loc += c[b];
        }
        const uint32_t excl = block_exclusive_scan(loc, sh);
        if ((int64_t)excl <= r && r < (int64_t)(excl + loc)) {
            uint32_t run = excl;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if ((int64_t)run <= r && r < (int64_t)(run + c[b])) {
                    sh.bin = 4 * tid + b;
                    sh.before = run;
                    sh.count = c[b];
                }
                run += c[b];
            }
        }
        __syncthreads();
        prefix |= (uint64_t)sh.bin << sft;
        mask |= dmask << sft;
        r -= sh.before;
        const uint32_t cnt = sh.count;
        __syncthreads();
        if (cnt == 1 && pass < 5) {
            for (int64_t i = tid; i < n; i += kSvgdThreads) {
                const uint64_t u = (uint64_t)__double_as_longlong(v[i]);
                if ((u & mask) == prefix) sh.u64a = u;
            }
            __syncthreads();
            const uint64_t res = sh.u64a;
            __syncthreads();
            return res;
        }
    }
    return prefix;
}

// Median-heuristic bandwidth over n = K(K-1)/2 squared distances.
__device__ inline double median_bandwidth(const double* __restrict__ v, int64_t n, int K, SelectShared& sh)
{
    const int64_t ra = (n - 1) / 2, rb = n / 2;
    const uint64_t ua = block_select(v, n, ra, sh);
    uint64_t ub = ua;
    if (rb != ra) {
        if (threadIdx.x == 0) {
            sh.u64b = ~0ull;
            sh.found = 0;
        }
        __syncthreads();
        uint32_t le = 0;
        uint64_t gt = ~0ull;
        for (int64_t i = threadIdx.x; i < n; i += kSvgdThreads) {
            const uint64_t u = (uint64_t)__double_as_longlong(v[i]);
            if (u <= ua) ++le;
            else gt = min(gt, u);
        }
        atomicAdd(&sh.found, le);
        atomicMin((unsigned long long*)&sh.u64b, (unsigned long long)gt);
        __syncthreads();
        ub = ((int64_t)sh.found >= rb + 1) ? ua : sh.u64b;
        __syncthreads();
    }
    const double a = sqrt(__longlong_as_double((long long)ua));
    const double b = sqrt(__longlong_as_double((long long)ub));
    const double med = (ra == rb) ? a : 0.5 * (a + b);
    if (!(med > 0.0)) return 1.0;
    return (med * med) / log((double)K);
}

__global__ __launch_bounds__(kSvgdThreads) void svgd_update_kernel(SvgdArgs a)
{
    const int64_t p = blockIdx.x;
    const int K = a.K;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const PairDesc pd = a.pairs[p];
    double* __restrict__ th = a.theta + p * K * 6;
    double* __restrict__ G = a.G + p * K * 6;
    const double* __restrict__ gb = a.gbar + p * K * 6;
    const int64_t t_old = a.step[p];
    __shared__ SelectShared sh;
    __shared__ double hh[2];

    // 1. posterior score per particle
    for (int e = tid; e < 6 * K; e += kSvgdThreads) {
        const int d = e % 6;
        double pg = 0.0;
        if (a.prm.prior == 1) {
            const double x = th[e] - a.prm.prior_mu[d];
            pg = d < 3 ? -x / a.prm.prior_var[d] : -a.prm.prior_kappa[d - 3] * sin(x);
        }
        G[e] = -(double)pd.n_scale * gb[e] + pg;
    }

    // 2. bandwidths
    double ht = 1.0, hr = 1.0;
    if (a.prm.bandwidth == 1) {
        ht = a.prm.h_fixed_t;
        hr = a.prm.h_fixed_r;
    } else if (K >= 2) {
        const int64_t np = (int64_t)K * (K - 1) / 2;
        double* __restrict__ dt = a.dscr + p * 2 * np;
        double* __restrict__ dr = dt + np;
        for (int64_t e = tid; e < (int64_t)K * K; e += kSvgdThreads) {
            const int k = (int)(e / K), l = (int)(e - (int64_t)k * K);
            if (l > k) {
                const int64_t lin = (int64_t)k * K - (int64_t)k * (k + 1) / 2 + (l - k - 1);
                dt[lin] = dist2_trans(th + 6 * k, th + 6 * l);
                dr[lin] = dist2_rot(th + 6 * k, th + 6 * l);
            }
        }
        __threadfence_block();
        __syncthreads();
        ht = median_bandwidth(dt, np, K, sh);
        hr = median_bandwidth(dr, np, K, sh);
    }
    __threadfence_block();
    __syncthreads();

    // 3. Stein direction, one wavefront per particle
    const int nwaves = kSvgdThreads / kWave;
    for (int k = wave; k < K; k += nwaves) {
        const double* tk = th + 6 * k;
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int l = lane; l < K; l += kWave) {
            const double* tl = th + 6 * l;
            const double* Gl = G + 6 * l;
            const double kt = exp(-dist2_trans(tl, tk) / ht);
            const double kr = exp(-dist2_rot(tl, tk) / hr);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                acc[d] += Gl[d] * kt + (-(2.0 / ht) * (tl[d] - tk[d]) * kt);
                acc[3 + d] += Gl[3 + d] * kr + (-(2.0 / hr) * wrap_pi(tl[3 + d] - tk[3 + d]) * kr);
            }
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            double x = acc[d];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
            acc[d] = x;
        }
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < 6; ++d) a.phi[(p * K + k) * 6 + d] = acc[d] / K;
        }
    }
    if (tid == 0) {
        a.h[2 * p] = ht;
        a.h[2 * p + 1] = hr;
    }
    __threadfence_block();
    __syncthreads();

    // 4. update
    const int64_t t_new = t_old + 1;
    const double* __restrict__ ph = a.phi + p * K * 6;
    if (a.prm.optimizer == 1) {
        for (int e = tid; e < 6 * K; e += kSvgdThreads) {
#pragma clang fp contract(off)
            th[e] = th[e] + a.prm.lr * ph[e];
        }
    } else {
        const double bc1 = 1.0 - pow(a.prm.beta1, (double)t_new);
        const double bc2 = 1.0 - pow(a.prm.beta2, (double)t_new);
        double* __restrict__ mo = a.mom + p * K * 6;
        double* __restrict__ ve = a.vel + p * K * 6;
        for (int e = tid; e < 6 * K; e += kSvgdThreads) {
#pragma clang fp contract(off)
            const double g = -ph[e];
            const double mm = a.prm.beta1 * mo[e] + (1.0 - a.prm.beta1) * g;
            const double vv = a.prm.beta2 * ve[e] + (1.0 - a.prm.beta2) * (g * g);
            mo[e] = mm;
            ve[e] = vv;
            const double mhat = mm / bc1;
            const double vhat = vv / bc2;
            th[e] = th[e] - a.prm.lr * mhat / (sqrt(vhat) + a.prm.eps);
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int k = tid; k < K; k += kSvgdThreads) pose_from_theta(th + 6 * k, a.pose + p * K + k);
    if (tid == 0) a.step[p] = t_new;
}

}  // namespace sicp
