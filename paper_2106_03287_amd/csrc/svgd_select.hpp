// Median-heuristic bandwidths (Sec. V, Eq. 17) of the Stein direction: the
// argument structures of the direction / update stage, the particle
// distances, the exact order-statistic selection on a workgroup, and the
// bandwidth workgroup body. Device functions only (the kernels that run them
// live with their launches), so both translation units can include it.
#pragma once

#include "common.hpp"

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
    double* theta;        // current particles, K x 6 per pair
    double* theta_next;   // particles after this iteration's update (the buffers alternate)
    double* mom;
    double* vel;
    int64_t* step;        // completed updates per pair
    int64_t* step_next;   // step + 1, written by the update
    const double* gbar;
    double* phi;
    double* h;            // 2 per pair
    double* dscr;         // K(K-1)/2 per pair and block: the pair distances or keys in global memory
    Pose* pose;
    const float4* src4;
    const int32_t* sched;
    float4* queries;      // FP32 queries of the next iteration
    int32_t K, m, rows, pad_;
    SvgdParams prm;
};

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kSvgdWaves = kSvgdThreads / kWave;
constexpr int kCandCap = 1024;   // values ranked directly once a bin holds this few
constexpr int kUnroll = 8;       // global loads in flight per thread in a pass

// Wrapped angle difference in (-pi, pi]: x - 2 pi round(x / 2 pi). Odd:
// wrap_pi(-x) == -wrap_pi(x) exactly (round-half-even and the products are
// sign-symmetric).
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

// Start of row k of the row-major upper triangle (pairs (k, l), l > k).
__device__ __forceinline__ int64_t tri_row(int k, int K) { return (int64_t)k * K - (int64_t)k * (k + 1) / 2; }

// Pair (k, l), k < l, of upper-triangle index q.
__device__ __forceinline__ void tri_pair(int64_t q, int K, int& k, int& l)
{
    const double b = 2.0 * K - 1.0;
    int kk = (int)floor((b - sqrt(b * b - 8.0 * (double)q)) * 0.5);
    kk = max(0, min(kk, K - 2));
    while (kk > 0 && tri_row(kk, K) > q) --kk;
    while (kk < K - 2 && tri_row(kk + 1, K) <= q) ++kk;
    k = kk;
    l = (int)(q - tri_row(kk, K)) + kk + 1;
}

struct SelectShared {
    uint32_t hist[4096];
    double cand[kCandCap];
    uint32_t wsum[kSvgdWaves];
    double wmin[kSvgdWaves], wmax[kSvgdWaves];
    double dres;
    uint64_t u64a, u64b;
    uint32_t bin, before, count, ncand, found, bin_b, end_b;
};

// Exact squared distance of upper-triangle pair q from the particles in LDS.
__device__ __forceinline__ double pair_dist(int64_t q, int K, int rot, const double* th)
{
    int k, l;
    tri_pair(q, K, k, l);
    return rot ? dist2_rot(th + 6 * k, th + 6 * l) : dist2_trans(th + 6 * k, th + 6 * l);
}

// 16-bit order key of a non-negative distance: the top half of its FP32 bit
// pattern. Both roundings are monotone, so key(x) < key(y) implies x < y and
// the pairs whose keys lie in [lo, hi] form a contiguous run of the exact
// order.
__device__ __forceinline__ uint16_t order_key(double x) { return (uint16_t)(__float_as_uint((float)x) >> 16); }

// The selection below runs on a workgroup of NT threads (NT = 256, 512 or
// 1024; the bandwidth role of the gradient launch uses 1024, that of a
// nearest-neighbour launch the search's workgroup size).

// Exact distances of the pairs whose LDS key lies in [lo, hi], recomputed on
// each visit (radix fallback for runs of equal keys).
template <int NT>
struct KeyRunValues {
    const uint16_t* key;
    int64_t n;
    uint32_t lo, hi;
    int K, rot;
    const double* th;
    template <class F>
    __device__ __forceinline__ void visit(F&& f) const
    {
        for (int64_t q = threadIdx.x; q < n; q += NT) {
            const uint32_t x = key[q];
            if (x >= lo && x <= hi) f(pair_dist(q, K, rot, th));
        }
    }
};

// Values in global memory, visited with kUnroll loads in flight per thread.
template <int NT>
struct GlobalValues {
    const double* v;
    int64_t n;
    template <class F>
    __device__ __forceinline__ void visit(F&& f) const
    {
        for (int64_t base = threadIdx.x; base < n; base += (int64_t)kUnroll * NT) {
            double x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = base + (int64_t)u * NT;
                x[u] = i < n ? v[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (base + (int64_t)u * NT < n) f(x[u]);
        }
    }
};

// Exclusive prefix of one value per thread over the workgroup.
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

// Find the histogram bin holding rank r (0-based) of nb <= 4096 bins; sets
// sh.bin / sh.before / sh.count. 4096 / NT consecutive bins per thread.
template <int NT>
__device__ __forceinline__ void find_rank_bin(uint32_t nb, int64_t r, SelectShared& sh)
{
    constexpr int BPT = 4096 / NT;
    const int tid = threadIdx.x;
    if (tid == 0) {
        sh.bin = 0;
        sh.before = 0;
        sh.count = 0;
    }
    uint32_t c[BPT], loc = 0;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const uint32_t bin = BPT * tid + b;
        c[b] = bin < nb ? sh.hist[bin] : 0u;
        loc += c[b];
    }
    const uint32_t excl = block_exclusive_scan(loc, sh);
    if ((int64_t)excl <= r && r < (int64_t)(excl + loc)) {
        uint32_t run = excl;
#pragma unroll
        for (int b = 0; b < BPT; ++b) {
            if ((int64_t)run <= r && r < (int64_t)(run + c[b])) {
                sh.bin = BPT * tid + b;
                sh.before = run;
                sh.count = c[b];
            }
            run += c[b];
        }
    }
    __syncthreads();
}

// Block-wide min and max over the values accepted by `pred`.
template <int NT, class Src, class P>
__device__ __forceinline__ void block_minmax(const Src& src, P&& pred, SelectShared& sh, double& mn, double& mx)
{
    double a = __builtin_inf(), b = -__builtin_inf();
    src.visit([&](double x) {
        if (pred(x)) {
            a = fmin(a, x);
            b = fmax(b, x);
        }
    });
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a = fmin(a, __shfl_xor(a, o));
        b = fmax(b, __shfl_xor(b, o));
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    if (lane == 0) {
        sh.wmin[wave] = a;
        sh.wmax[wave] = b;
    }
    __syncthreads();
    mn = sh.wmin[0];
    mx = sh.wmax[0];
    for (int w = 1; w < NT / kWave; ++w) {
        mn = fmin(mn, sh.wmin[w]);
        mx = fmax(mx, sh.wmax[w]);
    }
    __syncthreads();
}

// Exact rank-r order statistic of non-negative doubles by radix selection on
// their bit patterns (any finite or infinite values).
template <int NT, class Src>
__device__ __forceinline__ double select_radix(const Src& src, int64_t r, SelectShared& sh)
{
    const int tid = threadIdx.x;
    uint64_t prefix = 0, mask = 0;
    // digits: bits 63..52, 51..40, 39..28, 27..16, 15..4, 3..0
    for (int pass = 0; pass < 6; ++pass) {
        const int sft = pass < 5 ? 52 - 12 * pass : 0;
        const uint32_t nb = pass < 5 ? 4096u : 16u;
        const uint64_t dmask = (uint64_t)(nb - 1);
        for (uint32_t b = tid; b < 4096; b += NT) sh.hist[b] = 0;
        __syncthreads();
        src.visit([&](double x) {
            const uint64_t u = (uint64_t)__double_as_longlong(x);
            if ((u & mask) == prefix) atomicAdd(&sh.hist[(u >> sft) & dmask], 1u);
        });
        __syncthreads();
        find_rank_bin<NT>(nb, r, sh);
        prefix |= (uint64_t)sh.bin << sft;
        mask |= dmask << sft;
        r -= sh.before;
        const uint32_t cnt = sh.count;
        __syncthreads();
        if (cnt == 1 && pass < 5) {
            src.visit([&](double x) {
                const uint64_t u = (uint64_t)__double_as_longlong(x);
                if ((u & mask) == prefix) sh.u64a = u;
            });
            __syncthreads();
            const uint64_t res = sh.u64a;
            __syncthreads();
            return __longlong_as_double((long long)res);
        }
    }
    return __longlong_as_double((long long)prefix);
}

// Exact rank-r order statistic (0-based) of non-negative doubles.
template <int NT, class Src>
__device__ __forceinline__ double block_select(const Src& src, int64_t r, SelectShared& sh)
{
    const int tid = threadIdx.x;
    double lo, hi;
    block_minmax<NT>(src, [](double) { return true; }, sh, lo, hi);
    // every round shrinks the range by the bin count; the bound only matters
    // for non-finite inputs, which go to the bit-pattern radix select
    for (int round = 0; round < 64; ++round) {
        if (lo == hi) return lo;                       // every candidate equal
        const double width = hi - lo;
        const double scale = 4096.0 / width;
        if (!(width < __builtin_inf()) || !(scale < __builtin_inf())) break;
        auto inside = [&](double x) { return x >= lo && x <= hi; };
        auto bin_of = [&](double x) { return min(4095, (int)((x - lo) * scale)); };
        for (uint32_t b = tid; b < 4096; b += NT) sh.hist[b] = 0;
        if (tid == 0) sh.ncand = 0;
        __syncthreads();
        src.visit([&](double x) {
            if (inside(x)) atomicAdd(&sh.hist[bin_of(x)], 1u);
        });
        __syncthreads();
        find_rank_bin<NT>(4096, r, sh);
        const int b = (int)sh.bin;
        const uint32_t cnt = sh.count;
        r -= sh.before;
        __syncthreads();
        auto in_bin = [&](double x) { return inside(x) && bin_of(x) == b; };
        if (cnt <= kCandCap) {
            src.visit([&](double x) {
                if (in_bin(x)) {
                    const uint32_t slot = atomicAdd(&sh.ncand, 1u);
                    if (slot < kCandCap) sh.cand[slot] = x;
                }
            });
            __syncthreads();
            const uint32_t c = min(sh.ncand, (uint32_t)kCandCap);
            for (uint32_t t = tid; t < c; t += NT) {
                const double x = sh.cand[t];
                uint32_t less = 0, leq = 0;
#pragma unroll 8
                for (uint32_t j = 0; j < c; ++j) {
                    const double y = sh.cand[j];
                    less += y < x;
                    leq += y <= x;
                }
                if ((int64_t)less <= r && r < (int64_t)leq) sh.dres = x;   // same value for all writers
            }
            __syncthreads();
            const double res = sh.dres;
            __syncthreads();
            return res;
        }
        // narrow to the selected bin: the monotone bin map makes the bin's
        // values exactly those in [min, max] of the bin
        block_minmax<NT>(src, in_bin, sh, lo, hi);
    }
    return select_radix<NT>(src, r, sh);
}

// Exact order statistics r and, if `want_next`, r + 1 (0-based) of the n
// pair distances whose 16-bit keys are in LDS. Integer binning of the key
// range narrows the candidates to one bin (at most two rounds from 65536
// key values); the exact FP64 distances of the final candidates are
// recomputed and ranked by counting. *got_next is false when r + 1 lies
// outside the final candidates.
template <int NT>
__device__ inline double select_keyed(const uint16_t* key, int64_t n, int64_t r, bool want_next, int K, int rot,
                                      const double* th, SelectShared& sh, double* next, bool* got_next)
{
    const int tid = threadIdx.x;
    *got_next = false;
    uint32_t lo = 0, hi = 0xffffu;
    for (int round = 0; round < 4; ++round) {
        const uint32_t range = hi - lo + 1;
        int sft = 0;
        while ((range - 1) >> sft >= 4096u) ++sft;
        for (uint32_t i = tid; i < 4096; i += NT) sh.hist[i] = 0;
        __syncthreads();
        for (int64_t q = tid; q < n; q += NT) {
            const uint32_t x = key[q];
            if (x >= lo && x <= hi) atomicAdd(&sh.hist[(x - lo) >> sft], 1u);
        }
        __syncthreads();
        find_rank_bin<NT>(4096, r, sh);
        const uint32_t b = sh.bin, cnt = sh.count;
        r -= sh.before;
        __syncthreads();
        const uint32_t nlo = lo + (b << sft);
        const uint32_t nhi = min(hi, nlo + (1u << sft) - 1u);
        if (cnt <= (uint32_t)kCandCap) {
            if (tid == 0) {
                sh.ncand = 0;
                sh.found = 0;
            }
            __syncthreads();
            // walk the triangle as the keys were written (wavefront per row k,
            // lanes over l), so a taken key's pair needs no index inversion
            const int lane = tid & (kWave - 1);
            for (int k = tid >> 6; k < K; k += NT / kWave) {
                const int64_t row = tri_row(k, K);
                for (int l = k + 1 + lane; l < K; l += kWave) {
                    const uint32_t x = key[row + (l - k - 1)];
                    if (x >= nlo && x <= nhi) {
                        const uint32_t slot = atomicAdd(&sh.ncand, 1u);
                        if (slot < kCandCap)
                            sh.cand[slot] = rot ? dist2_rot(th + 6 * k, th + 6 * l) : dist2_trans(th + 6 * k, th + 6 * l);
                    }
                }
            }
            __syncthreads();
            const uint32_t c = min(sh.ncand, (uint32_t)kCandCap);
            // rank every candidate among all: candidate i and j range g of
            // G = NT / c ranges per thread, counts added in the histogram's
            // (no longer needed) slots (c > NT: a thread ranks several)
            for (uint32_t i = tid; i < 2 * c; i += NT) sh.hist[i] = 0;
            __syncthreads();
            const uint32_t G = c && c <= (uint32_t)NT ? (uint32_t)NT / c : 1u;
            for (uint32_t t = tid; t < c * G; t += NT) {
                const uint32_t i = t % c, g = t / c;
                const uint32_t j0 = c * g / G, j1 = c * (g + 1) / G;
                const double x = sh.cand[i];
                uint32_t less = 0, leq = 0;
#pragma unroll 8
                for (uint32_t j = j0; j < j1; ++j) {
                    const double y = sh.cand[j];
                    less += y < x;
                    leq += y <= x;
                }
                if (less) atomicAdd(&sh.hist[i], less);
                if (leq) atomicAdd(&sh.hist[c + i], leq);
            }
            __syncthreads();
            for (uint32_t t = tid; t < c; t += NT) {
                const double x = sh.cand[t];
                const uint32_t less = sh.hist[t], leq = sh.hist[c + t];
                if ((int64_t)less <= r && r < (int64_t)leq) sh.dres = x;   // same value for all writers
                if (want_next && (int64_t)less <= r + 1 && r + 1 < (int64_t)leq) {
                    sh.wmax[0] = x;
                    sh.found = 1;
                }
            }
            __syncthreads();
            const double res = sh.dres;
            *got_next = sh.found != 0;
            *next = sh.wmax[0];
            __syncthreads();
            return res;
        }
        lo = nlo;
        hi = nhi;
        if (lo == hi) break;    // one key value held by more than kCandCap pairs
    }
    return select_radix<NT>(KeyRunValues<NT>{key, n, lo, hi, K, rot, th}, r, sh);
}

// Ranks ra and rb (rb is ra or ra + 1) of the K(K-1)/2 pair distances
// whose 16-bit keys are in LDS, in one pass: the keys' own range is binned
// (one key value per bin when it spans at most 4096 values), one scan finds
// the bins of both ranks, and the exact FP64 distances of the pairs in those
// bins (adjacent ranks: nothing lies between them) are ranked by counting.
// When those bins hold more than kCandCap pairs, select_keyed narrows each
// rank on its own.
// Before the barrier that publishes the keys: the wavefronts' key ranges,
// a cleared histogram and reset selection fields (kmin / kmax: this
// thread's keys).
template <int NT>
__device__ inline void select_pair_prologue(uint32_t kmin, uint32_t kmax, SelectShared& sh)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o));
    }
    if (lane == 0) sh.wsum[wave] = kmin | (kmax << 16);
    for (uint32_t i = tid; i < 4096; i += NT) sh.hist[i] = 0;
    if (tid == 0) {
        sh.bin = 0;
        sh.before = 0;
        sh.bin_b = 0;
        sh.end_b = 0;
        sh.ncand = 0;
    }
}

template <int NT>
__device__ inline void select_pair_keyed(const uint16_t* key, int64_t n, int64_t ra, int64_t rb, int K, int rot,
                                         const double* th, SelectShared& sh, double& va, double& vb)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    uint32_t lo = 0xffffu, hi = 0u;
    constexpr int BPT = 4096 / NT;   // histogram bins per thread
    for (int w = 0; w < NT / kWave; ++w) {
        const uint32_t v = sh.wsum[w];
        lo = min(lo, v & 0xffffu);
        hi = max(hi, v >> 16);
    }
    const uint32_t range = hi - lo + 1;
    int sft = 0;
    while ((range - 1) >> sft >= 4096u) ++sft;
    for (int64_t q = tid; q < n; q += NT) atomicAdd(&sh.hist[((uint32_t)key[q] - lo) >> sft], 1u);
    __syncthreads();
    uint32_t c[BPT], loc = 0;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        c[b] = sh.hist[BPT * tid + b];
        loc += c[b];
    }
    const uint32_t excl = block_exclusive_scan(loc, sh);
    uint32_t run = excl;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        if ((int64_t)run <= ra && ra < (int64_t)(run + c[b])) {
            sh.bin = BPT * tid + b;
            sh.before = run;
        }
        if ((int64_t)run <= rb && rb < (int64_t)(run + c[b])) {
            sh.bin_b = BPT * tid + b;
            sh.end_b = run + c[b];
        }
        run += c[b];
    }
    __syncthreads();
    const uint32_t ba = sh.bin, bb = sh.bin_b, before = sh.before;
    const uint32_t cnt = sh.end_b - before;
    if (cnt > (uint32_t)kCandCap) {
        __syncthreads();   // every thread has read the bins before select_keyed resets them
        bool got = false;
        va = select_keyed<NT>(key, n, ra, rb != ra, K, rot, th, sh, &vb, &got);
        if (rb == ra) {
            vb = va;
        } else if (!got) {
            double unused;
            vb = select_keyed<NT>(key, n, rb, false, K, rot, th, sh, &unused, &got);
        }
        return;
    }
    const uint32_t klo = lo + (ba << sft);
    const uint32_t khi = min(hi, lo + ((bb + 1u) << sft) - 1u);
    // the pairs of the two bins, walking the triangle as the keys were
    // written (wavefront per row k, lanes over l)
    for (int k = wave; k < K; k += NT / kWave) {
        const int64_t row = tri_row(k, K);
        for (int l = k + 1 + lane; l < K; l += kWave) {
            const uint32_t x = key[row + (l - k - 1)];
            if (x >= klo && x <= khi) {
                const uint32_t slot = atomicAdd(&sh.ncand, 1u);
                if (slot < kCandCap)
                    sh.cand[slot] = rot ? dist2_rot(th + 6 * k, th + 6 * l) : dist2_trans(th + 6 * k, th + 6 * l);
            }
        }
    }
    __syncthreads();
    const uint32_t nc = min(sh.ncand, (uint32_t)kCandCap);
    const int64_t qa = ra - before, qb = rb - before;
    if (nc <= (uint32_t)NT / 4) {
        // few candidates: each ranked by one thread against all
        if ((uint32_t)tid < nc) {
            const double x = sh.cand[tid];
            uint32_t less = 0, leq = 0;
            for (uint32_t j = 0; j < nc; ++j) {
                const double y = sh.cand[j];
                less += y < x;
                leq += y <= x;
            }
            if ((int64_t)less <= qa && qa < (int64_t)leq) sh.dres = x;       // same value for all writers
            if ((int64_t)less <= qb && qb < (int64_t)leq) sh.wmax[0] = x;
        }
    } else {
        for (uint32_t i = tid; i < 2 * nc; i += NT) sh.hist[i] = 0;
        __syncthreads();
        // rank every candidate among all: candidate i and range g of the
        // G = NT / nc ranges per thread (nc > NT: a thread ranks several)
        const uint32_t G = nc <= (uint32_t)NT ? (uint32_t)NT / nc : 1u;
        for (uint32_t t = tid; t < nc * G; t += NT) {
            const uint32_t i = t % nc, g = t / nc;
            const uint32_t j0 = nc * g / G, j1 = nc * (g + 1) / G;
            const double x = sh.cand[i];
            uint32_t less = 0, leq = 0;
#pragma unroll 8
            for (uint32_t j = j0; j < j1; ++j) {
                const double y = sh.cand[j];
                less += y < x;
                leq += y <= x;
            }
            if (less) atomicAdd(&sh.hist[i], less);
            if (leq) atomicAdd(&sh.hist[nc + i], leq);
        }
        __syncthreads();
        for (uint32_t t = tid; t < nc; t += NT) {
            const double x = sh.cand[t];
            const uint32_t less = sh.hist[t], leq = sh.hist[nc + t];
            if ((int64_t)less <= qa && qa < (int64_t)leq) sh.dres = x;
            if ((int64_t)less <= qb && qb < (int64_t)leq) sh.wmax[0] = x;
        }
    }
    __syncthreads();
    va = sh.dres;
    vb = sh.wmax[0];
}

// Pair distances of the bandwidth kernel are kept as 16-bit keys in LDS up
// to this many pairs (K up to about 345); beyond, as FP64 in global memory.
constexpr int64_t kMaxKeyedPairs = 60000;

// Whether bandwidth_body may select over the 16-bit pair keys of K particles.
__host__ __device__ inline bool bandwidth_keyable(int K) { return (int64_t)K * (K - 1) / 2 <= kMaxKeyedPairs; }

// Where bandwidth_body keeps the pair distances: 16-bit keys in LDS, 16-bit
// keys in global memory (the `dscr` scratch), or FP64 distances in global
// memory. All three find the same exact order statistics.
enum BandwidthForm : int32_t { kKeysInLds = 0, kKeysInGlobal = 1, kDistancesInGlobal = 2 };

// grid (pairs, 2), 1024 threads. blockIdx.y: 0 translation, 1 rotation.
// Dynamic LDS: K x 6 particles (FP64) followed by the 16-bit pair keys.
// Median-heuristic bandwidth of pair p, block rot (0 translation, 1
// rotation), by one NT-thread workgroup; `sh` and `dyn`
// (bandwidth_lds_bytes(K, form)) are the workgroup's LDS. `form`
// (BandwidthForm; the key forms only where bandwidth_keyable(K)) places the
// pair distances.
template <int NT>
__device__ __forceinline__ void bandwidth_body(const SvgdArgs& a, int64_t p, int rot, int form, SelectShared& sh,
                                               double* dyn)
{
    const int K = a.K;
    const int tid = threadIdx.x;
    if (a.prm.bandwidth == 1 || K < 2) {
        if (tid == 0) a.h[2 * p + rot] = a.prm.bandwidth == 1 ? (rot ? a.prm.h_fixed_r : a.prm.h_fixed_t) : 1.0;
        return;
    }
    double* th = dyn;
    for (int e = tid; e < 6 * K; e += NT) th[e] = a.theta[p * K * 6 + e];
    __syncthreads();
    const int64_t np = (int64_t)K * (K - 1) / 2;
    const int64_t ra = (np - 1) / 2, rb = np / 2;
    double va, vb;
    if (form != kDistancesInGlobal) {
        uint16_t* key = form == kKeysInLds ? reinterpret_cast<uint16_t*>(dyn + 6 * K)
                                           : reinterpret_cast<uint16_t*>(a.dscr + (p * 2 + rot) * np);
        // the keys, their range (per wavefront) and the cleared histogram
        // of the selection, under one barrier
        uint32_t kmin = 0xffffu, kmax = 0u;
        for (int k = tid >> 6; k < K; k += NT / kWave) {
            const int64_t row = tri_row(k, K);
            for (int l = k + 1 + (tid & (kWave - 1)); l < K; l += kWave) {
                const uint16_t x = order_key(rot ? dist2_rot(th + 6 * k, th + 6 * l) : dist2_trans(th + 6 * k, th + 6 * l));
                key[row + (l - k - 1)] = x;
                kmin = min(kmin, (uint32_t)x);
                kmax = max(kmax, (uint32_t)x);
            }
        }
        select_pair_prologue<NT>(kmin, kmax, sh);
        if (form == kKeysInGlobal) __threadfence_block();
        __syncthreads();
        select_pair_keyed<NT>(key, np, ra, rb, K, rot, th, sh, va, vb);
    } else {
        double* d = a.dscr + (p * 2 + rot) * np;
        for (int k = tid >> 6; k < K; k += NT / kWave) {
            const int64_t row = tri_row(k, K);
            for (int l = k + 1 + (tid & (kWave - 1)); l < K; l += kWave)
                d[row + (l - k - 1)] = rot ? dist2_rot(th + 6 * k, th + 6 * l) : dist2_trans(th + 6 * k, th + 6 * l);
        }
        __threadfence_block();
        __syncthreads();
        const GlobalValues<NT> src{d, np};
        va = block_select<NT>(src, ra, sh);
        vb = rb == ra ? va : block_select<NT>(src, rb, sh);
    }
    if (tid == 0) {
        const double med = (ra == rb) ? sqrt(va) : 0.5 * (sqrt(va) + sqrt(vb));
        a.h[2 * p + rot] = med > 0.0 ? (med * med) / log((double)K) : 1.0;
    }
}

// LDS bytes of bandwidth_body besides SelectShared.
inline size_t bandwidth_lds_bytes(int K, int form)
{
    const int64_t np = (int64_t)K * (K - 1) / 2;
    size_t b = 48 * (size_t)K;
    if (form == kKeysInLds) b += 2 * (size_t)np;
    return (b + 15) / 16 * 16;
}

// Dynamic LDS bytes of a bandwidth workgroup (SelectShared, then the
// particles and keys of bandwidth_body).
inline size_t bandwidth_role_lds_bytes(int K, int form)
{
    return (sizeof(SelectShared) + 15) / 16 * 16 + bandwidth_lds_bytes(K, form);
}

// Bandwidth workgroup b of a launch (pair b / 2, block b % 2) on NT threads;
// lds: its dynamic LDS of bandwidth_role_lds_bytes(K, form) bytes.
template <int NT>
__device__ __forceinline__ void bandwidth_role(const SvgdArgs& v, int64_t b, int form, double* lds)
{
    SelectShared& sh = *reinterpret_cast<SelectShared*>(lds);
    double* dyn = lds + (sizeof(SelectShared) + 15) / 16 * 2;
    bandwidth_body<NT>(v, b >> 1, (int)(b & 1), form, sh, dyn);
}

}  // namespace sicp
