// Brute-force nearest neighbour (Eq. 1) in FP32 on gfx950 vector ALUs.
//
// Work item = (pair, query block, reference chunk); one workgroup of four
// wavefronts per item. Every lane owns Q queries (the particle's FP64
// transform of a minibatch point, rounded once to FP32). The chunk is split
// in four wave-uniform sub-ranges, so the reference coordinates are
// wave-uniform and are read with scalar loads straight into SGPRs: no LDS
// staging and no barrier in the scan. Per reference tile of kTile points a
// lane keeps only the tile minimum (3-input min), and per tile one compare
// and two selects record a better tile; the index inside the winning tile is
// recovered once at the end by rescanning that tile. Waves are merged through
// LDS with a 64-bit min over (distance bits, index) keys, which keeps the
// lowest index among equal distances, and one key per query and chunk is
// written; the gradient kernel reduces over chunks.
#pragma once

#include "common.hpp"

namespace sicp {

struct NNArgs {
    const WorkItem* work;
    const PairDesc* pairs;
    const float4* src4;
    const float4* ref4;
    const int32_t* sched;
    const Pose* pose;
    const int64_t* step;      // per-pair step counter (selects the schedule row)
    const float4* queries;    // direct-query mode: packed queries (offset src_off, count n_src)
    uint64_t* partial;
    int32_t K, m, rows, pad_;
};

template <int Q, bool FROM_POSE>
__global__ __launch_bounds__(256) void nn_fp32_kernel(NNArgs a)
{
    const WorkItem w = a.work[blockIdx.x];
    const PairDesc pd = a.pairs[w.pair];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x >> 6);
    const int64_t nq = FROM_POSE ? (int64_t)a.K * a.m : pd.n_src;
    const int64_t qbase = (int64_t)w.qblock * kWave * Q;

    float qx[Q], qy[Q], qz[Q];
    int64_t row = 0;
    if (FROM_POSE) row = a.step[w.pair] % a.rows;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const int64_t qi = qbase + s * kWave + lane;
        qx[s] = qy[s] = qz[s] = 0.0f;
        if (qi < nq) {
            if (FROM_POSE) {
                const int64_t k = qi / a.m;
                const int64_t i = qi - k * a.m;
                const int32_t si = a.sched[pd.sched_off + row * a.m + i];
                const float4 sp = a.src4[pd.src_off + si];
                const Pose* P = a.pose + (int64_t)w.pair * a.K + k;
                double q[3];
                transform_f64(P->R, P->u, sp.x, sp.y, sp.z, q);
                qx[s] = (float)q[0];
                qy[s] = (float)q[1];
                qz[s] = (float)q[2];
            } else {
                const float4 qq = a.queries[pd.src_off + qi];
                qx[s] = qq.x;
                qy[s] = qq.y;
                qz[s] = qq.z;
            }
        }
    }

    // this wave's tiles of the chunk
    const int64_t c0 = (int64_t)w.chunk * pd.chunk;
    const int64_t cend = min(c0 + (int64_t)pd.chunk, pd.n_ref_pad);
    const int64_t ntiles = (cend - c0) / kTile;
    const int64_t t0 = (ntiles * wave) / 4;
    const int64_t t1 = (ntiles * (wave + 1)) / 4;
    const float4* __restrict__ rp = a.ref4 + pd.ref_off + c0;

    float best[Q];
    int32_t btile[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        best[s] = __builtin_inff();
        btile[s] = (int32_t)t0;
    }
    for (int64_t tt = t0; tt < t1; ++tt) {
        const float4* __restrict__ r = rp + tt * kTile;
        float tm[Q];
#pragma unroll
        for (int u = 0; u < kTile; ++u) {
            const float4 rr = r[u];
#pragma unroll
            for (int s = 0; s < Q; ++s) {
                const float d = dist2_f32(qx[s], qy[s], qz[s], rr.x, rr.y, rr.z);
                tm[s] = (u == 0) ? d : __builtin_fminf(tm[s], d);
            }
        }
#pragma unroll
        for (int s = 0; s < Q; ++s) {
            const bool better = tm[s] < best[s];
            best[s] = better ? tm[s] : best[s];
            btile[s] = better ? (int32_t)tt : btile[s];
        }
    }

    // index recovery inside the winning tile: the lowest position whose
    // distance equals the minimum (same arithmetic, so bitwise equal)
    uint64_t key[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        uint32_t idx = (uint32_t)(c0 + (int64_t)btile[s] * kTile);
        bool found = false;
        const float4* __restrict__ r = rp + (int64_t)btile[s] * kTile;
        for (int u = 0; u < kTile; ++u) {
            const float4 rr = r[u];
            const float d = dist2_f32(qx[s], qy[s], qz[s], rr.x, rr.y, rr.z);
            if (!found && d == best[s]) {
                found = true;
                idx = (uint32_t)(c0 + (int64_t)btile[s] * kTile + u);
            }
        }
        key[s] = (t0 < t1) ? pack_key(best[s], idx) : ~0ull;
    }

    __shared__ uint64_t sk[4][kWave * Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) sk[wave][s * kWave + lane] = key[s];
    __syncthreads();
    for (int j = threadIdx.x; j < kWave * Q; j += 256) {
        const int64_t qi = qbase + j;
        if (qi < nq) {
            uint64_t k0 = sk[0][j];
            k0 = min(k0, sk[1][j]);
            k0 = min(k0, sk[2][j]);
            k0 = min(k0, sk[3][j]);
            a.partial[pd.part_off + (int64_t)w.chunk * nq + qi] = k0;
        }
    }
}

// Reduce the per-chunk keys of directly given queries (standalone search).
__global__ void nn_finish_kernel(const uint64_t* __restrict__ partial, int64_t nq, int32_t chunks,
                                 int32_t* __restrict__ idx, float* __restrict__ d2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    uint64_t k = ~0ull;
    for (int c = 0; c < chunks; ++c) k = min(k, partial[(int64_t)c * nq + i]);
    idx[i] = (int32_t)(uint32_t)(k & 0xffffffffull);
    if (d2) d2[i] = __uint_as_float((uint32_t)(k >> 32));
}

}  // namespace sicp
