// Brute-force nearest neighbour (Eq. 1) in FP32 on gfx950 vector ALUs.
//
// Work item = (pair, query block, reference chunk); one workgroup of W
// wavefronts per item. Every lane owns Q queries, read from the query buffer
// (each is a particle's FP64 transform of a minibatch point, rounded once to
// FP32, written when the particle's pose was last updated). The chunk is split
// in W wave-uniform sub-ranges, so the reference coordinates are
// wave-uniform and are read with scalar loads straight into SGPRs: no LDS
// staging and no barrier in the scan. Per reference tile of kTile points a
// lane keeps only the tile minimum (3-input min), and per tile one compare
// and two selects record a better tile. Waves are merged through LDS with a
// 64-bit min over (distance bits, tile) keys and one key per query and chunk
// is written. The consumer reduces the keys over chunks and rescans only the
// winning tile for the lowest index with the smallest distance, once per
// query instead of once per chunk and wave.
#pragma once

#include "common.hpp"

namespace sicp {

struct NNArgs {
    const WorkItem* work;
    const PairDesc* pairs;    // NN groups: queries at q_off, nq of them, keys at part_off
    const float4* ref4;
    const float4* queries;
    uint64_t* partial;
    int64_t nwork;
};

// One work item: queries of a block against one reference chunk.
template <int Q, int W>
__device__ __forceinline__ void nn_item(const NNArgs& a, const WorkItem w, uint64_t (*sk)[kWave * Q])
{
    const PairDesc pd = a.pairs[w.pair];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x >> 6);
    const int64_t nq = pd.nq;
    const int64_t qbase = (int64_t)w.qblock * kWave * Q;

    float qx[Q], qy[Q], qz[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const int64_t qi = qbase + s * kWave + lane;
        qx[s] = qy[s] = qz[s] = 0.0f;
        if (qi < nq) {
            const float4 qq = a.queries[pd.q_off + qi];
            qx[s] = qq.x;
            qy[s] = qq.y;
            qz[s] = qq.z;
        }
    }

    // this wave's tiles of the chunk
    const int64_t c0 = (int64_t)w.chunk * pd.chunk;
    const int64_t cend = min(c0 + (int64_t)pd.chunk, pd.n_ref_pad);
    const int64_t ntiles = (cend - c0) / kTile;
    const int64_t t0 = (ntiles * wave) / W;
    const int64_t t1 = (ntiles * (wave + 1)) / W;
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

    // key = (distance bits, global tile index): the minimum over waves and
    // chunks is the smallest distance and, among equal ones, the first tile;
    // the consumer rescans that one tile for the lowest index
    uint64_t key[Q];
#pragma unroll
    for (int s = 0; s < Q; ++s)
        key[s] = (t0 < t1) ? pack_key(best[s], (uint32_t)(c0 / kTile + btile[s])) : ~0ull;

#pragma unroll
    for (int s = 0; s < Q; ++s) sk[wave][s * kWave + lane] = key[s];
    __syncthreads();
    for (int j = threadIdx.x; j < kWave * Q; j += kWave * W) {
        const int64_t qi = qbase + j;
        if (qi < nq) {
            uint64_t k0 = sk[0][j];
#pragma unroll
            for (int v = 1; v < W; ++v) k0 = min(k0, sk[v][j]);
            a.partial[pd.part_off + (int64_t)w.chunk * nq + qi] = k0;
        }
    }
    __syncthreads();   // sk is reused by the next item of a persistent workgroup
}

// grid = nwork: one item per workgroup; a smaller grid makes the workgroups
// persistent, each walking the work table with a grid stride (the table is
// built so items have near-equal cost, which balances a static stride).
template <int Q, int W>
__global__ __launch_bounds__(kWave * W) void nn_fp32_kernel(NNArgs a)
{
    __shared__ uint64_t sk[W][kWave * Q];
    for (int64_t it = blockIdx.x; it < a.nwork; it += gridDim.x) nn_item<Q, W>(a, a.work[it], sk);
}

// Smallest of `chunks` keys strided by `stride`, eight loads in flight.
__device__ __forceinline__ uint64_t min_chunk_keys(const uint64_t* __restrict__ kp, int chunks, int64_t stride)
{
    uint64_t key = ~0ull;
    for (int c0 = 0; c0 < chunks; c0 += 8) {
        uint64_t kk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) kk[u] = c0 + u < chunks ? kp[(int64_t)(c0 + u) * stride] : ~0ull;
#pragma unroll
        for (int u = 0; u < 8; ++u) key = min(key, kk[u]);
    }
    return key;
}

// Reference index of a reduced key: the lowest position in the key's tile
// whose FP32 distance (same arithmetic as the scan) equals the key's.
__device__ __forceinline__ int32_t resolve_key(uint64_t key, float4 q, const float4* __restrict__ ref4,
                                               int64_t n_ref_pad)
{
    uint32_t tile = (uint32_t)(key & 0xffffffffull);
    if ((int64_t)tile >= n_ref_pad / kTile) tile = 0;   // never produced by the scan; keeps reads in bounds
    const float best = __uint_as_float((uint32_t)(key >> 32));
    const float4* __restrict__ r = ref4 + (int64_t)tile * kTile;
    float d[kTile];
#pragma unroll
    for (int u = 0; u < kTile; ++u) {
        const float4 rr = r[u];
        d[u] = dist2_f32(q.x, q.y, q.z, rr.x, rr.y, rr.z);
    }
    int32_t idx = (int32_t)(tile * kTile);
#pragma unroll
    for (int u = kTile - 1; u >= 0; --u)
        if (d[u] == best) idx = (int32_t)(tile * kTile + u);
    return idx;
}

// Reference index of a reduced key: keyed by tile (the FP32 search), or by
// the index itself (the BF16 screen, whose exact rerank knows it).
__device__ __forceinline__ int32_t key_index(uint64_t key, bool by_index, float4 q, const float4* __restrict__ ref4,
                                             int64_t n_ref_pad)
{
    if (!by_index) return resolve_key(key, q, ref4, n_ref_pad);
    const int64_t j = (int64_t)(key & 0xffffffffull);
    return (int32_t)(j < n_ref_pad ? j : 0);   // never out of range from the screen; keeps reads in bounds
}

// Reduce the per-chunk keys of directly given queries (standalone search).
__global__ void nn_finish_kernel(const uint64_t* __restrict__ partial, const float4* __restrict__ queries,
                                 const float4* __restrict__ ref4, int64_t n_ref_pad, int64_t nq, int32_t chunks,
                                 int32_t by_index, int32_t* __restrict__ idx, float* __restrict__ d2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const uint64_t k = min_chunk_keys(partial + i, chunks, nq);
    idx[i] = key_index(k, by_index != 0, queries[i], ref4, n_ref_pad);
    if (d2) d2[i] = __uint_as_float((uint32_t)(k >> 32));
}

}  // namespace sicp
