// Kernels of the learned initial-particle proposal: a point-set network that
// maps a (source, reference) cloud pair to K pose particles which then seed
// Stein ICP in place of the uniform draw of the particles (Sec. V).
//
// Network: a shared per-point MLP 3 -> 64 -> 128 -> 256 (ReLU after each
// layer) runs on every point of both clouds; each cloud is max-pooled to a
// 256-vector; the two vectors are concatenated (source first) and mapped by
// 512 -> 256 (ReLU) -> 6K, read as K row-major particles (x, y, z, roll,
// pitch, yaw).
//
// Precision: every matrix product rounds both operands to BF16 (round to
// nearest even) as it stages them into LDS and accumulates in FP32 on the
// matrix cores; master weights, activations, gradients and Adam moments are
// FP32; the set loss is evaluated in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sicp {
namespace prop {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bits, round to nearest even; infinities and NaNs keep their
// class (a NaN stays a NaN).
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u) return (uint16_t)((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------------- GEMM
// C = op(A) op(B) [+ bias] [ReLU] [+ C]   (M x N, FP32, row-major, ldc)
//   op(A) = A   with A row-major M x K (lda)   when ta == 0,
//         = A^T with A row-major K x M (lda)   when ta == 1;
//   op(B) = B   with B row-major K x N (ldb)   when tb == 0,
//         = B^T with B row-major N x K (ldb)   when tb == 1.
// Split K: workgroup z covers K range [z kper, (z + 1) kper) and writes its
// partial product, without bias, ReLU or accumulation, to C + z c_split
// (the caller then sums the splits with splitk_reduce_kernel).
// Pooled epilogue (pool_keys != nullptr, one K slice, ReLU on, rows in
// clouds of pool_P points with pool_P % 64 == 0 so that a 64-row tile lies
// in one cloud): C is not written; instead the maximum of every column over
// each cloud's rows, with its first row, is folded into
// pool_keys[cloud N + n] as the key (value bits << 32) | ~row_in_cloud
// (values are >= +0, whose bit patterns order like the values; a larger key
// is a larger value, or the same value at a smaller row).
struct GemmArgs {
    const float* A;
    const float* B;
    float* C;
    const float* bias;
    int64_t M, N, K, lda, ldb, ldc;
    int64_t kper, c_split;
    int32_t ta, tb, relu, accumulate;
    unsigned long long* pool_keys;
    int64_t pool_P;
};

constexpr int kGT = 64;    // output tile edge
constexpr int kGK = 32;    // K step (one MFMA 16x16x32 deep)
constexpr int kLdsPad = 8; // BF16 pad per LDS row: spreads banks, keeps 16-byte rows aligned

constexpr int kXcds = 8;   // workgroups are dealt to the 8 XCDs round robin

// Tile of workgroup b in a 1-D grid of ceil(Mt / 8) * 8 * Nt workgroups
// (Mt, Nt: row and column tiles). Workgroups b, b + 8, b + 16, ... land on
// the same XCD; they are given the Nt column tiles of one row tile, so the
// A rows they share are read once into that XCD's L2.
__device__ __forceinline__ bool gemm_tile(int64_t b, int64_t Mt, int64_t Nt, int64_t& mt, int64_t& nt)
{
    const int64_t grp = b / (kXcds * Nt), r = b % (kXcds * Nt);
    mt = grp * kXcds + r % kXcds;
    nt = r / kXcds;
    return mt < Mt;
}

// 256 threads, 64 x 64 output tile; wavefront w owns the 32 x 32 quarter
// (w / 2, w % 2) as 2 x 2 MFMA tiles. Both LDS tiles are K-contiguous
// ([row][k] and [col][k]), so a lane reads the eight K values of its
// fragment (row lane % 16, K slice 8 (lane / 16)) in one 16-byte load.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kGT][kGK + kLdsPad];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kGT][kGK + kLdsPad];
    int64_t mt, nt;
    if (!gemm_tile(blockIdx.x, (g.M + kGT - 1) / kGT, (g.N + kGT - 1) / kGT, mt, nt)) return;   // whole workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m0 = mt * kGT, n0 = nt * kGT;
    const int64_t kbeg = (int64_t)blockIdx.z * g.kper;
    const int64_t kend = min(g.K, kbeg + g.kper);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4_t){0.f, 0.f, 0.f, 0.f};

    for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
        // 8 elements of each operand tile per thread; the thread-to-element
        // map walks the contiguous dimension of global memory
#pragma unroll
        for (int u = 0; u < (kGT * kGK) / 256; ++u) {
            const int e = tid + 256 * u;
            const int r = g.ta ? (e % kGT) : (e / kGK);
            const int k = g.ta ? (e / kGT) : (e % kGK);
            const int64_t gm = m0 + r, gk = k0 + k;
            float v = 0.f;
            if (gm < g.M && gk < kend) v = g.ta ? g.A[gk * g.lda + gm] : g.A[gm * g.lda + gk];
            As[r][k] = to_bf16(v);
        }
#pragma unroll
        for (int u = 0; u < (kGT * kGK) / 256; ++u) {
            const int e = tid + 256 * u;
            const int c = g.tb ? (e / kGK) : (e % kGT);
            const int k = g.tb ? (e % kGK) : (e / kGT);
            const int64_t gn = n0 + c, gk = k0 + k;
            float v = 0.f;
            if (gn < g.N && gk < kend) v = g.tb ? g.B[gn * g.ldb + gk] : g.B[gk * g.ldb + gn];
            Bs[c][k] = to_bf16(v);
        }
        __syncthreads();
        const int fr = lane & 15, fk = 8 * (lane >> 4);
        bf16x8_t af[2], bfr[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
            af[a] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(&As[wm + 16 * a + fr][fk]));
#pragma unroll
        for (int b = 0; b < 2; ++b)
            bfr[b] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(&Bs[wn + 16 * b + fr][fk]));
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    // lane holds column lane % 16 and rows 4 (lane / 16) .. +3 of each tile
    if (g.pool_keys) {
        const int64_t cloud = m0 / g.pool_P;
        const int64_t rbase = m0 - cloud * g.pool_P + wm;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t gn = n0 + wn + 16 * b + (lane & 15);
            const float bias = (g.bias && gn < g.N) ? g.bias[gn] : 0.f;
            unsigned long long best = 0ull;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float v = acc[a][b][t] + bias;
                    const float r = v > 0.f ? v : 0.f;   // ReLU, canonical +0
                    const uint32_t row = (uint32_t)(rbase + 16 * a + 4 * (lane >> 4) + t);
                    const unsigned long long key =
                        ((unsigned long long)__float_as_uint(r) << 32) | (unsigned long long)(~row);
                    best = key > best ? key : best;
                }
            // the four lanes of a column hold rows 4 (lane / 16) .. +3 of the wavefront's 32
            unsigned long long o = __shfl_xor(best, 16);
            best = o > best ? o : best;
            o = __shfl_xor(best, 32);
            best = o > best ? o : best;
            if (lane < 16 && gn < g.N) atomicMax(g.pool_keys + cloud * g.N + gn, best);
        }
        return;
    }
    float* Cz = g.C + (int64_t)blockIdx.z * g.c_split;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t gm = m0 + wm + 16 * a + 4 * (lane >> 4) + t;
                const int64_t gn = n0 + wn + 16 * b + (lane & 15);
                if (gm < g.M && gn < g.N) {
                    float v = acc[a][b][t];
                    if (g.bias) v += g.bias[gn];
                    if (g.relu) v = fmaxf(v, 0.f);
                    float* dst = Cz + gm * g.ldc + gn;
                    *dst = g.accumulate ? *dst + v : v;
                }
            }
}

// -------------------------------------------------- fused per-point MLP
// The three per-point layers and the max-pool of one 64-point tile in one
// workgroup: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), h3 = relu(h2 W3 +
// b3), folded into the pool keys as in the pooled GEMM epilogue. Every
// product is a chain of v_mfma_f32_16x16x32_bf16 over K steps of 32 in
// increasing order, from zero, with the bias added to the FP32 sum and ReLU
// after it -- the arithmetic of gemm_bf16_kernel, so a row recomputed by
// that kernel has the same bits. Activations pass between the layers through
// LDS as BF16 and never reach HBM. The weights are staged once per workgroup
// as BF16, column-major with padded rows (the B-operand layout of the GEMM).
struct MlpArgs {
    const float* X;   // rows x 3
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    unsigned long long* keys;   // clouds x 256
    int64_t rows, P;            // P % 64 == 0
};

constexpr int kMT = 64;                 // points per tile
constexpr int kLd1 = 32 + kLdsPad;      // K stride of x and W1 (K = 3 padded to 32)
constexpr int kLd2 = 64 + kLdsPad;      // K stride of h1 and W2
constexpr int kLd3 = 128 + kLdsPad;     // K stride of h2 and W3
// LDS layout in BF16 elements
constexpr int kOffW1 = 0;
constexpr int kOffW2 = kOffW1 + 64 * kLd1;
constexpr int kOffW3 = kOffW2 + 128 * kLd2;
constexpr int kOffU = kOffW3 + 256 * kLd3;   // x tile, later h2 tile (one per tile in flight)
constexpr int kOffH1 = kOffU + 2 * kMT * kLd3;
constexpr int kMlpLdsElems = kOffH1 + 2 * kMT * kLd2;
constexpr int kMlpThreads = 512;              // two tiles at a time, four wavefronts each
constexpr size_t kMlpLdsBytes = 2 * (size_t)kMlpLdsElems;

__device__ __forceinline__ bf16x8_t lds_frag(const uint16_t* base, int row, int ld, int k)
{
    return __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u16x8_t*>(base + row * ld + k));
}

__global__ __launch_bounds__(kMlpThreads) void mlp_pool_kernel(MlpArgs g)
{
    extern __shared__ __attribute__((aligned(16))) uint16_t sm16[];
    uint16_t* W1s = sm16 + kOffW1;
    uint16_t* W2s = sm16 + kOffW2;
    uint16_t* W3s = sm16 + kOffW3;
    const int half = threadIdx.x >> 8;           // which of the two tiles in flight
    const int tid = threadIdx.x & 255, lane = tid & 63, wave = tid >> 6;
    uint16_t* U = sm16 + kOffU + half * kMT * kLd3;
    uint16_t* H1s = sm16 + kOffH1 + half * kMT * kLd2;
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    // weights, transposed to [column][k] BF16
    for (int e = threadIdx.x; e < 64 * 32; e += kMlpThreads) {
        const int n = e % 64, k = e / 64;
        W1s[n * kLd1 + k] = to_bf16(k < 3 ? g.W1[k * 64 + n] : 0.f);
    }
    for (int e = threadIdx.x; e < 128 * 64; e += kMlpThreads) {
        const int n = e % 128, k = e / 128;
        W2s[n * kLd2 + k] = to_bf16(g.W2[k * 128 + n]);
    }
    for (int e = threadIdx.x; e < 256 * 128; e += kMlpThreads) {
        const int n = e % 256, k = e / 256;
        W3s[n * kLd3 + k] = to_bf16(g.W3[k * 256 + n]);
    }
    const int64_t ntiles = g.rows / kMT;
    // each half takes every other tile of the workgroup's share; the loop
    // count is the same for all threads (the barriers are workgroup-wide)
    // and a half without a tile skips the work. The tile's 64 x 3 inputs,
    // one value per thread below 192, are loaded a round ahead.
    int64_t base = 2 * (int64_t)blockIdx.x;
    float xv = (base + half < ntiles && tid < 3 * kMT) ? g.X[(base + half) * kMT * 3 + tid] : 0.f;
    for (; base < ntiles; base += 2 * (int64_t)gridDim.x) {
        const int64_t tile = base + half;
        const bool live = tile < ntiles;
        const int64_t m0 = tile * kMT;
        const int64_t cloud = m0 / g.P;
        const int64_t rbase = m0 - cloud * g.P;
        for (int e = tid; e < kMT * 32; e += 256) {
            const int r = e / 32, k = e % 32;
            if (k >= 3) U[r * kLd1 + k] = 0;
        }
        if (tid < 3 * kMT) U[(tid / 3) * kLd1 + tid % 3] = to_bf16(xv);
        const int64_t next = tile + 2 * (int64_t)gridDim.x;
        if (next < ntiles && tid < 3 * kMT) xv = g.X[next * kMT * 3 + tid];
        __syncthreads();   // also orders the weight staging before the first tile
        // layer 1: wavefront w owns column block w, all four row blocks
        {
            const bf16x8_t b = lds_frag(W1s, 16 * wave + fr, kLd1, fk);
            const int col = 16 * wave + fr;
            const float bias = g.b1[col];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lds_frag(U, 16 * rb + fr, kLd1, fk), b, acc, 0, 0, 0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float v = fmaxf(acc[t] + bias, 0.f);
                    H1s[(16 * rb + 4 * (lane >> 4) + t) * kLd2 + col] = to_bf16(v);
                }
            }
        }
        __syncthreads();
        // layer 2: wavefront w owns column blocks 2w, 2w + 1
        {
            f32x4_t acc[4][2];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int c = 0; c < 2; ++c) acc[rb][c] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                bf16x8_t a[4], b[2];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) a[rb] = lds_frag(H1s, 16 * rb + fr, kLd2, 32 * ks + fk);
#pragma unroll
                for (int c = 0; c < 2; ++c) b[c] = lds_frag(W2s, 16 * (2 * wave + c) + fr, kLd2, 32 * ks + fk);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b[c], acc[rb][c], 0, 0, 0);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int col = 16 * (2 * wave + c) + fr;
                const float bias = g.b2[col];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float v = fmaxf(acc[rb][c][t] + bias, 0.f);
                        U[(16 * rb + 4 * (lane >> 4) + t) * kLd3 + col] = to_bf16(v);   // h2 replaces x
                    }
            }
        }
        __syncthreads();
        // layer 3: wavefront w owns column blocks 4w .. 4w + 3; then the
        // column maxima of the tile's 64 points go to the pool keys
        {
            f32x4_t acc[4][4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[rb][c] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                bf16x8_t a[4], b[4];
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) a[rb] = lds_frag(U, 16 * rb + fr, kLd3, 32 * ks + fk);
#pragma unroll
                for (int c = 0; c < 4; ++c) b[c] = lds_frag(W3s, 16 * (4 * wave + c) + fr, kLd3, 32 * ks + fk);
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b[c], acc[rb][c], 0, 0, 0);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = 16 * (4 * wave + c) + fr;
                const float bias = g.b3[col];
                unsigned long long best = 0ull;
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float v = acc[rb][c][t] + bias;
                        const float r = v > 0.f ? v : 0.f;
                        const uint32_t row = (uint32_t)(rbase + 16 * rb + 4 * (lane >> 4) + t);
                        const unsigned long long key =
                            ((unsigned long long)__float_as_uint(r) << 32) | (unsigned long long)(~row);
                        best = key > best ? key : best;
                    }
                unsigned long long o = __shfl_xor(best, 16);
                best = o > best ? o : best;
                o = __shfl_xor(best, 32);
                best = o > best ? o : best;
                if (live && lane < 16) atomicMax(g.keys + cloud * 256 + col, best);
            }
        }
        __syncthreads();   // the next tile overwrites U and H1s
    }
}

// C[m][n] (+)= sum_{z < S} W[z][m][n] (+ bias[n]) (ReLU), z in order.
__global__ void splitk_reduce_kernel(const float* __restrict__ W, int32_t S, int64_t M, int64_t N,
                                     float* __restrict__ C, int64_t ldc, const float* __restrict__ bias,
                                     int32_t relu, int32_t accumulate)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    const int64_t m = i / N, n = i % N;
    float s = 0.f;
    for (int32_t z = 0; z < S; ++z) s += W[(int64_t)z * M * N + i];
    if (bias) s += bias[n];
    if (relu) s = fmaxf(s, 0.f);
    float* dst = C + m * ldc + n;
    *dst = accumulate ? *dst + s : s;
}

// --------------------------------------------------------------- max-pool
// H holds `clouds` clouds of P points, F features each: row c P + p.
// Stage 1, grid (clouds, chunks): maximum and its first index over the
// chunk's points, per feature.
__global__ void maxpool_partial_kernel(const float* __restrict__ H, int64_t P, int64_t F, int64_t chunk,
                                       float* __restrict__ pv, int32_t* __restrict__ pi)
{
    const int64_t c = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
    const int64_t p0 = ch * chunk, p1 = min(P, p0 + chunk);
    for (int64_t f = threadIdx.x; f < F; f += blockDim.x) {
        float best = -__builtin_inff();
        int32_t bi = (int32_t)p0;
        for (int64_t p = p0; p < p1; ++p) {
            const float v = H[(c * P + p) * F + f];
            if (v > best) {
                best = v;
                bi = (int32_t)p;
            }
        }
        pv[(c * nch + ch) * F + f] = best;
        pi[(c * nch + ch) * F + f] = bi;
    }
}

// Stage 2, one thread per (cloud, feature): merge the chunks in order (the
// first maximum wins). Pair layout: clouds 2b (source) and 2b + 1
// (reference) fill columns [0, F) and [F, 2F) of row b of `out`.
__global__ void maxpool_merge_kernel(const float* __restrict__ pv, const int32_t* __restrict__ pi, int64_t clouds,
                                     int64_t nch, int64_t F, float* __restrict__ out, int64_t ld_out,
                                     int32_t* __restrict__ arg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= clouds * F) return;
    const int64_t c = i / F, f = i % F;
    float best = pv[(c * nch) * F + f];
    int32_t bi = pi[(c * nch) * F + f];
    for (int64_t ch = 1; ch < nch; ++ch) {
        const float v = pv[(c * nch + ch) * F + f];
        if (v > best) {
            best = v;
            bi = pi[(c * nch + ch) * F + f];
        }
    }
    out[(c / 2) * ld_out + (c % 2) * F + f] = best;
    arg[i] = bi;
}

// Keys of the pooled epilogue to the pooled features (pair layout as in
// maxpool_merge_kernel) and the winning rows. One thread per (cloud, feature).
__global__ void pool_keys_finish_kernel(const unsigned long long* __restrict__ keys, int64_t clouds, int64_t F,
                                        float* __restrict__ out, int64_t ld_out, int32_t* __restrict__ arg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= clouds * F) return;
    const int64_t c = i / F, f = i % F;
    const unsigned long long k = keys[i];
    out[(c / 2) * ld_out + (c % 2) * F + f] = __uint_as_float((uint32_t)(k >> 32));
    arg[i] = (int32_t)(~(uint32_t)k);
}

// Below the max-pool only the points that won a pooled feature receive
// gradient. winner_rows_kernel gives each cloud F3 rows: its distinct
// winning points first (in order of the first feature each wins), then zero
// rows. Row u holds the point's input (G0) and the pooled gradients of the
// features it wins (dA3[u][f] = dF[c][f] where F[c][f] > 0, else 0): the
// dense backward's nonzero rows, so every product below is the dense chain
// rule's product restricted to them (zero rows add exact zeros).
// grid: clouds; F3 threads, one per feature.
template <int F3>
__global__ __launch_bounds__(F3) void winner_rows_kernel(const float* __restrict__ X, const int32_t* __restrict__ arg,
                                                         const float* __restrict__ F, const float* __restrict__ dF,
                                                         int64_t ld_f, int64_t P, float* __restrict__ G0,
                                                         float* __restrict__ dA3)
{
    constexpr int kW = 64;   // wavefront width
    static_assert(F3 % kW == 0, "one thread per feature, whole wavefronts");
    __shared__ int32_t pt[F3];
    __shared__ int32_t row_of[F3];
    __shared__ int32_t wtot[F3 / kW];
    const int64_t c = blockIdx.x;
    const int f = threadIdx.x, lane = f % kW, wv = f / kW;
    const int32_t p = min(max(arg[c * F3 + f], 0), (int32_t)(P - 1));   // arg is in range; clamp anyway
    pt[f] = p;
    __syncthreads();
    int first = f;   // first feature won by the same point
    for (int j = 0; j < f; ++j)
        if (pt[j] == p) {
            first = j;
            break;
        }
    const bool owner = first == f;
    const unsigned long long ob = __ballot(owner);
    const int before = __popcll(ob & ((1ull << lane) - 1ull));
    if (lane == 0) wtot[wv] = __popcll(ob);
    __syncthreads();
    int r = before, rows = 0;
    for (int w = 0; w < F3 / kW; ++w) {
        r += w < wv ? wtot[w] : 0;
        rows += wtot[w];
    }
    if (owner) row_of[f] = r;
    float* __restrict__ Dc = dA3 + c * F3 * F3;
    for (int e = f; e < F3 * F3; e += F3) Dc[e] = 0.f;
    float* __restrict__ Gc = G0 + c * F3 * 3;
    if (owner) {
        const float* x = X + (c * P + p) * 3;
        Gc[3 * r] = x[0];
        Gc[3 * r + 1] = x[1];
        Gc[3 * r + 2] = x[2];
    }
    if (f >= rows) Gc[3 * f] = Gc[3 * f + 1] = Gc[3 * f + 2] = 0.f;
    __syncthreads();   // the zeros and row_of before the scatter
    const int64_t e = (c / 2) * ld_f + (c % 2) * F3 + f;
    Dc[(int64_t)row_of[first] * F3 + f] = F[e] > 0.f ? dF[e] : 0.f;
}

// ------------------------------------------------------------ elementwise
// dA = dH where H > 0, else 0 (in place; H is the ReLU output).
__global__ void relu_backward_kernel(const float* __restrict__ H, float* __restrict__ dH, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(H[i] > 0.f)) dH[i] = 0.f;
}

__global__ void fill_f32_kernel(float* __restrict__ x, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Column sums of X (rows x N) in two fixed-order stages: partial sums over
// row chunks (grid (ceil(N / 256), chunks)), then over chunks.
__global__ void colsum_partial_kernel(const float* __restrict__ X, int64_t rows, int64_t N, int64_t chunk,
                                      float* __restrict__ part)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
    float s = 0.f;
    for (int64_t r = r0; r < r1; ++r) s += X[r * N + n];
    part[(int64_t)blockIdx.y * N + n] = s;
}

__global__ void colsum_merge_kernel(const float* __restrict__ part, int64_t nch, int64_t N, float* __restrict__ out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int64_t c = 0; c < nch; ++c) s += part[c * N + n];
    out[n] = s;
}

// ------------------------------------------------------------- set loss
constexpr int kMaxLossScales = 4;
struct MmdScales {
    int32_t ns;
    double inv[kMaxLossScales][6];   // 1 / sigma per scale and coordinate
};

__device__ __forceinline__ double wrap_angle_diff(double t)
{
    constexpr double two_pi = 6.283185307179586476925286766559;
    return t - rint(t / two_pi) * two_pi;
}

// Multi-scale Gaussian kernel between particles u and v (6 coordinates;
// angle differences wrapped to [-pi, pi]) and, when du != nullptr, its
// gradient with respect to u.
__device__ __forceinline__ double mmd_k(const MmdScales& sc, const double* u, const double* v, double* du)
{
    double d[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) d[c] = c < 3 ? u[c] - v[c] : wrap_angle_diff(u[c] - v[c]);
    double k = 0.0;
    if (du)
#pragma unroll
        for (int c = 0; c < 6; ++c) du[c] = 0.0;
    for (int s = 0; s < sc.ns; ++s) {
        double q = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) q += (d[c] * sc.inv[s][c]) * (d[c] * sc.inv[s][c]);
        const double e = exp(-0.5 * q);
        k += e;
        if (du)
#pragma unroll
            for (int c = 0; c < 6; ++c) du[c] -= e * d[c] * sc.inv[s][c] * sc.inv[s][c];
    }
    return k;
}

// One workgroup per sample b: X[b] (K x 6, FP32 network output, or FP64 when
// Xd is given) against the target set Y[b] (FP64):
//   loss[b] = (1 / K^2) sum_ij [k(x_i, x_j) + k(y_i, y_j) - 2 k(x_i, y_j)]
// (the biased MMD^2 estimate) and, when dX != nullptr,
//   dX[b] = gscale * d loss[b] / d X[b]
//         = gscale (2 / K^2) sum_j [grad_u k(x_i, x_j) - grad_u k(x_i, y_j)].
// Thread t takes row i = t mod K and the j range of group t / K (G groups,
// G K <= 256); row sums of the groups are added in group order.
__global__ __launch_bounds__(256) void mmd_kernel(const float* __restrict__ Xf, const double* __restrict__ Xd,
                                                  const double* __restrict__ Y, int32_t K, MmdScales sc,
                                                  double gscale, float* __restrict__ dX, double* __restrict__ loss)
{
    extern __shared__ double sm[];   // X, Y (K x 6 each), then G x K x 6 gradient partials
    const int64_t b = blockIdx.x;
    const int G = max(1, 256 / K);
    double* x = sm;
    double* y = sm + 6 * K;
    double* gp = sm + 12 * K;
    for (int e = threadIdx.x; e < 6 * K; e += blockDim.x) {
        x[e] = Xd ? Xd[b * 6 * K + e] : (double)Xf[b * 6 * K + e];
        y[e] = Y[b * 6 * K + e];
    }
    __syncthreads();
    __shared__ double red[256];
    double part = 0.0;
    // rows beyond 256 / K groups are taken in further passes
    for (int base = 0; base < K; base += 256) {
        const int t = threadIdx.x;
        const int i = base + (K >= 256 ? t : t % K);
        const int grp = K >= 256 ? 0 : t / K;
        const bool live = (K >= 256 ? i < K : t < G * K);
        double g[6] = {0, 0, 0, 0, 0, 0}, du[6];
        if (live) {
            const int j0 = (int)((int64_t)K * grp / G), j1 = (int)((int64_t)K * (grp + 1) / G);
            for (int j = j0; j < j1; ++j) {
                const double kxx = mmd_k(sc, x + 6 * i, x + 6 * j, du);
#pragma unroll
                for (int c = 0; c < 6; ++c) g[c] += du[c];
                const double kxy = mmd_k(sc, x + 6 * i, y + 6 * j, du);
#pragma unroll
                for (int c = 0; c < 6; ++c) g[c] -= du[c];
                part += kxx + mmd_k(sc, y + 6 * i, y + 6 * j, nullptr) - 2.0 * kxy;
            }
            if (dX)
#pragma unroll
                for (int c = 0; c < 6; ++c) gp[((int64_t)grp * K + i) * 6 + c] = g[c];
        }
        if (K < 256) break;   // one pass covers every row when G K >= K
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[b] = red[0] / ((double)K * K);
    if (!dX) return;
    const double w = gscale * 2.0 / ((double)K * K);
    const int Gs = K >= 256 ? 1 : G;
    for (int e = threadIdx.x; e < 6 * K; e += blockDim.x) {
        double sum = 0.0;
        for (int q = 0; q < Gs; ++q) sum += gp[(int64_t)q * 6 * K + e];
        dX[b * 6 * K + e] = (float)(w * sum);
    }
}

// ------------------------------------------------------------- optimiser
// Adam on FP32 parameters, bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t
// (the moments are stored in FP32, the update is evaluated in FP64).
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, double lr, double b1, double b2, double eps,
                            double bc1, double bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mm = b1 * (double)m[i] + (1.0 - b1) * gi;
    const double vv = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
    m[i] = (float)mm;
    v[i] = (float)vv;
    w[i] = (float)((double)w[i] - lr * (mm / bc1) / (sqrt(vv / bc2) + eps));
}

// --------------------------------------------------------------- in / out
// Network output (FP32, pairs of `per` values) to particles (FP64);
// bad[i / per] = 1 where a value is not finite (bad cleared by the caller).
__global__ void output_particles_kernel(const float* __restrict__ Y, int64_t n, int64_t per, double* __restrict__ out,
                                        int32_t* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = Y[i];
    if (!isfinite(v)) bad[i / per] = 1;
    out[i] = (double)v;
}

__global__ void fill_i32_kernel(int32_t* __restrict__ x, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* __restrict__ x, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// Network input of one cloud: point p of P takes cloud point floor(p n / P)
// (each point once when n == P, evenly repeated when n < P).
__global__ void subsample_kernel(const float* __restrict__ xyz, int64_t n, int64_t P, float* __restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int64_t s = (p * n) / P;
    out[3 * p] = xyz[3 * s];
    out[3 * p + 1] = xyz[3 * s + 1];
    out[3 * p + 2] = xyz[3 * s + 2];
}

}  // namespace prop
}  // namespace sicp
