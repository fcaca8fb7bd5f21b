// Nearest neighbour (Eq. 1) with a matrix-core screen and an exact FP32
// rerank, in two formats: BF16 x 3 (below) and FP16 x 2 (further down, the
// faster; the same structure with one FP16 product per block).
//
// Screen: squared distances in the expanded form |q|^2 + |r|^2 - 2 q.r on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation. Both sides are centred on
// the pair's reference centroid c0, and every FP32 value is split into three
// BF16 parts (x = h + m + l, the usual BF16x3 decomposition), so each product
// keeps about 24 bits; 24 of 32 K slots are used, over two products of
// K = 16 accumulated in FP32:
//    k  0- 2: r_h  * -2 q_h      k  9-11: r_h * -2 q_l      k 18-20: |r|^2 (h, m, l) * 1
//    k  3- 5: r_h  * -2 q_m      k 12-14: r_l * -2 q_h      k 21-23: 1 * |q|^2 (h, m, l)
//    k  6- 8: r_m  * -2 q_h      k 15-17: r_m * -2 q_m      k 24-31: 0
// The references are the A operand (32 per block, pre-packed in the lane
// layout at init), the queries the B operand (32 per group, built once per
// wavefront). Lane l owns query l % 32 of each group and receives rows
// 8 i + 4 (l / 32) + 0..3 (i = 0..3) of each 32-reference block; it keeps
// only a key of the minimum of those sixteen values per block, or per two
// blocks (see the certificate below). The wide product gives each lane
// sixteen values to reduce per pair of matrix instructions (three-input
// minimums), where a 16 x 16 product gives four per instruction: the
// vector-ALU work per distance, which bounded a 16 x 16 screen, about
// halves.
//
// Rerank: the workgroup first finds each query's smallest key over its
// lanes; a lane whose best key, less the error margin, is within the margin
// of it (the lane holding it always is) recomputes the exact FP32 distance
// (the same operation sequence as the FP32 search) of its rows of its best
// key's blocks, keyed by the reference index; the two lanes of a query
// merge their (distance, index) keys. The FP32 search keys by 16-reference
// tile instead; both order by distance, then lowest index, so the chunk
// reduction is shared, and an index key needs no tile resolution
// downstream.
//
// Certificate: the result is the FP32 search's exact chunk minimum, ties
// included. Let S be the screened and F the FP32 distance of a reference.
// |S - F| <= eps = 52 u (|q_c| + R)^2 + 6.2 u F (u = 2^-24, R the pair's
// largest centred reference norm): the sum of 24 exact BF16 products whose
// magnitudes sum to at most (|q_c| + |r_c|)^2, the dropped BF16 cross terms
// and the FP32 norms, the FP32 centring, and the FP32 direct difference. The
// matrix core's order and rounding of its additions are not specified; the
// sum is bounded as if each of its additions lost up to one FP32 ulp of its
// partial sum (truncation as well as rounding to nearest), 2u of the
// magnitudes per addition, which measured errors on stress inputs stay well
// inside. Each lane keeps, per one or two consecutive blocks of its rows, a
// key: their minimum with its low significand bits replaced by the key's
// offset, and the smallest two keys; the smallest names the best blocks, the
// second bounds every other key's minimum from below to within 2^kb ulps
// (s2; for a lane that did not rerank, the best key bounds all of its
// blocks). After the workgroup merges its keys into the chunk minimum F_wg,
// a lane whose references outside its reranked blocks all satisfy F > F_wg
// (guaranteed when s2 - 60 u (|q_c| + R')^2 > F_wg (1 + 8 u) with
// R' = min(R, |q_c| + sqrt(F_wg)), as only references within sqrt(F_wg) of
// the query can win) has lost nothing; otherwise that lane's own rows
// of its wavefront's blocks are searched again in FP32 by the wavefront and
// folded into the chunk minimum. The result is the FP32 search's key, ties
// included.
#pragma once

#include "common.hpp"
#include "nn_bf16_launch.h"

namespace sicp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

// Round to nearest even BF16 (finite inputs), returned as bits.
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x = h + m + l with each part BF16 (each subtraction is exact in FP32).
__device__ __forceinline__ void split3(float x, uint16_t& h, uint16_t& m, uint16_t& l)
{
#pragma clang fp contract(off)
    h = bf16_bits(x);
    const float r1 = x - bf16_float(h);
    m = bf16_bits(r1);
    const float r2 = r1 - bf16_float(m);
    l = bf16_bits(r2);
}

constexpr uint16_t kBf16One = 0x3F80;
constexpr uint16_t kBf16Zero = 0;

// The two fragments of one side for the lane half h of a 32 x 32 x 16
// product pair: K slots 8 h .. 8 h + 7 (first product) and 16 + 8 h .. +7
// (second). `ref` selects the A (reference) or B (query) column of the slot
// table above.
__device__ __forceinline__ void slot_fragments(const float c[3], bool ref, int hh, u16x8_t& v0, u16x8_t& v1)
{
#pragma clang fp contract(off)
    uint16_t h[3], m[3], l[3], nh, nm, nl;
    for (int d = 0; d < 3; ++d) split3(c[d], h[d], m[d], l[d]);
    const float n = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
    split3(n, nh, nm, nl);
    uint16_t t[32];
    if (ref) {
        for (int d = 0; d < 3; ++d) {
            t[d] = h[d]; t[3 + d] = h[d]; t[6 + d] = m[d];
            t[9 + d] = h[d]; t[12 + d] = l[d]; t[15 + d] = m[d];
            t[21 + d] = kBf16One;
        }
        t[18] = nh; t[19] = nm; t[20] = nl;
    } else {
        // -2 x of a BF16 value is exact in FP32 and again a BF16 value
        auto m2 = [](uint16_t v) -> uint16_t { return bf16_bits(-2.0f * bf16_float(v)); };
        for (int d = 0; d < 3; ++d) {
            t[d] = m2(h[d]); t[3 + d] = m2(m[d]); t[6 + d] = m2(h[d]);
            t[9 + d] = m2(l[d]); t[12 + d] = m2(h[d]); t[15 + d] = m2(m[d]);
            t[18 + d] = kBf16One;
        }
        t[21] = nh; t[22] = nm; t[23] = nl;
    }
    for (int k = 24; k < 32; ++k) t[k] = kBf16Zero;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v0[k] = hh ? t[8 + k] : t[k];
        v1[k] = hh ? t[24 + k] : t[16 + k];
    }
}

// ---------------------------------------------------------------- FP16 x 2
// The second screen format. Centred coordinates are scaled by 2^sexp (exact:
// a power of two, chosen per pair so the largest centred reference norm R
// becomes at most 32) and split into two FP16 parts, x = h + m + rest with
// |m| <= 2^-11 |x| and |rest| <= 2^-22 |x| + 2^-25 (FP16 has an 11-bit
// significand, so two parts carry what BF16 needs three for). The norms take
// three FP16 parts. 15 of the 16 K slots of one 32 x 32 x 16 FP16 product:
//    k 0- 2: r_h * -2 q_h      k  9-11: |r|^2 (h, m, l) * 1
//    k 3- 5: r_h * -2 q_m      k 12-14: 1 * |q|^2 (h, m, l)
//    k 6- 8: r_m * -2 q_h      k 15: 0
// Error (scaled units, q' and r' the scaled centred points, u = 2^-24): the
// dropped cross parts m_q m_r, h_q rest_r, rest_q h_r, ... with the factor 2
// give at most 24.1 u |q'||r'| + 3.5 2^-25 (|q'| + |r'|); the norms' FP32
// rounding and split 3.1 u (|q'|^2 + |r'|^2) + 2^-24; the matrix core's sum
// of the exact products and its zero accumulator 32.1 u (|q'| + |r'|)^2 (up
// to one FP32 ulp of the partial sum lost per addition, as for the BF16
// screen); the centring 2.1 u (|q'| + |r'|)^2; the FP32 direct difference of
// the rerank 6.2 u (|q'| + |r'|)^2. All told
// |S - s^2 F| <= 50 u (|q'| + |r'|)^2 + 2^-22 (|q'| + |r'| + 1); the
// certificate uses 56 u in place of 50 u. A query whose scaled centred norm
// exceeds kF16QueryMax (its norm would leave FP16's comfortable range) is
// not screened: its lanes fail the certificate and search in FP32.
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

constexpr float kF16QueryMax = 200.0f;

__device__ __forceinline__ uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ __forceinline__ float f16_float(uint16_t v) { return (float)__builtin_bit_cast(_Float16, v); }

// x = h + m (+ rest) with h, m FP16 (the subtraction is exact in FP32).
__device__ __forceinline__ void split2_f16(float x, uint16_t& h, uint16_t& m)
{
#pragma clang fp contract(off)
    h = f16_bits(x);
    m = f16_bits(x - f16_float(h));
}

__device__ __forceinline__ void split3_f16(float x, uint16_t& h, uint16_t& m, uint16_t& l)
{
#pragma clang fp contract(off)
    h = f16_bits(x);
    const float r1 = x - f16_float(h);
    m = f16_bits(r1);
    l = f16_bits(r1 - f16_float(m));
}

// Scaled centred coordinates: c * 2^e (exact for |e| <= 60 on the FP32
// values the screen sees).
__device__ __forceinline__ void scale_coords(float c[3], int e)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = ldexpf(c[d], e);
}

// The FP16 fragment of one side for lane half hh: K slots 8 hh .. 8 hh + 7
// of the table above. c: scaled centred coordinates.
__device__ __forceinline__ void slot_fragment_f16(const float c[3], bool ref, int hh, u16x8_t& v)
{
#pragma clang fp contract(off)
    constexpr uint16_t kOne = 0x3C00, kZero = 0;
    uint16_t h[3], m[3], nh, nm, nl;
    for (int d = 0; d < 3; ++d) split2_f16(c[d], h[d], m[d]);
    const float n = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
    split3_f16(n, nh, nm, nl);
    uint16_t t[16];
    if (ref) {
        for (int d = 0; d < 3; ++d) {
            t[d] = h[d]; t[3 + d] = h[d]; t[6 + d] = m[d];
            t[12 + d] = kOne;
        }
        t[9] = nh; t[10] = nm; t[11] = nl;
    } else {
        // -2 x of an FP16 value is exact in FP32 and again an FP16 value
        auto m2 = [](uint16_t x) -> uint16_t { return f16_bits(-2.0f * f16_float(x)); };
        for (int d = 0; d < 3; ++d) {
            t[d] = m2(h[d]); t[3 + d] = m2(m[d]); t[6 + d] = m2(h[d]);
            t[9 + d] = kOne;
        }
        t[12] = nh; t[13] = nm; t[14] = nl;
    }
    t[15] = kZero;
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = hh ? t[8 + k] : t[k];
}

// Scale exponent of the FP16 screen for a largest centred norm R: the
// largest e with R 2^e <= 32 (R = f 2^x, f in [0.5, 1): e = 5 - x), within
// [-60, 60]; 0 for R = 0.
__host__ __device__ inline int f16_screen_exponent(float R)
{
    if (!(R > 0.0f) || !(R < 3.0e38f)) return 0;
    int x = 0;
    (void)frexpf(R, &x);
    const int e = 5 - x;
    return e < -60 ? -60 : (e > 60 ? 60 : e);
}

constexpr int kBlk = kRefPad;   // references per block of the screen (the A operand's 32 rows)

// Row of the 32-reference block held by output t (0..15) of a lane in half h
// (lane / 32) of the 32 x 32 product.
__device__ __forceinline__ int blk_row(int t, int h) { return 8 * (t >> 2) + 4 * h + (t & 3); }

// Phases of a block in its key (see the block loop of nn_bf16_item).
constexpr int kStart = 1, kEnd = 2, kBoth = 3;
template <int P>
struct PhaseT {
    static constexpr int value = P;
};

// grid (blocks of 32 references / 4, groups) x 256 threads, one wavefront
// per block: each lane's two A fragments (K slots 8 h .. 8 h + 7 and
// 16 + 8 h .. +7 of row lane % 32). A block takes 128 uint4: the 64 lanes'
// first fragments, then their second ones, so a wavefront reads each as
// one contiguous row. (The second fragments of lanes 32..63 hold K slots
// 24..31, which the queries' fragments zero.)
__global__ void pack_bf16_refs_kernel(const PairDesc* __restrict__ pairs, const float4* __restrict__ ref4,
                                      uint4* __restrict__ apack)
{
    const PairDesc pd = pairs[blockIdx.y];
    const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    if (blk >= pd.n_ref_pad / kBlk) return;
    const float4 r = ref4[pd.ref_off + blk * kBlk + (lane & 31)];
    float c[3];
    {
#pragma clang fp contract(off)
        c[0] = r.x - pd.c0[0];
        c[1] = r.y - pd.c0[1];
        c[2] = r.z - pd.c0[2];
    }
    u16x8_t v0, v1;
    slot_fragments(c, true, lane >> 5, v0, v1);
    uint4* out = apack + pd.apack_off + blk * 2 * kWave + lane;
    out[0] = __builtin_bit_cast(uint4, v0);
    out[kWave] = __builtin_bit_cast(uint4, v1);
}

// The FP16 screen's A fragments: one uint4 per lane, a block is the 64
// lanes' fragments in order (1 KB per 32 references).
__global__ void pack_f16_refs_kernel(const PairDesc* __restrict__ pairs, const float4* __restrict__ ref4,
                                     uint4* __restrict__ apack)
{
    const PairDesc pd = pairs[blockIdx.y];
    const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    if (blk >= pd.n_ref_pad / kBlk) return;
    const float4 r = ref4[pd.ref_off + blk * kBlk + (lane & 31)];
    float c[3];
    {
#pragma clang fp contract(off)
        c[0] = r.x - pd.c0[0];
        c[1] = r.y - pd.c0[1];
        c[2] = r.z - pd.c0[2];
    }
    scale_coords(c, pd.sexp);
    u16x8_t v;
    slot_fragment_f16(c, true, lane >> 5, v);
    if (blk * kBlk + (lane & 31) >= pd.n_ref) {
        // padding: no cross parts and the largest finite FP16 value in the
        // three norm slots, so S exceeds every real distance (scaled real
        // distances are below (kF16QueryMax + 32)^2 < 3 x 65504)
        constexpr uint16_t kMaxF16 = 0x7BFF;
        const int hh = lane >> 5;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int slot = 8 * hh + k;
            v[k] = (slot >= 9 && slot <= 11) ? kMaxF16 : (slot >= 12 && slot <= 14 ? (uint16_t)0x3C00 : (uint16_t)0);
        }
    }
    apack[pd.apack_off + blk * kWave + lane] = __builtin_bit_cast(uint4, v);
}

// Centre of the screen found on the device, for callers that hand the
// library no host copy of the cloud: c0[0..2] = the centroid of the n
// references (FP64 sums in a fixed order, rounded to FP32) and c0[3] an upper
// bound of the centred norms as the screen forms them (FP32 differences,
// FP64 norms), raised by 2^-20 relative and one FP32 step. The screen's
// answer does not depend on c0 (it is certified); its error bound needs
// c0[3] to bound every centred norm. One workgroup of kCentreThreads.
constexpr int kCentreThreads = 1024;
__global__ __launch_bounds__(kCentreThreads) void bf16_centre_kernel(PairDesc* __restrict__ pd,
                                                                     const float4* __restrict__ ref4, int64_t n)
{
    constexpr int WV = kCentreThreads / kWave;
    __shared__ double red[WV][3];
    __shared__ float c0s[3];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = tid; i < n; i += kCentreThreads) {
        const float4 r = ref4[i];
        acc[0] += r.x;
        acc[1] += r.y;
        acc[2] += r.z;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) acc[d] += __shfl_xor(acc[d], o);
        if (lane == 0) red[wv][d] = acc[d];
    }
    __syncthreads();
    if (tid < 3) {
        double sum = 0.0;
        for (int w = 0; w < WV; ++w) sum += red[w][tid];
        const double mean = sum / (double)n;
        c0s[tid] = isfinite(mean) ? (float)mean : 0.0f;
    }
    __syncthreads();
    const float cx = c0s[0], cy = c0s[1], cz = c0s[2];
    double r2 = 0.0;
    for (int64_t i = tid; i < n; i += kCentreThreads) {
        const float4 r = ref4[i];
        float dx, dy, dz;
        {
#pragma clang fp contract(off)
            dx = r.x - cx;
            dy = r.y - cy;
            dz = r.z - cz;
        }
        r2 = fmax(r2, ((double)dx * dx + (double)dy * dy) + (double)dz * dz);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o));
    if (lane == 0) red[wv][0] = r2;
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int w = 0; w < WV; ++w) m = fmax(m, red[w][0]);
        pd->c0[0] = cx;
        pd->c0[1] = cy;
        pd->c0[2] = cz;
        pd->c0[3] = nextafterf((float)(sqrt(m) * (1.0 + 0x1.0p-20)), __builtin_inff());
        pd->sexp = f16_screen_exponent(pd->c0[3]);
    }
}

// A work item holds 64 Q queries (as in the FP32 search), taken as 2 Q groups
// of 32 by every wavefront of the workgroup. SPAN: blocks per key (1 or 2).
template <int Q, int W, int FMT, int SPAN>
__device__ __forceinline__ void nn_bf16_item(const NNBf16Args& a, const WorkItem w, uint64_t (*sk)[kWave * Q],
                                             float (*sm)[kWave * Q])
{
    constexpr bool F16 = FMT == kFmtF16x2;
    constexpr int G = 2 * Q;   // query groups of 32
    const PairDesc pd = a.pairs[w.pair];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = uniform(threadIdx.x >> 6);
    const int64_t nq = pd.nq;
    const int64_t qbase = (int64_t)w.qblock * kWave * Q;
    const int j = lane & 31, h = lane >> 5;

    bf16x8_t b0[G], b1[G];   // BF16 x 3
    f16x8_t e0[G];           // FP16 x 2
    uint32_t far_q = 0u;     // FP16 x 2: groups whose query lies beyond kF16QueryMax (not screened)
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t qi = qbase + 32 * g + j;
        const float4 qf = qi < nq ? a.queries[pd.q_off + qi] : make_float4(0.f, 0.f, 0.f, 0.f);
        float c[3];
        {
#pragma clang fp contract(off)
            c[0] = qf.x - pd.c0[0];
            c[1] = qf.y - pd.c0[1];
            c[2] = qf.z - pd.c0[2];
        }
        if constexpr (F16) {
            scale_coords(c, pd.sexp);
            const bool far = !(fabsf(c[0]) <= kF16QueryMax && fabsf(c[1]) <= kF16QueryMax &&
                               fabsf(c[2]) <= kF16QueryMax &&
                               (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2] <= kF16QueryMax * kF16QueryMax);
            if (far) {
                c[0] = c[1] = c[2] = 0.0f;   // finite fragments; the lane searches in FP32 instead
                far_q |= 1u << g;
            }
            u16x8_t v;
            slot_fragment_f16(c, false, h, v);
            e0[g] = __builtin_bit_cast(f16x8_t, v);
        } else {
            u16x8_t v0, v1;
            slot_fragments(c, false, h, v0, v1);
            b0[g] = __builtin_bit_cast(bf16x8_t, v0);
            b1[g] = __builtin_bit_cast(bf16x8_t, v1);
        }
    }

    const int64_t c0 = (int64_t)w.chunk * pd.chunk;
    const int64_t cend = min(c0 + (int64_t)pd.chunk, pd.n_ref_pad);
    // the wavefront's block range [t0, t1) of the chunk (wave-uniform)
    const int32_t nblk = (int32_t)((cend - c0) / kBlk);
    const int32_t t0 = uniform((int32_t)(((int64_t)nblk * wave) / W));
    const int32_t t1 = uniform((int32_t)(((int64_t)nblk * (wave + 1)) / W));
    // fragments of a block: BF16 x 3 two uint4 per lane (2 kWave per block),
    // FP16 x 2 one (kWave per block)
    constexpr int kStride = F16 ? kWave : 2 * kWave;
    const uint4* __restrict__ ap0 = a.apack + pd.apack_off + (c0 / kBlk) * kStride + lane;
    const uint4* __restrict__ ap1 = a.apack + pd.apack_off + (c0 / kBlk) * kStride + kWave + j;

    // Block keys: the minimum of kSB consecutive blocks (one or two), its
    // FP32 bits with the low kb bits replaced by the key's offset in the
    // wavefront's range. A key is a finite float within 2^kb ulps of the
    // minimum it stands for, so float comparisons order keys by their minima
    // (to that resolution) and the best key names its blocks: no
    // compare-and-select per block. Two blocks per key save 1.5 vector
    // instructions per block and group (one key update per two blocks) and
    // double the rerank.
    constexpr int kSB = SPAN;
    const int32_t nkeys = (t1 - t0 + kSB - 1) / kSB;
    const int kb = uniform(nkeys > 1 ? 32 - __builtin_clz((uint32_t)(nkeys - 1)) : 0);
    const uint32_t kmask = ~((1u << kb) - 1u);
    // the mask held in a vector register: a three-operand instruction reads
    // at most one scalar, the block offset, so the key takes one and-or
    const uint32_t vmask = (uint32_t)__builtin_amdgcn_mov_dpp((int)kmask, 0xE4, 0xF, 0xF, false);
    float best[G], sec[G];   // smallest block key, and the smallest of the other blocks' keys
    float carry[G];          // minimum over the earlier blocks of the current key
#pragma unroll
    for (int g = 0; g < G; ++g) {
        best[g] = __builtin_inff();
        sec[g] = __builtin_inff();
        carry[g] = __builtin_inff();
    }
    const auto products = [&](const uint4& f0, const uint4& f1, f32x16_t (&acc)[G]) {
        if constexpr (F16) {
            const f16x8_t a0 = __builtin_bit_cast(f16x8_t, f0);
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int t = 0; t < 16; ++t) acc[g][t] = 0.f;
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, e0[g], acc[g], 0, 0, 0);
            }
        } else {
            const bf16x8_t a0 = __builtin_bit_cast(bf16x8_t, f0);
            const bf16x8_t a1 = __builtin_bit_cast(bf16x8_t, f1);
#pragma unroll
            for (int g = 0; g < G; ++g) {
#pragma unroll
                for (int t = 0; t < 16; ++t) acc[g][t] = 0.f;
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0[g], acc[g], 0, 0, 0);
            }
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1[g], acc[g], 0, 0, 0);
        }
    };
    // the minimum of the lane's sixteen values of block blk, and with the
    // key's last block the key; the new second smallest key is the median of
    // (best, sec, key) as best <= sec. phase: kStart a key's first block
    // (its minimum kept in carry), kEnd its last, kBoth a key of one block
    // (the loops below follow the parity of the block offset statically)
    const auto take_min = [&](const f32x16_t (&acc)[G], int32_t blk, auto phase) {
        constexpr int P = kSB == 1 ? kBoth : decltype(phase)::value;
        const uint32_t off = (uint32_t)(blk - t0) / kSB;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            float mn;
            if constexpr (P == kEnd) mn = __builtin_fminf(__builtin_fminf(carry[g], acc[g][0]), acc[g][1]);
            else mn = __builtin_fminf(acc[g][0], acc[g][1]);
#pragma unroll
            for (int t = 2; t < 16; t += 2) mn = __builtin_fminf(__builtin_fminf(mn, acc[g][t]), acc[g][t + 1]);
            if constexpr (P == kStart) {
                carry[g] = mn;
            } else {
                const float key = __uint_as_float((__float_as_uint(mn) & vmask) | off);
                sec[g] = __builtin_amdgcn_fmed3f(best[g], sec[g], key);
                best[g] = __builtin_fminf(best[g], key);
            }
        }
    };
    const PhaseT<kStart> S_;
    const PhaseT<kEnd> E_;
    const PhaseT<kBoth> B_;
    // fragments of block blk, clamped into the range (loads past its end
    // re-read its last block). The second fragment of lane l + 32 meets
    // the queries' zero K slots 24..31, so it is read from lane l's
    // (finite BF16 values, products exactly zero): the wavefront's second
    // load touches 512 bytes instead of 1 KB.
    const auto frag = [&](int32_t blk, uint4& f0, uint4& f1) {
        const int32_t b = min(blk, t1 - 1);
        f0 = ap0[(int64_t)b * kStride];
        if constexpr (F16) f1 = f0;   // unused
        else f1 = ap1[(int64_t)b * kStride];
    };
    if constexpr (G >= 4 && F16) {
        // The pipeline below with four fragment buffers (FP16 x 2 fragments
        // take one uint4, so the buffers fit in 256 registers): each refill
        // takes the block four ahead, four blocks of load latency.
        if (t0 < t1) {
            uint4 fa0, fa1, fb0, fb1, fc0, fc1, fd0, fd1;
            f32x16_t accp[G], accc[G];
            frag(t0, fa0, fa1);
            frag(t0 + 1, fb0, fb1);
            frag(t0 + 2, fc0, fc1);
            frag(t0 + 3, fd0, fd1);
            products(fa0, fa1, accp);   // block t0
            frag(t0 + 4, fa0, fa1);
            int32_t b = t0 + 1;
            // fb, fc, fd, fa hold blocks b .. b + 3 at the top of every trip
            for (; b + 3 < t1; b += 4) {
                products(fb0, fb1, accc);   // block b
                frag(b + 4, fb0, fb1);
                take_min(accp, b - 1, S_);
                __builtin_amdgcn_sched_barrier(0);
                products(fc0, fc1, accp);   // block b + 1
                frag(b + 5, fc0, fc1);
                take_min(accc, b, E_);
                __builtin_amdgcn_sched_barrier(0);
                products(fd0, fd1, accc);   // block b + 2
                frag(b + 6, fd0, fd1);
                take_min(accp, b + 1, S_);
                __builtin_amdgcn_sched_barrier(0);
                products(fa0, fa1, accp);   // block b + 3
                frag(b + 7, fa0, fa1);
                take_min(accc, b + 2, E_);
                __builtin_amdgcn_sched_barrier(0);
            }
            // zero to three blocks remain; accp holds block b - 1
            if (b < t1) {
                products(fb0, fb1, accc);
                take_min(accp, b - 1, S_);
                if (b + 1 < t1) {
                    products(fc0, fc1, accp);
                    take_min(accc, b, E_);
                    if (b + 2 < t1) {
                        products(fd0, fd1, accc);
                        take_min(accp, b + 1, S_);
                        take_min(accc, b + 2, E_);
                    } else {
                        take_min(accp, b + 1, B_);
                    }
                } else {
                    take_min(accc, b, E_);
                }
            } else {
                take_min(accp, b - 1, B_);
            }
        }
    } else if constexpr (G >= 4) {
        // Software pipeline: the products of block b are issued before the
        // minimum of block b - 1 is taken, so the matrix pipeline and the
        // vector ALU work on different blocks (two accumulator sets); two
        // fragment buffers keep the next blocks' loads in flight.
        if (t0 < t1) {
            uint4 fa0, fa1, fb0, fb1;
            f32x16_t accp[G], accc[G];
            frag(t0, fa0, fa1);
            frag(t0 + 1, fb0, fb1);
            products(fa0, fa1, accp);   // block t0
            frag(t0 + 2, fa0, fa1);
            int32_t b = t0 + 1;
            // fb holds block b and fa block b + 1 at the top of every trip
            for (; b + 1 < t1; b += 2) {
                // (the scheduling barriers keep each refill in the half
                // trip that consumed its buffer: two blocks of latency)
                products(fb0, fb1, accc);   // block b
                frag(b + 2, fb0, fb1);
                take_min(accp, b - 1, S_);
                __builtin_amdgcn_sched_barrier(0);
                products(fa0, fa1, accp);   // block b + 1
                frag(b + 3, fa0, fa1);
                take_min(accc, b, E_);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (b < t1) {
                products(fb0, fb1, accc);   // block b = t1 - 1
                take_min(accp, b - 1, S_);
                take_min(accc, b, E_);
            } else {
                take_min(accp, b - 1, B_);
            }
        }
    } else {
        // one accumulator set (fewer registers: four wavefronts per SIMD
        // fit); two fragment buffers, each refilled with the block two ahead
        // as soon as its products are issued
        if (t0 < t1) {
            uint4 fa0, fa1, fb0, fb1;
            f32x16_t acc[G];
            frag(t0, fa0, fa1);
            frag(t0 + 1, fb0, fb1);
            int32_t b = t0;
            for (; b + 1 < t1; b += 2) {
                products(fa0, fa1, acc);   // block b
                frag(b + 2, fa0, fa1);
                take_min(acc, b, S_);
                __builtin_amdgcn_sched_barrier(0);
                products(fb0, fb1, acc);   // block b + 1
                frag(b + 3, fb0, fb1);
                take_min(acc, b + 1, E_);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (b < t1) {
                products(fa0, fa1, acc);   // block b = t1 - 1
                take_min(acc, b, B_);
            }
        }
    }

    constexpr double u = 0x1.0p-24;
    // The screen's error margin for a query of centred norm qn whose chunk
    // minimum is fw (an FP32 squared distance), in the screen's units. A
    // reference that could match or beat fw lies within sqrt(fw) of the
    // query, so its centred norm is at most qn + sqrt(fw) (triangle
    // inequality; the 2^-20 slack covers the rounding of the centring and
    // of the FP32 distance): that norm, when below R, bounds the error.
    const auto margin_of = [&](double qn, double fw) {
        const double rmax = fmin((double)pd.c0[3], qn + sqrt(fw));
        const double span = (qn + rmax) * (1.0 + 0x1.0p-20);
        if constexpr (F16) {
            // in scaled units: S and the bound carry 4^sexp, the absolute
            // term of the bound is added there
            const double sp = ldexp(span, pd.sexp);
            return 56.0 * u * sp * sp + 0x1.0p-22 * (sp + 1.0);
        } else {
            return 60.0 * u * span * span;
        }
    };
    const double unit2 = F16 ? ldexp(1.0, 2 * pd.sexp) : 1.0;   // screen units per squared input unit
    // every block minimum a key stands for is at least the key less its
    // 2^kb ulps (no bound when the offsets would take most of the
    // significand: every lane is then searched again)
    const auto lower = [&](float key) {
        const double d = key;
        return kb > 20 ? -HUGE_VAL : isinf(d) ? d : d - ldexp(fabs(d), kb - 22);
    };
    // (the queries are loaded again rather than kept from the prologue: the
    // pointer is passed through an empty asm statement so that the compiler
    // does not carry them through the block loop in registers)
    const float4* qsrc = a.queries + pd.q_off;
    asm volatile("" : "+v"(qsrc));
    float4 qv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t qi = qbase + 32 * g + j;
        qv[g] = qi < nq ? qsrc[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // centred norm of a query (recomputed where needed: registers are short)
    const auto qnorm = [&](const float4& q) {
        float c[3];
        {
#pragma clang fp contract(off)
            c[0] = q.x - pd.c0[0];
            c[1] = q.y - pd.c0[1];
            c[2] = q.z - pd.c0[2];
        }
        return sqrt((double)c[0] * c[0] + (double)c[1] * c[1] + (double)c[2] * c[2]);
    };

    // The smallest key of each query over the workgroup's lanes. Only a lane
    // whose best blocks could hold the query's chunk minimum reranks it: one
    // whose key, less the margin, is within the margin of that smallest key
    // (the lane holding it always does). The others certify all of their
    // blocks, the best included, from their best key below.
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float m = fminf(best[g], __shfl_xor(best[g], 32));
        if (h == 0) sm[wave][32 * g + j] = m;
    }
    __syncthreads();
    for (int jj = threadIdx.x; jj < kWave * Q; jj += kWave * W) {
        float m0 = sm[0][jj];
#pragma unroll
        for (int v = 1; v < W; ++v) m0 = fminf(m0, sm[v][jj]);
        sm[0][jj] = m0;
    }
    __syncthreads();
    uint32_t rerank = 0u;   // groups whose best blocks this lane reranks
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float m = sm[0][32 * g + j];
        const int64_t qi = qbase + 32 * g + j;
        const bool far = F16 && ((far_q >> g) & 1u) != 0u;   // searched again in FP32 below
        if (qi < nq && t0 < t1 && !far) {
            const double hi = (double)m + ldexp(fabs((double)m), kb - 22);   // the smallest block minimum, from above
            const double marg = margin_of(qnorm(qv[g]), fmax(hi, 0.0) / unit2 * (1.0 + 0x1.0p-10));
            if (!(lower(best[g]) - marg > (hi + marg) * (1.0 + 8.0 * u))) rerank |= 1u << g;
        }
    }

    // exact FP32 rerank of the lane's rows of its best key's blocks (16 kSB
    // references, keyed by the reference index), then the minimum over the
    // two lanes of each query
    const float4* __restrict__ rp = a.ref4 + pd.ref_off + c0;
    uint64_t key[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float4 qf = qv[g];
        const int32_t bblk = min(t0 + kSB * (int32_t)(__float_as_uint(best[g]) & ~kmask), t1 - 1);
        uint64_t k = ~0ull;
        if ((rerank >> g) & 1u) {
#pragma unroll 4
            for (int t = 0; t < 16 * kSB; ++t) {
                const int64_t r = (int64_t)min(bblk + (t >> 4), t1 - 1) * kBlk + blk_row(t & 15, h);
                const float4 rr = rp[r];
                k = min(k, pack_key(dist2_f32(qf.x, qf.y, qf.z, rr.x, rr.y, rr.z), (uint32_t)(c0 + r)));
            }
        }
        k = min(k, (uint64_t)__shfl_xor((unsigned long long)k, 32));
        key[g] = k;
    }

    // lanes 0..31 hold the merged keys of the G groups; merge the W waves
    // into the chunk minimum of each query (kept in sk[0])
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (h == 0) sk[wave][32 * g + j] = key[g];
    __syncthreads();
    for (int jj = threadIdx.x; jj < kWave * Q; jj += kWave * W) {
        uint64_t k0 = sk[0][jj];
#pragma unroll
        for (int v = 1; v < W; ++v) k0 = min(k0, sk[v][jj]);
        sk[0][jj] = k0;
    }
    __syncthreads();
    // certificate of every lane against the chunk minimum; a lane that fails
    // has its own rows of its own blocks (16 (t1 - t0) references) searched
    // again in FP32 by its wavefront, folded into the chunk minimum in LDS
    if (t0 < t1) {
        // gathers kept in flight together (one query per lane: the
        // unrolled loop's registers would cost occupancy; measured best:
        // eight for FP16 x 2, four for BF16 x 3)
        constexpr int kRescanUnroll = Q == 1 ? 1 : (F16 ? 8 : 4);
        const int32_t ntrip = (t1 - t0 + 3) >> 2;   // four blocks per trip
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t qi = qbase + 32 * g + j;
            bool fail = false;
            if (qi < nq) {
                const float fwg = __uint_as_float((uint32_t)(sk[0][32 * g + j] >> 32));
                // a reranked lane's other blocks are bounded by its second
                // key, a lane that did not rerank has all of them bounded by
                // its best key
                const double s2 = lower(((rerank >> g) & 1u) ? sec[g] : best[g]);
                const bool far = F16 && ((far_q >> g) & 1u) != 0u;
                fail = far || !(s2 - margin_of(qnorm(qv[g]), (double)fwg) > (double)fwg * unit2 * (1.0 + 8.0 * u));
            }
            unsigned long long mask = __ballot(fail);
            if (mask != 0ull && a.rescans != nullptr && lane == 0)
                atomicAdd(a.rescans, (unsigned long long)__popcll(mask));
            while (mask != 0ull) {   // wave-uniform
                const int b = __ffsll((long long)mask) - 1;
                mask &= mask - 1ull;
                const int fj = b & 31, fh = b >> 5;
                const float4 qf = a.queries[pd.q_off + qbase + 32 * g + fj];
                // lane l takes row blk_row(l % 16, fh) of blocks t0 + l / 16,
                // t0 + l / 16 + 4, ...: a fixed row per lane, the wavefront
                // four blocks per trip; past the range a lane reads the
                // range's last block again (a duplicate leaves the minimum
                // unchanged), so the gathers carry no branch
                const int32_t lb = t0 + (lane >> 4);
                const int64_t rrow = c0 + blk_row(lane & 15, fh);
                const float4* __restrict__ rq = a.ref4 + pd.ref_off + rrow;
                uint64_t kr = ~0ull;
#pragma unroll kRescanUnroll
                for (int32_t it = 0; it < ntrip; ++it) {
                    const int64_t bo = (int64_t)min(lb + 4 * it, t1 - 1) * kBlk;
                    const float4 rr = rq[bo];
                    kr = min(kr, pack_key(dist2_f32(qf.x, qf.y, qf.z, rr.x, rr.y, rr.z), (uint32_t)(rrow + bo)));
                }
#pragma unroll
                for (int o = kWave / 2; o > 0; o >>= 1) kr = min(kr, (uint64_t)__shfl_xor((unsigned long long)kr, o));
                if (lane == 0) atomicMin((unsigned long long*)&sk[0][32 * g + fj], (unsigned long long)kr);
            }
        }
    }
    __syncthreads();
    for (int jj = threadIdx.x; jj < kWave * Q; jj += kWave * W) {
        const int64_t qi = qbase + jj;
        if (qi < nq) a.partial[pd.part_off + (int64_t)w.chunk * nq + qi] = sk[0][jj];
    }
    __syncthreads();
}

// The raw screened values |q|^2 + |r|^2 - 2 q.r of a screen, in the
// units of the input (FP16 x 2: divided by 4^sexp, exactly), for checking
// its error bound: the same fragments and matrix products as the screen.
// grid (reference blocks of 32, query groups of 32), one wavefront each.
// values: nq x n_ref row-major; NaN for a query the FP16 screen does not
// screen (beyond kF16QueryMax after scaling).
template <int FMT>
__global__ __launch_bounds__(kWave) void screen_values_kernel(const PairDesc* __restrict__ pairs,
                                                              const uint4* __restrict__ apack,
                                                              const float4* __restrict__ queries, int64_t nq,
                                                              float* __restrict__ values)
{
    constexpr bool F16 = FMT == kFmtF16x2;
    const PairDesc pd = pairs[0];
    const int lane = threadIdx.x, j = lane & 31, h = lane >> 5;
    const int64_t blk = blockIdx.x;
    const int64_t qi = (int64_t)blockIdx.y * 32 + j;
    const float4 qf = qi < nq ? queries[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
    float c[3];
    {
#pragma clang fp contract(off)
        c[0] = qf.x - pd.c0[0];
        c[1] = qf.y - pd.c0[1];
        c[2] = qf.z - pd.c0[2];
    }
    f32x16_t acc;
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = 0.f;
    bool far = false;
    if constexpr (F16) {
        scale_coords(c, pd.sexp);
        far = !(fabsf(c[0]) <= kF16QueryMax && fabsf(c[1]) <= kF16QueryMax && fabsf(c[2]) <= kF16QueryMax &&
                (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2] <= kF16QueryMax * kF16QueryMax);
        if (far) c[0] = c[1] = c[2] = 0.0f;
        u16x8_t v;
        slot_fragment_f16(c, false, h, v);
        const uint4 f0 = apack[pd.apack_off + blk * kWave + lane];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, f0), __builtin_bit_cast(f16x8_t, v),
                                                     acc, 0, 0, 0);
    } else {
        u16x8_t v0, v1;
        slot_fragments(c, false, h, v0, v1);
        const uint4 f0 = apack[pd.apack_off + blk * 2 * kWave + lane];
        const uint4 f1 = apack[pd.apack_off + blk * 2 * kWave + kWave + j];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, f0), __builtin_bit_cast(bf16x8_t, v0),
                                                      acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, f1), __builtin_bit_cast(bf16x8_t, v1),
                                                      acc, 0, 0, 0);
    }
    if (qi >= nq) return;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int64_t r = blk * kBlk + blk_row(t, h);
        if (r < pd.n_ref) {
            const float x = F16 ? ldexpf(acc[t], -2 * pd.sexp) : acc[t];
            // the quiet NaN goes out as its bit pattern: this file is built
            // with NaNs assumed away
            reinterpret_cast<uint32_t*>(values)[qi * pd.n_ref + r] = far ? 0x7fc00000u : __float_as_uint(x);
        }
    }
}

// Two queries per lane: at least two wavefronts per SIMD (at most 256
// registers), so workgroups of four wavefronts run two to a compute unit;
// one query per lane: four per SIMD.
// BW: the launch may carry bandwidth workgroups (a separate instantiation,
// so launches without them run the search's code alone).
template <int Q, int W, int FMT, bool BW, int SPAN>
__global__ __launch_bounds__(kWave * W, Q == 1 ? 4 : 2) void nn_bf16_kernel(NNBf16Args a)
{
    __shared__ uint64_t sk[W][kWave * Q];
    __shared__ float sm[W][kWave * Q];
    if (BW && (int)blockIdx.x < a.bw_blocks) {
        extern __shared__ double bw_lds[];
        bandwidth_role<kWave * W>(a.bw, blockIdx.x, a.bw_form, bw_lds);
        return;
    }
    for (int64_t it = blockIdx.x - a.bw_blocks; it < a.nwork; it += gridDim.x - a.bw_blocks)
        nn_bf16_item<Q, W, FMT, SPAN>(a, a.work[it], sk, sm);
}

}  // namespace sicp
