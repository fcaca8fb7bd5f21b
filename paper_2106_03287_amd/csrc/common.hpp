// Layouts and small device helpers shared by the Stein-ICP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sicp {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kTile = 16;            // references per tile of the NN scan (and of a key's tile index)
constexpr int kRefPad = 32;          // references are padded to a multiple of this (the BF16 screen's block)
constexpr float kPadCoord = 1e18f;   // coordinate of padding references
constexpr int kMaxK = 1024;          // particles per pair (one workgroup)
constexpr int kSvgdThreads = 1024;   // threads of the per-pair SVGD workgroup
constexpr int kGradThreads = 512;    // threads per particle in the gradient launch

// One cloud pair inside a (possibly batched) context. Offsets are in
// elements of the packed arrays they index.
struct PairDesc {
    int64_t src_off;    // into src4 (float4 per point)
    int64_t ref_off;    // into ref4
    int64_t n_src;
    int64_t n_ref;      // real references
    int64_t n_ref_pad;  // padded to a multiple of kRefPad with far-away points
    int64_t sched_off;  // into the int32 schedule (rows x m)
    int64_t part_off;   // into the uint64 partial-argmin buffer (chunks x K*m)
    int64_t n_scale;    // N in "N gbar"
    int64_t q_off;      // into the float4 query buffer
    int64_t nq;         // queries of this pair (K * m in a solver context)
    int64_t apack_off;  // into the BF16 reference fragments (4 uint4 per reference)
    int64_t part_stride;  // distance between a query's chunk keys (queries of its NN group)
    float c0[4];        // reference centroid (centres the BF16 screen)
    int32_t chunks;     // reference chunks, one partial argmin each
    int32_t chunk;      // references per chunk (multiple of kRefPad)
    int32_t qblocks;    // query blocks of kWave * Q queries
    int32_t sexp;       // FP16 screen: centred coordinates are scaled by 2^sexp
};

// Work item of the NN kernel: NN group, query block, reference chunk. An NN
// group is a run of consecutive pairs on one packed reference (often a
// single pair); the search treats its queries as one set.
struct WorkItem {
    int32_t pair, qblock, chunk, pad_;
};

// Per-particle pose data recomputed after every update (FP64):
// R (row-major 3x3), u (translation), dR/droll, dR/dpitch, dR/dyaw.
struct Pose {
    double R[9];
    double u[3];
    double dR[27];
    double pad_;
};

// Packed (squared distance, index) key: a non-negative FP32 distance orders
// like its bit pattern, so the unsigned minimum of the key is the smallest
// distance and, among equal distances, the lowest index.
__device__ __forceinline__ uint64_t pack_key(float d2, uint32_t idx)
{
    return (static_cast<uint64_t>(__float_as_uint(d2)) << 32) | idx;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// FP32 squared distance, fixed operation order (the NN decision).
__device__ __forceinline__ float dist2_f32(float qx, float qy, float qz, float rx, float ry, float rz)
{
#pragma clang fp contract(off)
    const float dx = qx - rx;
    const float dy = qy - ry;
    const float dz = qz - rz;
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// s' = R s + u in FP64, each product and sum rounded (no contraction).
__device__ __forceinline__ void transform_f64(const double* __restrict__ R, const double* __restrict__ u,
                                              double s0, double s1, double s2, double q[3])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = ((R[3 * r] * s0 + R[3 * r + 1] * s1) + R[3 * r + 2] * s2) + u[r];
}

}  // namespace sicp
