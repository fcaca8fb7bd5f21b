// Host launchers of the BF16-screen nearest-neighbour kernels, compiled in
// their own translation unit (nn_bf16.hip) with IEEE mode off: the screen's
// minimum over matrix-core outputs then needs no NaN canonicalisation.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace sicp {

struct NNBf16Args {
    const WorkItem* work;
    const PairDesc* pairs;
    const float4* ref4;
    const uint4* apack;
    const float4* queries;
    uint64_t* partial;
    int64_t nwork;
    unsigned long long* rescans;   // if set: certificates that failed, accumulated
};

// Shapes the screen is built for: q queries per lane (1 or 2) and w
// wavefronts per workgroup (4, 8, 16 for one query per lane; 4, 8 for two).
bool nn_bf16_shape_ok(int q, int w);

// q, w as above, grid workgroups (grid < nwork makes them persistent).
hipError_t launch_nn_bf16_kernel(int q, int w, unsigned grid, const NNBf16Args& a, hipStream_t s);

// The screen's centre c0 of one pair from its n_ref packed references, on
// the device (written into pair->c0).
hipError_t launch_bf16_centre(PairDesc* pair, const float4* ref4, int64_t n_ref, hipStream_t s);

// A fragments of the centred references of every pair; grid covers the
// largest pair's 16-reference blocks.
hipError_t launch_pack_bf16(const PairDesc* pairs, int32_t n_pairs, int64_t max_blocks, const float4* ref4,
                            uint4* apack, hipStream_t s);

}  // namespace sicp
