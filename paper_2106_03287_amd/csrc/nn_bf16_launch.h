// Host launchers of the BF16-screen nearest-neighbour kernels, compiled in
// their own translation unit (nn_bf16.hip) with IEEE mode off: the screen's
// minimum over matrix-core outputs then needs no NaN canonicalisation.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "svgd_select.hpp"

namespace sicp {

// Screen formats: three BF16 parts, two 32 x 32 x 16 products per block of
// 32 references; or two FP16 parts of scaled coordinates, one product.
constexpr int kFmtBf16x3 = 0;
constexpr int kFmtF16x2 = 1;

struct NNBf16Args {
    const WorkItem* work;
    const PairDesc* pairs;
    const float4* ref4;
    const uint4* apack;
    const float4* queries;
    uint64_t* partial;
    int64_t nwork;
    unsigned long long* rescans;   // if set: certificates that failed, accumulated
    // bw_blocks > 0: the launch's first bw_blocks workgroups compute the
    // iteration's median-heuristic bandwidths instead (bw_lds bytes of
    // dynamic LDS each; bw_form: where the pair distances go, a
    // BandwidthForm), beside the search
    SvgdArgs bw;
    int32_t bw_blocks;
    uint32_t bw_lds;
    int32_t bw_form;
};

// Shapes the screen is built for: q queries per lane (1 or 2) and w
// wavefronts per workgroup (4, 8, 16 for one query per lane; 4, 8 for two).
bool nn_bf16_shape_ok(int q, int w);

// Blocks of 32 references per key for shape (q, w) when the shortest
// chunk holds min_chunk references: 2 (q = 2 only) when every wavefront
// sweeps at least 192 blocks per work item, else 1. A key over two blocks
// takes 1.5 fewer vector instructions per block and query group and
// doubles the rerank, which only long sweeps repay.
int nn_bf16_key_span(int q, int w, int64_t min_chunk);

// q, w as above; fmt: 0 the BF16 x 3 screen, 1 the FP16 x 2 screen; span:
// blocks per key (1, or 2 for q = 2); grid workgroups (grid < nwork makes
// them persistent).
hipError_t launch_nn_bf16_kernel(int q, int w, int fmt, int span, unsigned grid, const NNBf16Args& a,
                                 hipStream_t s);

// FP16 screen scale exponent for a largest centred norm R (host copy of the
// device rule).
int f16_screen_exponent_host(float R);

// The screen's centre c0 of one pair from its n_ref packed references, on
// the device (written into pair->c0).
hipError_t launch_bf16_centre(PairDesc* pair, const float4* ref4, int64_t n_ref, hipStream_t s);

// The raw screened values of every (query, reference) of one pair (the
// screen's own fragments and products), nq x n_ref row-major.
hipError_t launch_screen_values(const PairDesc* pair, int64_t n_ref_pad, const uint4* apack, const float4* queries,
                                int64_t nq, int fmt, float* values, hipStream_t s);

// A fragments of the centred references of every pair; grid covers the
// largest pair's 16-reference blocks.
hipError_t launch_pack_bf16(const PairDesc* pairs, int32_t n_pairs, int64_t max_blocks, const float4* ref4,
                            uint4* apack, int fmt, hipStream_t s);

}  // namespace sicp
