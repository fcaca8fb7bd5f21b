// One launch for the two stages that follow the nearest neighbours and
// depend on nothing but the particles and the matches: the median-heuristic
// bandwidths (Sec. V) and the mean gradients (Eqs. 4-5). The first 2 P
// workgroups compute the bandwidths of pair w / 2, block w % 2; the others
// compute the gradients of two particles each. The roles share one dynamic
// LDS buffer of grad_bw_lds_bytes(K) bytes.
#pragma once

#include "grad.hpp"
#include "svgd.hpp"

namespace sicp {

static_assert(kGradGroups * kGradThreads == kSvgdThreads, "both roles use the same workgroup size");

inline size_t grad_bw_lds_bytes(int K)
{
    const size_t sel = (sizeof(SelectShared) + 15) / 16 * 16;
    const size_t bw = sel + bandwidth_lds_bytes(K, bandwidth_keyable(K) ? kKeysInLds : kDistancesInGlobal);
    const size_t gr = sizeof(double) * 6 * kGradGroups * (kGradThreads / kWave);
    return bw > gr ? bw : gr;
}

// grid: 2 bw_pairs + ceil(P K / kGradGroups) workgroups of kSvgdThreads
// threads. bw_pairs is P, or 0 when the bandwidths are constants (a fixed
// bandwidth, or K = 1) written once at init.
__global__ __launch_bounds__(kSvgdThreads) void grad_bandwidth_kernel(GradArgs g, SvgdArgs v, int32_t n_pairs,
                                                                      int32_t bw_pairs)
{
    extern __shared__ double lds[];
    const int64_t bw_blocks = 2 * (int64_t)bw_pairs;
    if ((int64_t)blockIdx.x < bw_blocks) {   // whole workgroup
        bandwidth_role<kSvgdThreads>(v, blockIdx.x, bandwidth_keyable(v.K) ? kKeysInLds : kDistancesInGlobal, lds);
        return;
    }
    const int64_t wg = (int64_t)blockIdx.x - bw_blocks;
    // the group (and so the particle and pair) is uniform over a wavefront:
    // say so, and the pair's descriptor lives in scalar registers
    const int grp = uniform(threadIdx.x / kGradThreads), lt = threadIdx.x % kGradThreads;
    grad_group(g, wg * kGradGroups + grp, (int64_t)n_pairs * v.K, grp, lt, lds);
}

}  // namespace sicp
