// Per-particle mean gradient (Eqs. 4-5, point-to-point or point-to-plane),
// fused with the final reduction of the per-chunk nearest-neighbour keys.
//
// One group of 512 threads per particle, two groups to a workgroup. Each
// thread takes minibatch points i = t, t + 512, ...: it reduces the chunk
// keys of its query to the matched reference index (resolving the winning
// tile of the FP32 search; the BF16 screen's keys carry the index),
// recomputes the FP64 transform s' = R s + u, forms the residual
// e = s' - r and the six contributions e and e^T (dR/dtheta_d) s,
// accumulating in FP64. With the point-to-plane metric e is first replaced by
// its projection rho n on the matched reference's unit normal n
// (rho = n^T e), which gives rho n and rho n^T (dR/dtheta_d) s. The
// group's partial sums are combined by a fixed-shape tree (shuffles within
// each wavefront, then the wavefronts in order), so the result does not
// depend on scheduling.
#pragma once

#include "common.hpp"
#include "nn.hpp"

namespace sicp {

struct GradArgs {
    const PairDesc* pairs;
    const float4* src4;
    const float4* ref4;
    const float4* queries;
    const int32_t* sched;
    const Pose* pose;
    const int64_t* step;
    const uint64_t* partial;
    int32_t* match;       // K*m per pair, pair-relative reference indices
    double* gbar;         // 6 per particle
    const double* nrm;    // point-to-plane: 4 doubles (n, 0) per packed reference; NULL: point-to-point
    int32_t K, m, rows;
    int32_t index_keys;   // 1: the keys carry the reference index (BF16 screen), 0: the tile
};

constexpr int kGradGroups = 2;   // particles per 1024-thread workgroup, kGradThreads threads each

// Gradient of particle pk (global index over pairs, pk < nparticles) by the
// group `grp` of kGradThreads threads (lt = thread within the group); red is
// the workgroup's LDS for the wavefront sums (6 FP64 per wavefront). Every
// thread of the workgroup takes part in the barrier, also for pk >= n.
__device__ __forceinline__ void grad_group(const GradArgs& a, int64_t pk, int64_t n, int grp, int lt, double* red)
{
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool live = pk < n;
    int64_t p = 0, k = 0;
    if (live) {
        p = pk / a.K;
        k = pk - p * a.K;
        const PairDesc pd = a.pairs[p];
        const int64_t nq = (int64_t)a.K * a.m;
        const int64_t row = a.step[p] % a.rows;
        const Pose* __restrict__ P = a.pose + pk;
        for (int i = lt; i < a.m; i += kGradThreads) {
            const int64_t qi = k * a.m + i;
            // the loads that do not depend on the match go first, so that
            // their latency overlaps the key's; the match is stored after
            // the last load
            const float4 s = a.src4[pd.src_off + a.sched[pd.sched_off + row * a.m + i]];
            const float4 qf = a.queries[pd.q_off + qi];
            const uint64_t key = min_chunk_keys(a.partial + pd.part_off + qi, pd.chunks, pd.part_stride);
            const int32_t j = key_index(key, a.index_keys != 0, qf, a.ref4 + pd.ref_off, pd.n_ref_pad);
            const float4 r = a.ref4[pd.ref_off + j];
            a.match[p * nq + qi] = j;
            double q[3];
            transform_f64(P->R, P->u, s.x, s.y, s.z, q);
            {
#pragma clang fp contract(off)
                double e0 = q[0] - (double)r.x, e1 = q[1] - (double)r.y, e2 = q[2] - (double)r.z;
                if (a.nrm) {
                    asm volatile("" ::: "memory");   // load the normal here, not earlier
                    const double* n = a.nrm + 4 * (pd.ref_off + j);
                    const double n0 = n[0], n1 = n[1], n2 = n[2];
                    const double rho = (n0 * e0 + n1 * e1) + n2 * e2;
                    e0 = rho * n0;
                    e1 = rho * n1;
                    e2 = rho * n2;
                }
                acc[0] += e0;
                acc[1] += e1;
                acc[2] += e2;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    // compiler barrier (no instruction): load each 3 x 3 block of
                    // dR where it is used instead of keeping all 27 in registers
                    asm volatile("" ::: "memory");
                    const double* D = P->dR + 9 * d;
                    const double v0 = (D[0] * s.x + D[1] * s.y) + D[2] * s.z;
                    const double v1 = (D[3] * s.x + D[4] * s.y) + D[5] * s.z;
                    const double v2 = (D[6] * s.x + D[7] * s.y) + D[8] * s.z;
                    acc[3 + d] += (e0 * v0 + e1 * v1) + e2 * v2;
                }
            }
        }
    }
    // fixed-shape reduction: a shuffle tree inside each wavefront, then the
    // group's wavefronts in order (one barrier)
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        double x = acc[d];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
        acc[d] = x;
    }
    constexpr int WV = kGradThreads / kWave;   // wavefronts per group
    double* r0 = red + grp * WV * 6;
    const int wv = lt / kWave, lane = lt % kWave;
    if (lane < 6) {
        double v = 0.0;
#pragma unroll
        for (int d = 0; d < 6; ++d)
            if (lane == d) v = acc[d];
        r0[wv * 6 + lane] = v;
    }
    __syncthreads();
    if (live && lt < 6) {
        double sum = r0[lt];
#pragma unroll
        for (int v = 1; v < WV; ++v) sum += r0[v * 6 + lt];
        a.gbar[pk * 6 + lt] = sum / (double)a.m;
    }
}

}  // namespace sicp
