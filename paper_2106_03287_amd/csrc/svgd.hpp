// Stein direction (Eq. 16) and particle update (Eq. 12 with Adam).
//
// Per iteration:
//  * bandwidth_body, one workgroup per (pair, block): block 0 the
//    translation kernel, block 1 the wrapped-angle rotation kernel of
//    Eq. 17. It depends only on the particles, so it runs beside other
//    work: as 1024-thread workgroups of the gradient launch that carry no
//    particles, or (matrix-core screen, few particles in flight) as extra
//    workgroups of the nearest-neighbour launch on its workgroup size.
//    The median heuristic h = med^2 / ln K needs the middle order
//    statistics of the K(K-1)/2 distances between distinct particles, found
//    exactly: the distances are stored as 16-bit monotone keys in LDS (K up
//    to about 345, where the launch's LDS allows), a 4096-bin integer
//    histogram of the keys' own range finds the bins of both middle ranks in
//    one pass, and the exact FP64 distances of those bins' few pairs are
//    recomputed and ranked by counting (wider ranges narrow bin by bin).
//    Otherwise the FP64 distances go to global memory and are binned by
//    value. A radix select over IEEE-754 bit patterns covers the degenerate
//    cases. Both forms return the same order statistics.
//  * svgd_phi_update_kernel, one 256-thread workgroup per particle k:
//    phi_k = (1/K) sum_l [G_l k(l,k) + grad_{theta_l} k(l,k)] with
//    G_l = -N gbar_l + grad log p(theta_l) (Eq. 10 with Eqs. 14-15), threads
//    over l and a fixed-shape reduction; then Adam on -phi (or
//    theta += lr phi) for particle k, written to the other particle buffer
//    (other wavefronts still read the current particles; the buffers swap
//    roles every iteration), the particle's next pose and its FP32 queries
//    of the next iteration, and the pair's next step count.
#pragma once

#include "common.hpp"
#include "prep.hpp"
#include "svgd_select.hpp"

namespace sicp {

constexpr int kPhiThreads = 256;   // threads per particle of the direction / update kernel

// grid (K, pairs), kPhiThreads threads: one workgroup per particle. Thread t
// takes the kernel terms of particles l = t, t + 256, ...; the sums are
// combined by a fixed-shape tree (wavefront shuffles, then the four
// wavefronts in order), Adam updates the six components, and every thread
// transforms its minibatch points for the next iteration.
__global__ __launch_bounds__(kPhiThreads) void svgd_phi_update_kernel(SvgdArgs a)
{
    __shared__ double red[kPhiThreads / kWave][6];
    __shared__ double tn_sh[6];
    const int64_t p = blockIdx.y;
    const int K = a.K;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int k = blockIdx.x;
    const PairDesc pd = a.pairs[p];
    const double* __restrict__ th = a.theta + p * K * 6;
    const double* __restrict__ gb = a.gbar + p * K * 6;
    const double ht = a.h[2 * p], hr = a.h[2 * p + 1];
    const double ct = -(2.0 / ht), cr = -(2.0 / hr);
    const double N = (double)pd.n_scale;
    double tk[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) tk[d] = th[6 * k + d];
    // what does not depend on the new particle goes first, so that its
    // latency overlaps the sums: this thread's minibatch points of the next
    // iteration (m <= 4 kPhiThreads per pass) and Adam's bias corrections
    const int64_t row = (a.step[p] + 1) % a.rows;
    const int32_t* __restrict__ srow = a.sched + pd.sched_off + row * a.m;
    float4 sp0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = tid + u * kPhiThreads;
        sp0[u] = i < a.m ? a.src4[pd.src_off + srow[i]] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    double bc1 = 1.0, bc2 = 1.0;
    if (tid < 6 && a.prm.optimizer != 1) {
        const double t_new = (double)(a.step[p] + 1);
        bc1 = 1.0 - pow(a.prm.beta1, t_new);
        bc2 = 1.0 - pow(a.prm.beta2, t_new);
    }

    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = tid; l < K; l += kPhiThreads) {
        double tl[6], G[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) tl[d] = th[6 * l + d];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            double pg = 0.0;
            if (a.prm.prior == 1) {
                const double y = tl[d] - a.prm.prior_mu[d];
                pg = d < 3 ? -y / a.prm.prior_var[d] : -a.prm.prior_kappa[d - 3] * sin(y);
            }
            G[d] = -N * gb[6 * l + d] + pg;
        }
        double kt = 1.0, kr = 1.0;
        if (l != k) {
            kt = exp(-dist2_trans(tl, tk) / ht);
            kr = exp(-dist2_rot(tl, tk) / hr);
        }
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                acc[d] += G[d] * kt + ct * (tl[d] - tk[d]) * kt;
                acc[3 + d] += G[3 + d] * kr + cr * wrap_pi(tl[3 + d] - tk[3 + d]) * kr;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        double x = acc[d];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o);
        acc[d] = x;
    }
    if (lane < 6) {
        double v = 0.0;
#pragma unroll
        for (int d = 0; d < 6; ++d)
            if (lane == d) v = acc[d];
        red[wave][lane] = v;
    }
    __syncthreads();
    // threads 0..5 update one component each
    if (tid < 6) {
#pragma clang fp contract(off)
        double sum = red[0][tid];
#pragma unroll
        for (int w = 1; w < kPhiThreads / kWave; ++w) sum += red[w][tid];
        const double phi_d = sum / K;
        const int64_t e = (p * K + k) * 6 + tid;
        double tnew;
        a.phi[e] = phi_d;
        if (a.prm.optimizer == 1) {
            tnew = th[6 * k + tid] + a.prm.lr * phi_d;
        } else {
            const double g = -phi_d;
            const double mm = a.prm.beta1 * a.mom[e] + (1.0 - a.prm.beta1) * g;
            const double vv = a.prm.beta2 * a.vel[e] + (1.0 - a.prm.beta2) * (g * g);
            a.mom[e] = mm;
            a.vel[e] = vv;
            const double mhat = mm / bc1;
            const double vhat = vv / bc2;
            tnew = th[6 * k + tid] - a.prm.lr * mhat / (sqrt(vhat) + a.prm.eps);
        }
        a.theta_next[e] = tnew;
        tn_sh[tid] = tnew;
    }
    __syncthreads();
    double tn[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) tn[d] = tn_sh[d];
    // the new pose (every thread computes the same bits) and this particle's
    // queries of the next iteration
    Pose P;
    pose_from_theta(tn, &P);
    if (tid == 0) a.pose[p * K + k] = P;
    if (k == 0 && tid == 0) a.step_next[p] = a.step[p] + 1;   // read only by the next iteration
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = tid + u * kPhiThreads;
        if (i < a.m) a.queries[pd.q_off + (int64_t)k * a.m + i] = make_query(&P, sp0[u]);
    }
    for (int i0 = tid + 4 * kPhiThreads; i0 < a.m; i0 += 4 * kPhiThreads) {   // m > 1024
        int32_t si[4];
        float4 sp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) si[u] = i0 + u * kPhiThreads < a.m ? srow[i0 + u * kPhiThreads] : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) sp[u] = a.src4[pd.src_off + si[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * kPhiThreads < a.m)
                a.queries[pd.q_off + (int64_t)k * a.m + i0 + u * kPhiThreads] = make_query(&P, sp[u]);
    }
}

}  // namespace sicp
