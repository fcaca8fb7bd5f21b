// Translation unit of the BF16-screen nearest-neighbour kernels (built with
// -fno-honor-nans -mno-amdgpu-ieee; see nn_bf16_launch.h).
#include "nn_bf16.hpp"

namespace sicp {

bool nn_bf16_shape_ok(int q, int w)
{
    // two queries per lane need about 250 registers per lane: sixteen
    // wavefronts (128 registers each) would spill, so that shape is not built
    return (q == 1 && (w == 4 || w == 8 || w == 16)) || (q == 2 && (w == 4 || w == 8));
}

int nn_bf16_key_span(int q, int w, int64_t min_chunk)
{
    return q == 2 && min_chunk / ((int64_t)kBlk * w) >= 192 ? 2 : 1;
}

// grid: the work items' workgroups; the bandwidth workgroups come on top
template <int FMT, bool BW>
static void launch_fmt(int q, int w, int span, unsigned grid, const NNBf16Args& a, hipStream_t s)
{
    const dim3 g(grid + (BW ? (unsigned)a.bw_blocks : 0u));
    const size_t lds = BW ? a.bw_lds : 0;
    if (q == 1) {
        switch (w) {
        case 4: hipLaunchKernelGGL((nn_bf16_kernel<1, 4, FMT, BW, 1>), g, dim3(kWave * 4), lds, s, a); break;
        case 8: hipLaunchKernelGGL((nn_bf16_kernel<1, 8, FMT, BW, 1>), g, dim3(kWave * 8), lds, s, a); break;
        default: hipLaunchKernelGGL((nn_bf16_kernel<1, 16, FMT, BW, 1>), g, dim3(kWave * 16), lds, s, a); break;
        }
    } else if (span == 2) {
        if (w == 4) hipLaunchKernelGGL((nn_bf16_kernel<2, 4, FMT, BW, 2>), g, dim3(kWave * 4), lds, s, a);
        else hipLaunchKernelGGL((nn_bf16_kernel<2, 8, FMT, BW, 2>), g, dim3(kWave * 8), lds, s, a);
    } else {
        if (w == 4) hipLaunchKernelGGL((nn_bf16_kernel<2, 4, FMT, BW, 1>), g, dim3(kWave * 4), lds, s, a);
        else hipLaunchKernelGGL((nn_bf16_kernel<2, 8, FMT, BW, 1>), g, dim3(kWave * 8), lds, s, a);
    }
}

hipError_t launch_nn_bf16_kernel(int q, int w, int fmt, int span, unsigned grid, const NNBf16Args& a,
                                 hipStream_t s)
{
    if (!nn_bf16_shape_ok(q, w) || (span != 1 && span != 2) || (span == 2 && q != 2)) return hipErrorInvalidValue;
    const bool bw = a.bw_blocks > 0;
    if (fmt == kFmtF16x2) {
        if (bw) launch_fmt<kFmtF16x2, true>(q, w, span, grid, a, s);
        else launch_fmt<kFmtF16x2, false>(q, w, span, grid, a, s);
    } else if (fmt == kFmtBf16x3) {
        if (bw) launch_fmt<kFmtBf16x3, true>(q, w, span, grid, a, s);
        else launch_fmt<kFmtBf16x3, false>(q, w, span, grid, a, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int f16_screen_exponent_host(float R) { return f16_screen_exponent(R); }

hipError_t launch_screen_values(const PairDesc* pair, int64_t n_ref_pad, const uint4* apack, const float4* queries,
                                int64_t nq, int fmt, float* values, hipStream_t s)
{
    if (nq < 1) return hipSuccess;
    const dim3 grid((unsigned)(n_ref_pad / kBlk), (unsigned)((nq + 31) / 32));
    if (fmt == kFmtF16x2)
        hipLaunchKernelGGL(screen_values_kernel<kFmtF16x2>, grid, dim3(kWave), 0, s, pair, apack, queries, nq, values);
    else
        hipLaunchKernelGGL(screen_values_kernel<kFmtBf16x3>, grid, dim3(kWave), 0, s, pair, apack, queries, nq, values);
    return hipGetLastError();
}

hipError_t launch_bf16_centre(PairDesc* pair, const float4* ref4, int64_t n_ref, hipStream_t s)
{
    hipLaunchKernelGGL(bf16_centre_kernel, dim3(1), dim3(kCentreThreads), 0, s, pair, ref4, n_ref);
    return hipGetLastError();
}

hipError_t launch_pack_bf16(const PairDesc* pairs, int32_t n_pairs, int64_t max_blocks, const float4* ref4,
                            uint4* apack, int fmt, hipStream_t s)
{
    if (n_pairs < 1 || max_blocks < 1) return hipSuccess;
    const dim3 grid((unsigned)((max_blocks + 3) / 4), (unsigned)n_pairs);
    if (fmt == kFmtF16x2) hipLaunchKernelGGL(pack_f16_refs_kernel, grid, dim3(256), 0, s, pairs, ref4, apack);
    else hipLaunchKernelGGL(pack_bf16_refs_kernel, grid, dim3(256), 0, s, pairs, ref4, apack);
    return hipGetLastError();
}

}  // namespace sicp
