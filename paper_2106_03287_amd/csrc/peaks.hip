// Device ceilings measured on the device (include/stein_icp_peaks.h): a
// streaming copy, unpacked FP32 fused multiply-adds, and 32x32x16 FP16 /
// BF16 matrix-core products. Not part of the method: they give the
// roofline fractions a measured denominator beside the published peaks.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "stein_icp.h"
#include "stein_icp_peaks.h"

namespace sicp {
int report_error(int code, const std::string& msg);
}

namespace {

constexpr int kProbeThreads = 256;   // threads per workgroup of every probe
constexpr int kWaveWidth = 64;
constexpr int kFmaChains = 16;       // independent FMA chains per thread
constexpr int kMfmaTiles = 4;        // independent accumulator tiles per wavefront
constexpr double kMfmaFlops = 2.0 * 32 * 32 * 16;

typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

int fail(int code, const std::string& msg) { return sicp::report_error(code, msg); }

// grid-stride float4 copy, four loads in flight per thread
__global__ __launch_bounds__(kProbeThreads) void copy_probe_kernel(const float4* __restrict__ in,
                                                                   float4* __restrict__ out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const float4 a = in[i], b = in[i + stride], c = in[i + 2 * stride], d = in[i + 3 * stride];
        out[i] = a;
        out[i + stride] = b;
        out[i + 2 * stride] = c;
        out[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) out[i] = in[i];
}

// b and c arrive as arguments, so the compiler cannot fold the products
__global__ __launch_bounds__(kProbeThreads) void fma_probe_kernel(float* __restrict__ out, float b, float c,
                                                                  int32_t iters)
{
    const int64_t gid = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    float a[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) a[k] = (float)(gid + k);
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k) a[k] = fmaf(a[k], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += a[k];
    out[gid] = s;
}

template <bool BF16>
__global__ __launch_bounds__(kProbeThreads) void mfma_probe_kernel(const uint4* __restrict__ frag,
                                                                   float* __restrict__ out, int32_t iters)
{
    const int lane = threadIdx.x & (kWaveWidth - 1);
    const uint4 fa = frag[lane], fb = frag[kWaveWidth + lane];
    f32x16_t acc[kMfmaTiles];
#pragma unroll
    for (int k = 0; k < kMfmaTiles; ++k)
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[k][t] = 0.f;
    for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kMfmaTiles; ++k) {
            if constexpr (BF16)
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, fa),
                                                                  __builtin_bit_cast(bf16x8_t, fb), acc[k], 0, 0, 0);
            else
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, fa),
                                                                 __builtin_bit_cast(f16x8_t, fb), acc[k], 0, 0, 0);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kMfmaTiles; ++k)
#pragma unroll
        for (int t = 0; t < 16; ++t) s += acc[k][t];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

bool arithmetic_kind(int kind)
{
    return kind == STEIN_ICP_PEAK_FMA32 || kind == STEIN_ICP_PEAK_MFMA_F16 || kind == STEIN_ICP_PEAK_MFMA_BF16;
}

}  // namespace

extern "C" {

double stein_icp_peak_work(int kind, int64_t n, int32_t iters)
{
    switch (kind) {
    case STEIN_ICP_PEAK_COPY: return 32.0 * (double)n;
    case STEIN_ICP_PEAK_FMA32: return 2.0 * kFmaChains * (double)n * (double)iters;
    case STEIN_ICP_PEAK_MFMA_F16:
    case STEIN_ICP_PEAK_MFMA_BF16: return (double)(n / kWaveWidth) * kMfmaTiles * kMfmaFlops * (double)iters;
    default: return -1.0;
    }
}

int stein_icp_peak_probe(int kind, const void* in, void* out, int64_t n, int32_t iters, float b, float c,
                         void* hip_stream)
{
    if (kind < STEIN_ICP_PEAK_COPY || kind > STEIN_ICP_PEAK_MFMA_BF16)
        return fail(STEIN_ICP_E_INVALID, "peak_probe: unknown kind");
    if (n < 1 || !out) return fail(STEIN_ICP_E_INVALID, "peak_probe: n < 1 or out is NULL");
    if (arithmetic_kind(kind) && (n % kProbeThreads != 0 || iters < 1 || iters > (1 << 24)))
        return fail(STEIN_ICP_E_INVALID, "peak_probe: n must be a multiple of 256 and 1 <= iters <= 2^24");
    if (kind != STEIN_ICP_PEAK_FMA32 && !in) return fail(STEIN_ICP_E_INVALID, "peak_probe: in is NULL");
    if (n / kProbeThreads > 0x7fffffff) return fail(STEIN_ICP_E_INVALID, "peak_probe: n too large");
    const hipStream_t s = (hipStream_t)hip_stream;
    if (kind == STEIN_ICP_PEAK_COPY) {
        const int64_t groups = (n + 4 * kProbeThreads - 1) / (4 * kProbeThreads);
        const unsigned grid = (unsigned)(groups < 65536 ? groups : 65536);
        hipLaunchKernelGGL(copy_probe_kernel, dim3(grid), dim3(kProbeThreads), 0, s, (const float4*)in,
                           (float4*)out, n);
    } else if (kind == STEIN_ICP_PEAK_FMA32) {
        hipLaunchKernelGGL(fma_probe_kernel, dim3((unsigned)(n / kProbeThreads)), dim3(kProbeThreads), 0, s,
                           (float*)out, b, c, iters);
    } else if (kind == STEIN_ICP_PEAK_MFMA_F16) {
        hipLaunchKernelGGL(mfma_probe_kernel<false>, dim3((unsigned)(n / kProbeThreads)), dim3(kProbeThreads), 0, s,
                           (const uint4*)in, (float*)out, iters);
    } else {
        hipLaunchKernelGGL(mfma_probe_kernel<true>, dim3((unsigned)(n / kProbeThreads)), dim3(kProbeThreads), 0, s,
                           (const uint4*)in, (float*)out, iters);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("peak_probe launch: ") + hipGetErrorString(e));
    return STEIN_ICP_OK;
}

int stein_icp_device_info(int32_t* compute_units, int32_t* lds_bytes_per_cu, int32_t* wave_size, int32_t* clock_khz,
                          char* arch, int32_t arch_len)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (e == hipSuccess) e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return fail(STEIN_ICP_E_DEVICE, std::string("device_info: ") + hipGetErrorString(e));
    if (compute_units) *compute_units = p.multiProcessorCount;
    if (lds_bytes_per_cu) *lds_bytes_per_cu = (int32_t)p.maxSharedMemoryPerMultiProcessor;
    if (wave_size) *wave_size = p.warpSize;
    if (clock_khz) *clock_khz = p.clockRate;
    if (arch && arch_len > 0) {
        std::strncpy(arch, p.gcnArchName, (size_t)arch_len - 1);
        arch[arch_len - 1] = '\0';
    }
    return STEIN_ICP_OK;
}

}  // extern "C"
