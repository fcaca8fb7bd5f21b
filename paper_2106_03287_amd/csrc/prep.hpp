// Packing, validation and pose kernels.
#pragma once

#include "common.hpp"

namespace sicp {

// Pose of one particle: R = Rz(yaw) Ry(pitch) Rx(roll) (Sec. III-A) and its
// partial derivatives with respect to roll, pitch, yaw (the factors of Eq. 5),
// written in closed form from A = Rz Ry:
//   R        = [A0 | A1 cr + A2 sr | -A1 sr + A2 cr]      (columns)
//   dR/droll = [0 | R2 | -R1]                              (columns)
//   dR/dpitch= [B0 | B2 sr | B2 cr], B = Rz dRy/dpitch     (columns)
//   dR/dyaw  = rows (-R row1, R row0, 0)
__device__ inline void pose_from_theta(const double* __restrict__ th, Pose* __restrict__ P)
{
#pragma clang fp contract(off)
    double sr, cr, sp, cp, sy, cy;
    sincos(th[3], &sr, &cr);
    sincos(th[4], &sp, &cp);
    sincos(th[5], &sy, &cy);
    const double A0[3] = {cy * cp, sy * cp, -sp};
    const double A1[3] = {-sy, cy, 0.0};
    const double A2[3] = {cy * sp, sy * sp, cp};
    const double B0[3] = {-cy * sp, -sy * sp, -cp};
    const double B2[3] = {cy * cp, sy * cp, -sp};
    double R[9], D[27];
    for (int r = 0; r < 3; ++r) {
        R[3 * r + 0] = A0[r];
        R[3 * r + 1] = A1[r] * cr + A2[r] * sr;
        R[3 * r + 2] = -A1[r] * sr + A2[r] * cr;
    }
    for (int r = 0; r < 3; ++r) {
        D[3 * r + 0] = 0.0;                // d/droll
        D[3 * r + 1] = R[3 * r + 2];
        D[3 * r + 2] = -R[3 * r + 1];
        D[9 + 3 * r + 0] = B0[r];          // d/dpitch
        D[9 + 3 * r + 1] = B2[r] * sr;
        D[9 + 3 * r + 2] = B2[r] * cr;
    }
    for (int c = 0; c < 3; ++c) {          // d/dyaw
        D[18 + c] = -R[3 + c];
        D[18 + 3 + c] = R[c];
        D[18 + 6 + c] = 0.0;
    }
    for (int i = 0; i < 9; ++i) P->R[i] = R[i];
    for (int i = 0; i < 3; ++i) P->u[i] = th[i];
    for (int i = 0; i < 27; ++i) P->dR[i] = D[i];
    P->pad_ = 0.0;
}

__global__ void pose_kernel(const double* __restrict__ theta, Pose* __restrict__ pose, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) pose_from_theta(theta + 6 * k, pose + k);
}

// FP32 queries of one iteration: query k * m + i of a pair is the FP64
// transform of minibatch point i by particle k's pose, rounded once.
__device__ __forceinline__ float4 make_query(const Pose* __restrict__ P, float4 s)
{
    double q[3];
    transform_f64(P->R, P->u, s.x, s.y, s.z, q);
    return make_float4((float)q[0], (float)q[1], (float)q[2], 0.0f);
}

// grid (ceil(K m / 256), pairs): queries of the iteration whose step count
// is step[p] (schedule row step mod rows).
__global__ void queries_kernel(const PairDesc* __restrict__ pairs, const float4* __restrict__ src4,
                               const int32_t* __restrict__ sched, const Pose* __restrict__ pose,
                               const int64_t* __restrict__ step, float4* __restrict__ queries, int32_t K,
                               int32_t m, int32_t rows)
{
    const int64_t p = blockIdx.y;
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const PairDesc pd = pairs[p];
    if (qi >= pd.nq) return;
    const int64_t k = qi / m, i = qi - k * m;
    const int64_t row = step[p] % rows;
    const float4 sp = src4[pd.src_off + sched[pd.sched_off + row * m + i]];
    queries[pd.q_off + qi] = make_query(pose + p * K + k, sp);
}

__device__ inline bool coord_ok(float v) { return isfinite(v) && fabsf(v) <= 1e9f; }

// n x 3 row-major -> float4 (x, y, z, 0); entries [n, n_pad) get the padding
// point. Sets *bad when any coordinate is non-finite or larger than 1e9.
__global__ void pack_points_kernel(const float* __restrict__ xyz, int64_t n, int64_t n_pad,
                                   float4* __restrict__ out, int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    if (i < n) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (!(coord_ok(x) && coord_ok(y) && coord_ok(z))) atomicOr(bad, 1);
        out[i] = make_float4(x, y, z, 0.0f);
    } else {
        out[i] = make_float4(kPadCoord, kPadCoord, kPadCoord, 0.0f);
    }
}

// Copy a rows x m schedule, checking every index lies in [0, n_src).
__global__ void copy_schedule_kernel(const int32_t* __restrict__ in, int64_t n, int64_t n_src,
                                     int32_t* __restrict__ out, int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = in[i];
    if (v < 0 || v >= n_src) atomicOr(bad, 2);
    out[i] = v;
}

// Copy FP64 values, flagging non-finite ones.
__global__ void copy_finite_kernel(const double* __restrict__ in, int64_t n, double* __restrict__ out,
                                   int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = in[i];
    if (!isfinite(v)) atomicOr(bad, 4);
    out[i] = v;
}

// Flag (bit 4) a non-finite FP64 value without copying it.
__global__ void check_finite_kernel(const double* __restrict__ in, int64_t n, int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(in[i])) atomicOr(bad, 4);
}

// FP32 particles in (widened exactly to FP64) and out (rounded to nearest),
// n values; the input side flags (bit 4) a non-finite value.
__global__ void check_finite_f32_kernel(const float* __restrict__ in, int64_t n, int* __restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(in[i])) atomicOr(bad, 4);
}

__global__ void widen_f32_kernel(const float* __restrict__ in, int64_t n, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

__global__ void narrow_f64_kernel(const double* __restrict__ in, int64_t n, float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void fill_i32_kernel(int* __restrict__ out, int64_t n, int v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void fill_f64_kernel(double* __restrict__ out, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void fill_i64_kernel(int64_t* __restrict__ out, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

}  // namespace sicp
