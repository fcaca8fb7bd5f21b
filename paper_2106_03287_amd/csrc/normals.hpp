// Reference normals for the point-to-plane metric: the k nearest references
// of each point (Eq. 1's FP32 distance, ties to the lower index) and the
// eigenvector of the smallest eigenvalue of their covariance.
//
// knn_partial_kernel: a workgroup takes 256 queries (one per thread) and one
// chunk of the references, staged through LDS 256 at a time; every thread
// keeps its k smallest (distance, index) keys in registers as a sorted list,
// screening 32 references at a time before inserting.
// knn_merge_kernel: one thread per query merges the chunks' lists, writes the
// neighbours and/or forms the FP64 covariance of the neighbourhood and its
// normal.
#pragma once

#include "common.hpp"

namespace sicp {

constexpr int kKnnThreads = 256;   // queries per workgroup of the partial scan
constexpr int kKnnTile = 256;      // references staged in LDS per step
constexpr int kKnnMax = 32;        // largest k
constexpr uint64_t kNoKey = ~0ull;

// Insert `key` into the ascending list b, dropping the largest entry. Every
// index is a compile-time constant, so the list stays in registers.
template <int KMAX>
__device__ __forceinline__ void topk_insert(uint64_t (&b)[KMAX], uint64_t key)
{
#pragma unroll
    for (int i = KMAX - 1; i > 0; --i) b[i] = key < b[i - 1] ? b[i - 1] : (key < b[i] ? key : b[i]);
    b[0] = key < b[0] ? key : b[0];
}

// A list of k <= KMAX live entries: the first KMAX - k slots hold 0, which
// no key displaces (an equal key is inserted after them), the rest kNoKey.
template <int KMAX>
__device__ __forceinline__ void topk_init(uint64_t (&b)[KMAX], int k)
{
#pragma unroll
    for (int s = 0; s < KMAX; ++s) b[s] = s < KMAX - k ? 0ull : kNoKey;
}

struct KnnArgs {
    const float4* q4;      // queries (x, y, z, -)
    const float4* ref4;    // references
    int64_t nq, n_ref;
    int64_t chunk;         // references per chunk, a multiple of kKnnTile
    uint64_t* partial;     // chunks x nq x k keys, each list ascending
    int32_t k, pad_;
};

// grid: (ceil(nq / kKnnThreads), chunks), kKnnThreads threads.
template <int KMAX>
__global__ __launch_bounds__(kKnnThreads) void knn_partial_kernel(KnnArgs a)
{
    __shared__ float4 tile[kKnnTile];
    const int64_t qi = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
    const bool live = qi < a.nq;
    const float4 q = live ? a.q4[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
    uint64_t b[KMAX];
    topk_init(b, a.k);
    const int64_t j0 = (int64_t)blockIdx.y * a.chunk;
    const int64_t j1 = j0 + a.chunk < a.n_ref ? j0 + a.chunk : a.n_ref;
    for (int64_t t0 = j0; t0 < j1; t0 += kKnnTile) {
        const int64_t j = t0 + threadIdx.x;
        __syncthreads();
        if (j < j1) tile[threadIdx.x] = a.ref4[j];
        __syncthreads();
        const int n = j1 - t0 < kKnnTile ? (int)(j1 - t0) : kKnnTile;
        for (int u0 = 0; u0 < n; u0 += 32) {
            // screen 32 references against the list's current worst distance
            // (a stale, so conservative, bound), then insert the lane's own
            // survivors: the wavefront runs as many insertions as its busiest
            // lane needs, not one for every reference some lane keeps
            const uint64_t worst = b[KMAX - 1];
            const float thr = worst == kNoKey ? __builtin_inff() : __uint_as_float((uint32_t)(worst >> 32));
            uint32_t mask = 0;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const float4 r = tile[u0 + u];
                const float d = dist2_f32(q.x, q.y, q.z, r.x, r.y, r.z);
                if (u0 + u < n && d <= thr) mask |= 1u << u;
            }
            while (mask) {
                const int u = __builtin_ctz(mask);
                mask &= mask - 1;
                const float4 r = tile[u0 + u];
                const uint64_t key = pack_key(dist2_f32(q.x, q.y, q.z, r.x, r.y, r.z), (uint32_t)(t0 + u0 + u));
                if (key < b[KMAX - 1]) topk_insert(b, key);
            }
        }
    }
    if (!live) return;
    uint64_t* out = a.partial + ((int64_t)blockIdx.y * a.nq + qi) * a.k;
    const int lo = KMAX - a.k;
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s >= lo) out[s - lo] = b[s];
}

struct KnnMergeArgs {
    const uint64_t* partial;
    const float4* ref4;    // the references the keys index
    int64_t nq;
    int32_t k, chunks;
    int32_t* idx;          // optional: nq x k neighbour indices (-1 past n_ref)
    float* d2;             // optional with idx: their FP32 squared distances (inf past n_ref)
    double* nrm;           // optional: normals, nrm_stride doubles per query
    double* eig;           // optional with nrm: covariance eigenvalues, 3 per query, ascending
    int32_t nrm_stride, pad_;
};

// Unit eigenvector of the symmetric matrix A for its eigenvalue w: the
// largest cross product of two rows of A - w I (those rows span the
// complement of the eigenvector when w is a simple eigenvalue).
__device__ __forceinline__ bool sym3_eigvec(double a00, double a01, double a02, double a11, double a12, double a22,
                                            double w, double v[3])
{
#pragma clang fp contract(off)
    const double u0 = a00 - w, u1 = a01, u2 = a02;   // row 0
    const double v0 = a01, v1 = a11 - w, v2 = a12;   // row 1
    const double t0 = a02, t1 = a12, t2 = a22 - w;   // row 2
    const double c0x = u1 * v2 - u2 * v1, c0y = u2 * v0 - u0 * v2, c0z = u0 * v1 - u1 * v0;
    const double c1x = u1 * t2 - u2 * t1, c1y = u2 * t0 - u0 * t2, c1z = u0 * t1 - u1 * t0;
    const double c2x = v1 * t2 - v2 * t1, c2y = v2 * t0 - v0 * t2, c2z = v0 * t1 - v1 * t0;
    const double n0 = (c0x * c0x + c0y * c0y) + c0z * c0z;
    const double n1 = (c1x * c1x + c1y * c1y) + c1z * c1z;
    const double n2 = (c2x * c2x + c2y * c2y) + c2z * c2z;
    double x = c0x, y = c0y, z = c0z, nn = n0;
    if (n1 > nn) {
        x = c1x;
        y = c1y;
        z = c1z;
        nn = n1;
    }
    if (n2 > nn) {
        x = c2x;
        y = c2y;
        z = c2z;
        nn = n2;
    }
    if (!(nn > 0.0)) return false;
    const double len = sqrt(nn);
    v[0] = x / len;
    v[1] = y / len;
    v[2] = z / len;
    return true;
}

// Eigenvalues w (ascending) of the symmetric 3x3 matrix
// [a00 a01 a02; a01 a11 a12; a02 a12 a22] and a unit eigenvector n of the
// smallest (n = 0 when all three are equal). The closed-form (trigonometric)
// roots of the characteristic cubic are accurate for the root that lies
// apart from the other two (the smallest when det(A - tr/3 I) < 0, else the
// largest) but not for two roots close together, so only that root is taken
// from the cubic: its eigenvector from cross products, then the 2x2 problem
// on the plane orthogonal to it, solved with the half-angle rotation, gives
// the other two roots and their eigenvectors.
__device__ __forceinline__ void sym3_smallest(double a00, double a01, double a02, double a11, double a12, double a22,
                                              double w[3], double n[3])
{
#pragma clang fp contract(off)
    const double q = ((a00 + a11) + a22) / 3.0;
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p1 = (a01 * a01 + a02 * a02) + a12 * a12;
    const double p2 = ((b00 * b00 + b11 * b11) + b22 * b22) + 2.0 * p1;
    n[0] = n[1] = n[2] = 0.0;
    w[0] = w[1] = w[2] = q;
    if (!(p2 > 0.0)) return;
    const double p = sqrt(p2 / 6.0);
    const double det = b00 * (b11 * b22 - a12 * a12) - a01 * (a01 * b22 - a12 * a02) + a02 * (a01 * a12 - b11 * a02);
    double r = det / (2.0 * p * p * p);
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    const bool low = r < 0.0;   // the smallest root lies apart
    const double two_pi_3 = 2.0943951023931954923;   // 2 pi / 3
    const double wi = low ? q + 2.0 * p * cos(phi + two_pi_3) : q + 2.0 * p * cos(phi);
    double v[3];
    if (!sym3_eigvec(a00, a01, a02, a11, a12, a22, wi, v)) return;
    // orthonormal u, t spanning the plane orthogonal to v: u = v x e for the
    // axis e least aligned with v, t = v x u
    const double ax = fabs(v[0]), ay = fabs(v[1]), az = fabs(v[2]);
    double u[3];
    if (ax <= ay && ax <= az) {          // e = x
        u[0] = 0.0;
        u[1] = v[2];
        u[2] = -v[1];
    } else if (ay <= az) {               // e = y
        u[0] = -v[2];
        u[1] = 0.0;
        u[2] = v[0];
    } else {                             // e = z
        u[0] = v[1];
        u[1] = -v[0];
        u[2] = 0.0;
    }
    const double ul = sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
    u[0] /= ul;
    u[1] /= ul;
    u[2] /= ul;
    const double t[3] = {v[1] * u[2] - v[2] * u[1], v[2] * u[0] - v[0] * u[2], v[0] * u[1] - v[1] * u[0]};
    // A restricted to span(u, t): [[a, b], [b, c]]
    const double Au0 = (a00 * u[0] + a01 * u[1]) + a02 * u[2];
    const double Au1 = (a01 * u[0] + a11 * u[1]) + a12 * u[2];
    const double Au2 = (a02 * u[0] + a12 * u[1]) + a22 * u[2];
    const double At0 = (a00 * t[0] + a01 * t[1]) + a02 * t[2];
    const double At1 = (a01 * t[0] + a11 * t[1]) + a12 * t[2];
    const double At2 = (a02 * t[0] + a12 * t[1]) + a22 * t[2];
    const double ra = (u[0] * Au0 + u[1] * Au1) + u[2] * Au2;
    const double rb = (u[0] * At0 + u[1] * At1) + u[2] * At2;
    const double rc = (t[0] * At0 + t[1] * At1) + t[2] * At2;
    const double mid = 0.5 * (ra + rc), h = 0.5 * (ra - rc);
    const double rad = sqrt(h * h + rb * rb);
    if (low) {
        w[0] = wi;
        w[1] = mid - rad;
        w[2] = mid + rad;
        n[0] = v[0];
        n[1] = v[1];
        n[2] = v[2];
    } else {
        w[0] = mid - rad;
        w[1] = mid + rad;
        w[2] = wi;
        // (cos th, sin th) with th = atan2(b, h) / 2 is the eigenvector of the
        // larger root of the 2x2 problem; the smaller one is orthogonal to it
        double sn, cs;
        sincos(0.5 * atan2(rb, h), &sn, &cs);
        n[0] = -sn * u[0] + cs * t[0];
        n[1] = -sn * u[1] + cs * t[1];
        n[2] = -sn * u[2] + cs * t[2];
    }
}

// grid: ceil(nq / 256) workgroups of 256 threads, one query each.
template <int KMAX>
__global__ __launch_bounds__(256) void knn_merge_kernel(KnnMergeArgs a)
{
#pragma clang fp contract(off)
    const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= a.nq) return;
    uint64_t b[KMAX];
    topk_init(b, a.k);
    for (int ch = 0; ch < a.chunks; ++ch) {
        const uint64_t* l = a.partial + ((int64_t)ch * a.nq + qi) * a.k;
        for (int s = 0; s < a.k; ++s) {
            const uint64_t key = l[s];
            if (!(key < b[KMAX - 1])) break;   // the list ascends
            topk_insert(b, key);
        }
    }
    const int lo = KMAX - a.k;
    if (a.idx) {
#pragma unroll
        for (int s = 0; s < KMAX; ++s) {
            if (s < lo) continue;
            const uint64_t key = b[s];
            a.idx[qi * a.k + (s - lo)] = key == kNoKey ? -1 : (int32_t)(uint32_t)key;
            a.d2[qi * a.k + (s - lo)] = key == kNoKey ? __builtin_inff() : __uint_as_float((uint32_t)(key >> 32));
        }
    }
    if (!a.nrm) return;
    // covariance (1/c) sum (p - mean)(p - mean)^T over the c neighbours, in
    // rank order
    int c = 0;
    double mu[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < lo || b[s] == kNoKey) continue;
        const float4 p = a.ref4[(uint32_t)b[s]];
        mu[0] += (double)p.x;
        mu[1] += (double)p.y;
        mu[2] += (double)p.z;
        ++c;
    }
    for (int d = 0; d < 3; ++d) mu[d] /= (double)c;
    double C[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // 00 01 02 11 12 22
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        if (s < lo || b[s] == kNoKey) continue;
        const float4 p = a.ref4[(uint32_t)b[s]];
        const double v0 = (double)p.x - mu[0], v1 = (double)p.y - mu[1], v2 = (double)p.z - mu[2];
        C[0] += v0 * v0;
        C[1] += v0 * v1;
        C[2] += v0 * v2;
        C[3] += v1 * v1;
        C[4] += v1 * v2;
        C[5] += v2 * v2;
    }
    for (int e = 0; e < 6; ++e) C[e] /= (double)c;
    double w[3], n[3];
    sym3_smallest(C[0], C[1], C[2], C[3], C[4], C[5], w, n);
    // no unique plane: the smallest eigenvalue not separated from the middle
    const double trace = (w[0] + w[1]) + w[2];
    if (!(w[1] - w[0] > 1e-10 * trace)) n[0] = n[1] = n[2] = 0.0;
    double* o = a.nrm + qi * a.nrm_stride;
    o[0] = n[0];
    o[1] = n[1];
    o[2] = n[2];
    if (a.nrm_stride > 3) o[3] = 0.0;
    if (a.eig) {
        a.eig[qi * 3 + 0] = w[0];
        a.eig[qi * 3 + 1] = w[1];
        a.eig[qi * 3 + 2] = w[2];
    }
}

}  // namespace sicp
