// Device-side building blocks for the gfx950 SketchyCGAL kernels:
// wave64 / workgroup reductions in a fixed order, a deterministic grid-wide
// reduction finished by the last workgroup to arrive, the XCD-aware
// workgroup -> work-range map, and the Philox4x64-10 normal stream used for
// Omega and the Lanczos start vectors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scg {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kXcd = 8;              // MI355X: 8 XCDs, 32 CUs each, one L2 per XCD

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b % 8).  Renumber so that each XCD owns one contiguous eighth of the
// work ranges, keeping neighbouring rows (and their gathered x entries) in
// one L2.  The grid size is a multiple of 8, so this is a bijection.
__device__ __forceinline__ int xcd_lid() {
    const int G = gridDim.x;
    const int b = blockIdx.x;
    return (b % kXcd) * (G / kXcd) + b / kXcd;
}

// [lo, hi) of `total` items owned by logical workgroup lid of G.
__device__ __forceinline__ void split_range(int64_t total, int lid, int G, int64_t& lo, int64_t& hi) {
    lo = total * lid / G;
    hi = total * (lid + 1) / G;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup; the result is returned to every thread.
// `red` is __shared__ double[kWaves].  Fixed order, so deterministic.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s += red[i];
    return s;
}

// Grid-wide sum of W per-thread values.  Every workgroup of the launch must
// call it exactly once.  Each workgroup stores its W partial sums in
// part[blockIdx.x * W + w]; the last workgroup to arrive (ticket on
// *counter, release/acquire at agent scope) adds the partials in workgroup
// order and returns true with the totals in out[] (valid in every thread of
// that workgroup), then rearms the counter.  The summation order does not
// depend on arrival order, so results are bitwise reproducible.
template <int W>
__device__ bool grid_sum(const double (&val)[W], double* part, unsigned* counter, double (&out)[W]) {
    __shared__ double red[kWaves];
    __shared__ int is_last;
    double bs[W];
#pragma unroll
    for (int w = 0; w < W; ++w) bs[w] = block_sum(val[w], red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) part[(size_t)blockIdx.x * W + w] = bs[w];
        __threadfence();
        unsigned ticket = atomicAdd(counter, 1u);
        is_last = (ticket == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    const int G = gridDim.x;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        double s = 0.0;
        for (int g = threadIdx.x; g < G; g += kBlock) s += part[(size_t)g * W + w];
        out[w] = block_sum(s, red);
    }
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

// Sum of W partials per producer workgroup written by the previous kernel in
// the stream (part[g * W + w], g < nparts), in a fixed order; every thread of
// the calling workgroup gets the totals.  The kernel boundary makes the
// producer's plain stores visible on every XCD, so no fence is needed and
// each consumer workgroup computes bitwise-identical totals.  Loads are
// issued several producers at a time so their latencies overlap.
template <int W>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nparts, double (&out)[W]) {
    __shared__ double red[kWaves];
    double s[W];
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] = 0.0;
    const int stride = blockDim.x;
    constexpr int U = (W >= 4) ? 2 : 8;
    for (int g0 = threadIdx.x; g0 < nparts; g0 += U * stride) {
        double t[U][W];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = g0 + u * stride;
#pragma unroll
            for (int w = 0; w < W; ++w) t[u][w] = (g < nparts) ? part[(size_t)g * W + w] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int w = 0; w < W; ++w) s[w] += t[u][w];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = (blockDim.x == kBlock) ? block_sum(s[w], red) : wave_sum(s[w]);
}

// Store this workgroup's W partial sums (thread 0 writes after the block sums).
template <int W>
__device__ __forceinline__ void write_partials(const double (&val)[W], double* part) {
    __shared__ double red[kWaves];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const double bs = block_sum(val[w], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * W + w] = bs;
    }
}

// LDS ordering among the lanes of one wave (a wave executes its LDS
// operations in order; the barrier keeps the compiler from reordering).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------- 4-row vector access
// Streaming kernels walk their rows in aligned quads (4 consecutive rows),
// so FP32 data moves as 16-byte loads/stores and FP64 data as two 16-byte
// accesses.  Every array starts 256-byte aligned and column strides are
// multiples of 64 elements, so a quad at row 4i is always 16-byte aligned.
// m < 4 marks the tail quad, handled element by element.
__device__ __forceinline__ void ld4(const float* p, int m, double (&o)[4]) {
    if (m == 4) {
        const float4 t = *reinterpret_cast<const float4*>(p);
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = (j < m) ? (double)p[j] : 0.0;
    }
}
__device__ __forceinline__ void ld4(const double* p, int m, double (&o)[4]) {
    if (m == 4) {
        const double2 a = reinterpret_cast<const double2*>(p)[0];
        const double2 b = reinterpret_cast<const double2*>(p)[1];
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = (j < m) ? p[j] : 0.0;
    }
}
// Stores round to the array's type; the rounded values are returned in v.
__device__ __forceinline__ void st4(float* p, int m, double (&v)[4]) {
    float t[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { t[j] = (float)v[j]; v[j] = (double)t[j]; }
    if (m == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(t[0], t[1], t[2], t[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) if (j < m) p[j] = t[j];
    }
}
__device__ __forceinline__ void st4(double* p, int m, double (&v)[4]) {
    if (m == 4) {
        reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
        reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) if (j < m) p[j] = v[j];
    }
}

// ---------------------------------------------------------------- Philox4x64-10
// J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11: 10 rounds of the 4x64 S-box
// (two 64x64 -> 128 multiplications, key added by XOR) with a Weyl key bump.
struct u64x4 { uint64_t x0, x1, x2, x3; };

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 c, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c.x0), lo0 = M0 * c.x0;
        const uint64_t hi1 = __umul64hi(M1, c.x2), lo1 = M1 * c.x2;
        c = u64x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Four standard normals: block `blk` of stream (seed; index, instance,
// purpose).  Box-Muller on 53-bit uniforms u1 in (0, 1], u2 in [0, 1):
// (r cos th, r sin th), r = sqrt(-2 log u1), th = 2 pi u2.
__device__ __forceinline__ void normal4(uint64_t seed, uint64_t blk, uint64_t index, uint64_t instance,
                                        uint64_t purpose, double out[4]) {
    const u64x4 x = philox4x64_10(u64x4{blk, index, instance, purpose}, seed, 0ull);
    const double two_pi = 2.0 * 3.141592653589793;  // 2*pi in double, as 2.0 * pi
    const double s53 = 0x1p-53;
    {
        const double u1 = ((double)(x.x0 >> 11) + 1.0) * s53;
        const double u2 = (double)(x.x1 >> 11) * s53;
        const double r = sqrt(-2.0 * log(u1));
        const double th = two_pi * u2;
        out[0] = r * cos(th);
        out[1] = r * sin(th);
    }
    {
        const double u1 = ((double)(x.x2 >> 11) + 1.0) * s53;
        const double u2 = (double)(x.x3 >> 11) * s53;
        const double r = sqrt(-2.0 * log(u1));
        const double th = two_pi * u2;
        out[2] = r * cos(th);
        out[3] = r * sin(th);
    }
}

// Quad 4 qd .. 4 qd + 3 of column c of the Gaussian test matrix Omega, drawn
// from Philox (seed; quad, column, instance, purpose 1) exactly as it is when
// stored, rounded to the storage type T; zeros past the m rows that exist.
template <typename T>
__device__ __forceinline__ void omega_quad(uint64_t seed, uint64_t instance, int64_t qd, int c, int m,
                                           double (&o)[4]) {
    double g[4];
    normal4(seed, (uint64_t)qd, (uint64_t)c, instance, 1ull, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (j < m) ? (double)(T)g[j] : 0.0;
}
template <typename T>
__device__ __forceinline__ double omega_entry(uint64_t seed, uint64_t instance, int64_t r, int c) {
    double g[4];
    normal4(seed, (uint64_t)(r >> 2), (uint64_t)c, instance, 1ull, g);
    return (double)(T)g[r & 3];
}

}  // namespace scg
