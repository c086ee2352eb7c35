// Vector quantisation of the SH coefficients (the post-processing of Sec. 5:
// each Gaussian's 16 x 3 SH coefficients are replaced by a codebook entry).
// Lloyd's k-means over the 48-vectors (basis-major, then channel):
//   assign: a(i) = argmin_j ||x_i - c_j||^2, equal distances to the lower j;
//   update: c_j = mean of the x_i with a(i) = j; an empty cluster keeps c_j.
// The assignment is a thread per Gaussian against codebook tiles staged in LDS
// (every lane reads the same entry: LDS broadcasts), distances accumulated in
// float32 in component order.  The update sorts (cluster, index) pairs with
// the stable radix sort, so each cluster's members are contiguous and in
// index order, and sums them in float64 in that order: deterministic, and the
// float32 mean is within one rounding of the exact one.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kD = 48;        // coefficients per vector
constexpr int kNT = 256;
constexpr int kTile = 64;     // codebook entries per LDS tile

// code[j][d] = sh plane d at Gaussian init[j] (indices clamped into the model)
__global__ void __launch_bounds__(kNT) vq_gather_kernel(const float *sh, int64_t n, const uint32_t *init,
                                                        int64_t k, float *code) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= k * kD) return;
    const int64_t j = i / kD;
    const int d = (int)(i % kD);
    const int64_t g = min((int64_t)init[j], n - 1);
    code[i] = sh[(int64_t)d * n + g];
}

__global__ void __launch_bounds__(kNT) vq_assign_kernel(const float *sh, int64_t n, const float *code, int64_t k,
                                                        uint32_t *assign) {
    __shared__ float4 s_c[kTile * kD / 4];
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    const int64_t gi = min(i, n - 1);
    float x[kD];
#pragma unroll
    for (int d = 0; d < kD; ++d) x[d] = sh[(int64_t)d * n + gi];
    float best = INFINITY;
    uint32_t bj = 0;
    for (int64_t j0 = 0; j0 < k; j0 += kTile) {
        const int cnt = (int)min((int64_t)kTile, k - j0);
        __syncthreads();
        const float4 *src = reinterpret_cast<const float4 *>(code + j0 * kD);
        for (int e = threadIdx.x; e < cnt * kD / 4; e += kNT) s_c[e] = src[e];
        __syncthreads();
        for (int jj = 0; jj < cnt; ++jj) {
            const float4 *c = s_c + jj * (kD / 4);
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < kD / 4; ++q) {
                const float4 v = c[q];
                float t = x[4 * q] - v.x;
                acc = fmaf(t, t, acc);
                t = x[4 * q + 1] - v.y;
                acc = fmaf(t, t, acc);
                t = x[4 * q + 2] - v.z;
                acc = fmaf(t, t, acc);
                t = x[4 * q + 3] - v.w;
                acc = fmaf(t, t, acc);
            }
            if (acc < best) {
                best = acc;
                bj = (uint32_t)(j0 + jj);
            }
        }
    }
    if (i < n) assign[i] = bj;
}

__global__ void __launch_bounds__(kNT) vq_keys_kernel(const uint32_t *assign, int64_t n, uint32_t *keys,
                                                      uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    keys[i] = assign[i];
    vals[i] = (uint32_t)i;
}

// Block j (kD threads, one per component): float64 sum of cluster j's members
// in index order; an empty cluster keeps its vector.
__global__ void __launch_bounds__(64) vq_update_kernel(const float *sh, int64_t n, const uint32_t *members,
                                                       const uint32_t *ranges, float *code) {
    const int d = threadIdx.x;
    if (d >= kD) return;
    const uint32_t s = ranges[2 * blockIdx.x], e = ranges[2 * blockIdx.x + 1];
    if (e <= s) return;
    double acc = 0.0;
    for (uint32_t m = s; m < e; ++m) acc += (double)sh[(int64_t)d * n + min((int64_t)members[m], n - 1)];
    code[(int64_t)blockIdx.x * kD + d] = (float)(acc / (double)(e - s));
}

inline unsigned blocks(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

size_t vq_scratch_bytes(int64_t n, int64_t k) {
    // keys, vals and their alternates, cluster ranges, radix scratch
    return sizeof(uint32_t) * (size_t)(4 * n + 2 * k) + sort_scratch_bytes(n) + 256;
}

hipError_t vq_kmeans(const float *sh, int64_t n, const uint32_t *init, int64_t k, int32_t iterations, float *code,
                     uint32_t *assign, void *scratch, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    uint32_t *keys = static_cast<uint32_t *>(scratch);
    uint32_t *vals = keys + n, *keys2 = vals + n, *vals2 = keys2 + n, *ranges = vals2 + n;
    void *sort_scratch = reinterpret_cast<void *>((reinterpret_cast<uintptr_t>(ranges + 2 * k) + 255) & ~uintptr_t(255));
    hipLaunchKernelGGL(vq_gather_kernel, dim3(blocks(k * kD, kNT)), dim3(kNT), 0, s, sh, n, init, k, code);
    for (int32_t it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(vq_assign_kernel, dim3(blocks(n, kNT)), dim3(kNT), 0, s, sh, n, (const float *)code, k,
                           assign);
        hipLaunchKernelGGL(vq_keys_kernel, dim3(blocks(n, kNT)), dim3(kNT), 0, s, (const uint32_t *)assign, n, keys,
                           vals);
        int alt = 0;
        int bits = 1;
        while (bits < 32 && (int64_t(1) << bits) < k) ++bits;
        hipError_t e = radix_sort_u32(keys, vals, keys2, vals2, nullptr, n, 0, bits, sort_scratch, &alt, s);
        if (e != hipSuccess) return e;
        const uint32_t *sk = alt ? keys2 : keys, *sv = alt ? vals2 : vals;
        e = launch_tile_ranges(sk, nullptr, n, (int32_t)k, ranges, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(vq_update_kernel, dim3((unsigned)k), dim3(64), 0, s, sh, n, sv,
                           (const uint32_t *)ranges, code);
    }
    hipLaunchKernelGGL(vq_assign_kernel, dim3(blocks(n, kNT)), dim3(kNT), 0, s, sh, n, (const float *)code, k, assign);
    return hipGetLastError();
}

}  // namespace fdgs
