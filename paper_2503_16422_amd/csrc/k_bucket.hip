// Depth order of the visible Gaussians of one view by bucketing (Eq. 2 blends
// "sorted by depth"; the order is (float64 depth, processing position)).
//
// A frame of a few hundred thousand Gaussians is far too small for a
// multi-pass radix sort to be bound by anything but its launches (three per
// digit pass).  Here three kernels produce the same order:
//   1. count: each visible key (float32 depth bits, a monotone image of the
//      float64 depth) falls into one of NB buckets spread linearly over the
//      frame's [min, max] key range (found by the compaction); per-block LDS
//      counts, one global add per non-empty bucket.
//   2. scatter: every block scans the NB counts itself (no separate scan
//      launch), reserves a contiguous slot range per bucket with one global
//      add per non-empty bucket, and writes its positions there.  The order
//      inside a bucket depends on the scheduling and is repaired by 3.
//   3. sort: one block per bucket sorts its positions by (float64 depth bits,
//      position) -- a strict total order, so the result is unique and no tie
//      repair is needed -- by ranking them in LDS.  A bucket larger
//      than the LDS tile (many Gaussians at one depth) is sorted in LDS-sized
//      chunks that the block then merges pairwise through a second buffer
//      (each output element placed by a binary search of its co-rank).
// The bucket map is monotone in the key, so buckets in index order hold
// increasing depths and the concatenation of the sorted buckets is the
// sorted sequence.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kNT = 256;
constexpr int kKeysPerThread = 4;   // 1024 keys per counting / scattering workgroup
constexpr int kChunk = kNT * kKeysPerThread;
constexpr int kSortNT = 256;
constexpr int kCap = 2048;                 // positions a block sorts in LDS at once

__device__ __forceinline__ int64_t count_of(const int64_t *n_dev, int64_t n_max) {
    return n_dev ? min(*n_dev, n_max) : n_max;
}

// Monotone map of a key in [kmin, kmax] to [0, nb).
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, uint32_t kmin, double scale, uint32_t nb) {
    const double x = fmin((double)(key - kmin) * scale, (double)(nb - 1u));
    return (uint32_t)x;
}

__device__ __forceinline__ double bucket_scale(const uint32_t *zrange, uint32_t nb) {
    const uint32_t kmin = zrange[0], kmax = zrange[1];
    return kmax >= kmin ? (double)nb / ((double)(kmax - kmin) + 1.0) : 0.0;
}

__global__ void __launch_bounds__(kNT) bucket_count_kernel(const uint32_t *keys32, const int64_t *n_dev,
                                                           int64_t n_max, const uint32_t *zrange, uint32_t nb,
                                                           uint32_t *count) {
    extern __shared__ uint32_t s_cnt[];
    const int64_t n = count_of(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= n) return;                                   // uniform
    for (uint32_t b = threadIdx.x; b < nb; b += kNT) s_cnt[b] = 0;
    const uint32_t kmin = zrange[0];
    const double scale = bucket_scale(zrange, nb);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeysPerThread; ++r) {
        const int64_t j = base + (int64_t)r * kNT + threadIdx.x;
        if (j < n) atomicAdd(&s_cnt[bucket_of(keys32[j], kmin, scale, nb)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kNT)
        if (s_cnt[b]) atomicAdd(&count[b], s_cnt[b]);
}

// Every block scans the bucket counts into s_start (exclusive); block 0 also
// publishes them (start[nb] = total) for the sort.  Loads and the returning
// cursor atomics are issued in batches before their results are used.
constexpr int kMaxPer = 4096 / kNT;      // buckets per thread at the largest nb

__global__ void __launch_bounds__(kNT) bucket_scatter_kernel(const uint32_t *keys32, const uint32_t *vals,
                                                             const int64_t *n_dev, int64_t n_max,
                                                             const uint32_t *zrange, uint32_t nb,
                                                             const uint32_t *count, uint32_t *cursor,
                                                             uint32_t *start, uint32_t *out) {
    extern __shared__ uint32_t s_mem[];
    uint32_t *s_start = s_mem;          // [nb]
    uint32_t *s_loc = s_mem + nb;       // [nb]: block-local count, then the block's slot base
    __shared__ uint32_t s_tmp[kNT / 64 + 1];
    const int64_t n = count_of(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    if (base >= n && blockIdx.x != 0) return;                // uniform; block 0 always publishes
    // exclusive scan of the counts: thread t owns the contiguous slice [t * per, (t + 1) * per)
    const uint32_t per = nb >= (uint32_t)kNT ? nb / kNT : 1u;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t c[kMaxPer];
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) c[k] = count[min(b0 + (uint32_t)k, nb - 1u)];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
        if ((uint32_t)k < per && b0 + k < nb) sum += c[k];
    uint32_t total;
    uint32_t run = block_exclusive_sum<kNT>(sum, s_tmp, &total);
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
        if ((uint32_t)k < per && b0 + k < nb) {
            s_start[b0 + k] = run;
            run += c[k];
        }
    for (uint32_t b = threadIdx.x; b < nb; b += kNT) s_loc[b] = 0;
    __syncthreads();
    if (blockIdx.x == 0) {
        for (uint32_t b = threadIdx.x; b < nb; b += kNT) start[b] = s_start[b];
        if (threadIdx.x == 0) start[nb] = total;
    }
    if (base >= n) return;                                   // uniform (block 0 only)
    const uint32_t kmin = zrange[0];
    const double scale = bucket_scale(zrange, nb);
    uint32_t bk[kKeysPerThread], rank[kKeysPerThread];
#pragma unroll
    for (int r = 0; r < kKeysPerThread; ++r) {
        const int64_t j = base + (int64_t)r * kNT + threadIdx.x;
        bk[r] = j < n ? bucket_of(keys32[j], kmin, scale, nb) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kKeysPerThread; ++r) {
        const int64_t j = base + (int64_t)r * kNT + threadIdx.x;
        rank[r] = j < n ? atomicAdd(&s_loc[bk[r]], 1u) : 0u;
    }
    __syncthreads();
    // thread t reserves the slots of buckets t, t + kNT, ...
    uint32_t lc[kMaxPer], lb[kMaxPer];
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const uint32_t b = threadIdx.x + (uint32_t)k * kNT;
        lc[k] = b < nb ? s_loc[b] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const uint32_t b = threadIdx.x + (uint32_t)k * kNT;
        lb[k] = lc[k] ? atomicAdd(&cursor[b], lc[k]) : 0u;
    }
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k) {
        const uint32_t b = threadIdx.x + (uint32_t)k * kNT;
        if (b < nb) s_loc[b] = s_start[b] + lb[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeysPerThread; ++r) {
        const int64_t j = base + (int64_t)r * kNT + threadIdx.x;
        const uint32_t slot = s_loc[bk[r]] + rank[r];
        if (j < n && slot < (uint64_t)n) out[slot] = vals[j];
    }
}

// (depth bits, position) order; positions are distinct, so it is strict.
__device__ __forceinline__ bool before(uint64_t da, uint32_t pa, uint64_t db, uint32_t pb) {
    return da < db || (da == db && pa < pb);
}

// One block sorts m <= kCap (key, position) pairs held in LDS by rank:
// element e goes to the number of elements that precede it.  The order is
// strict, so the ranks are a permutation.  Every thread compares its own
// elements (e = t + kSortNT r) against all m, eight at a time from LDS
// broadcasts: m^2 / kSortNT compares per thread and two barriers, which for
// buckets of tens to a few hundred entries is far cheaper than a sorting
// network's barrier-separated steps.  Entries [m, m rounded up to 8) are set
// to (all ones, all ones), which precede nothing.
template <int R>
__device__ __forceinline__ void rank_sort_r(const uint64_t *s_key, const uint32_t *s_pos, int m, uint32_t *dst) {
    uint64_t ke[R];
    uint32_t pe[R], rk[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = (int)threadIdx.x + kSortNT * r;
        ke[r] = e < m ? s_key[e] : ~0ull;
        pe[r] = e < m ? s_pos[e] : ~0u;
        rk[r] = 0;
    }
    const int m8 = (m + 7) & ~7;
    for (int f0 = 0; f0 < m8; f0 += 8) {
        uint64_t kf[8];
        uint32_t pf[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            kf[u] = s_key[f0 + u];
            pf[u] = s_pos[f0 + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) rk[r] += before(kf[u], pf[u], ke[r], pe[r]) ? 1u : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if ((int)threadIdx.x + kSortNT * r < m) dst[rk[r]] = pe[r];
}

__device__ void rank_sort(uint64_t *s_key, uint32_t *s_pos, int m, uint32_t *dst) {
    for (int i = m + (int)threadIdx.x; i < ((m + 7) & ~7); i += kSortNT) {
        s_key[i] = ~0ull;
        s_pos[i] = ~0u;
    }
    __syncthreads();
    if (m <= kSortNT) rank_sort_r<1>(s_key, s_pos, m, dst);
    else if (m <= 2 * kSortNT) rank_sort_r<2>(s_key, s_pos, m, dst);
    else if (m <= 4 * kSortNT) rank_sort_r<4>(s_key, s_pos, m, dst);
    else rank_sort_r<kCap / kSortNT>(s_key, s_pos, m, dst);
}

// Block b sorts bucket b.
__global__ void __launch_bounds__(kSortNT) bucket_sort_kernel(const uint32_t *start, const uint32_t *bucketed,
                                                              const uint64_t *depth_key, int64_t n_max,
                                                              uint32_t *alt, uint32_t *out) {
    __shared__ uint64_t s_key[kCap + 8];
    __shared__ uint32_t s_pos[kCap + 8];
    const uint32_t lo = start[blockIdx.x], hi = (uint32_t)min((int64_t)start[blockIdx.x + 1], n_max);
    const int64_t m = (int64_t)hi - lo;
    if (m <= 0) return;
    const uint32_t last = (uint32_t)(n_max - 1);    // positions index depth_key[0, n_max)
    // sorted runs of kCap (all of the bucket when it fits)
    for (int64_t c0 = 0; c0 < m; c0 += kCap) {
        const int len = (int)min((int64_t)kCap, m - c0);
        for (int i = threadIdx.x; i < len; i += kSortNT) {
            const uint32_t pos = min(bucketed[lo + c0 + i], last);
            s_pos[i] = pos;
            s_key[i] = depth_key[pos];
        }
        rank_sort(s_key, s_pos, len, out + lo + c0);
        __syncthreads();
    }
    if (m <= kCap) return;
    // pairwise merges of runs of width w: output element i of a pair takes
    // the i-th smallest of the two runs, found by a binary search of how many
    // of them come from the first run
    uint32_t *src = out + lo, *dst = alt + lo;
    for (int64_t w = kCap; w < m; w <<= 1) {
        for (int64_t a0 = 0; a0 < m; a0 += 2 * w) {
            const int64_t la = min(w, m - a0);
            const int64_t lb = max((int64_t)0, min(w, m - a0 - w));
            const uint32_t *A = src + a0, *B = src + a0 + la;
            for (int64_t i = threadIdx.x; i < la + lb; i += kSortNT) {
                int64_t s = max((int64_t)0, i - lb), e = min(i, la);
                while (s < e) {
                    const int64_t mid = (s + e) >> 1;
                    const uint32_t pa = A[mid], pb = B[i - 1 - mid];
                    if (before(depth_key[pa], pa, depth_key[pb], pb)) s = mid + 1; else e = mid;
                }
                const int64_t ia = s, ib = i - s;
                uint32_t v;
                if (ib >= lb) v = A[ia];
                else if (ia >= la) v = B[ib];
                else {
                    const uint32_t pa = A[ia], pb = B[ib];
                    v = before(depth_key[pa], pa, depth_key[pb], pb) ? pa : pb;
                }
                dst[a0 + i] = v;
            }
        }
        __syncthreads();
        uint32_t *t = src; src = dst; dst = t;
    }
    if (src != out + lo)
        for (int64_t i = threadIdx.x; i < m; i += kSortNT) out[lo + i] = src[i];
}

}  // namespace

// About 64 positions per bucket, between 64 and 4096 buckets.
int bucket_log2_for(int64_t n_max) {
    int l = 6;
    while (l < 12 && (int64_t(1) << l) * 64 < n_max) ++l;
    return l;
}

size_t bucket_scratch_words(int64_t n_max) {
    const int64_t nb = int64_t(1) << bucket_log2_for(n_max);
    return (size_t)(3 * nb + 1 + 2);
}

hipError_t depth_order_buckets(const uint32_t *keys32, const uint32_t *vals, const int64_t *n_vis_dev, int64_t n_max,
                               const uint64_t *depth_key, uint32_t *work, uint32_t *alt, uint32_t *bucketed,
                               uint32_t *out, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    const uint32_t nb = 1u << bucket_log2_for(n_max);
    uint32_t *count = work, *cursor = work + nb, *start = work + 2 * nb, *zrange = work + 3 * nb + 1;
    const unsigned blocks = (unsigned)((n_max + kChunk - 1) / kChunk);
    hipLaunchKernelGGL(bucket_count_kernel, dim3(blocks), dim3(kNT), sizeof(uint32_t) * nb, s, keys32, n_vis_dev,
                       n_max, (const uint32_t *)zrange, nb, count);
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(blocks), dim3(kNT), 2 * sizeof(uint32_t) * nb, s, keys32, vals,
                       n_vis_dev, n_max, (const uint32_t *)zrange, nb, (const uint32_t *)count, cursor, start,
                       bucketed);
    hipLaunchKernelGGL(bucket_sort_kernel, dim3(nb), dim3(kSortNT), 0, s, (const uint32_t *)start,
                       (const uint32_t *)bucketed, depth_key, n_max, alt, out);
    return hipGetLastError();
}

}  // namespace fdgs
