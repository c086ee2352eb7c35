// Device-wide exclusive scans (reduce, scan of block sums, downsweep) and the
// ballot-based compaction of active-set bits into ascending indices.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kNT = 256;         // threads per block
constexpr int kItems = 4;        // items per thread: 1024-item chunks, so a frame's ~130k entries
                                 // spread over ~130 workgroups (offsets 16.2 -> 12.4 us against 8)
constexpr int kChunk = kNT * kItems;
constexpr int kTopNT = 1024;

__device__ __forceinline__ int64_t count_of(const int64_t *n_dev, int64_t n_max) {
    return n_dev ? min(*n_dev, n_max) : n_max;
}

// Loader for the scanned value of element j: flags (u8) or u32 counts,
// optionally read through a gather index.  A thread whose first element lies
// past the count loads nothing; otherwise its element indices are clamped to
// the last counted element (so a gather only follows indices that were
// written) and the values past the count are masked to zero afterwards.  The
// loads of all items then carry no branch and are issued together (a gather
// issues its index loads, then its value loads).
struct LoadU8 {
    const uint8_t *in;
    template <int K>
    __device__ __forceinline__ void load(const int64_t (&j)[K], uint64_t (&v)[K]) const {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = in[j[k]];
    }
};
struct LoadU32 {
    const uint32_t *in;
    const uint32_t *gather;
    template <int K>
    __device__ __forceinline__ void load(const int64_t (&j)[K], uint64_t (&v)[K]) const {
        if (gather) {
            uint32_t g[K];
#pragma unroll
            for (int k = 0; k < K; ++k) g[k] = gather[j[k]];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = in[g[k]];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = in[j[k]];
        }
    }
};

// The thread's kItems consecutive elements starting at base, zero past n.
template <typename Load>
__device__ __forceinline__ void load_items(const Load &ld, int64_t base, int64_t n, uint64_t (&v)[kItems]) {
    if (base >= n) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = 0;
        return;
    }
    int64_t j[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) j[k] = min(base + k, n - 1);
    ld.load(j, v);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k >= n) v[k] = 0;
}

template <typename Load>
__global__ void __launch_bounds__(kNT) reduce_kernel(Load ld, const int64_t *n_dev, int64_t n_max,
                                                     uint64_t *partial) {
    __shared__ uint64_t tmp[kNT / 64 + 1];
    const int64_t n = count_of(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
    uint64_t v[kItems];
    load_items(ld, base, n, v);
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += v[k];
    uint64_t total;
    block_exclusive_sum<kNT>(s, tmp, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of nb block sums by one block; writes the grand total.
// Optionally clears n_clear words and resets a [min, max] key range to
// (all ones, 0) for the kernel that follows.  With group_in, block sum j is
// instead the sum of group_in[j * group .. j * group + group) (entries past
// n_in count as 0), written to partial[j] before the scan.
__global__ void __launch_bounds__(kTopNT) top_scan_kernel(uint64_t *partial, int64_t nb, int64_t *total,
                                                          uint32_t *clear, int64_t n_clear, uint32_t *range,
                                                          const uint32_t *group_in, int64_t n_in, int group) {
    __shared__ uint64_t tmp[kTopNT / 64 + 1];
    for (int64_t i = threadIdx.x; i < n_clear; i += kTopNT) clear[i] = 0u;
    if (range && threadIdx.x == 0) {
        range[0] = ~0u;
        range[1] = 0u;
    }
    uint64_t carry = 0;
    for (int64_t start = 0; start < nb; start += kTopNT) {
        const int64_t j = start + threadIdx.x;
        uint64_t v = 0;
        if (j < nb) {
            if (group_in) {
                for (int g = 0; g < group; ++g) {
                    const int64_t i = j * group + g;
                    if (i < n_in) v += group_in[i];
                }
            } else {
                v = partial[j];
            }
        }
        uint64_t tot;
        const uint64_t ex = block_exclusive_sum<kTopNT>(v, tmp, &tot);
        if (j < nb) partial[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = (int64_t)carry;
}

template <typename Load, typename Out>
__global__ void __launch_bounds__(kNT) downsweep_kernel(Load ld, const int64_t *n_dev, int64_t n_max,
                                                        const uint64_t *partial, Out *out) {
    __shared__ uint64_t tmp[kNT / 64 + 1];
    const int64_t n = count_of(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
    uint64_t v[kItems];
    load_items(ld, base, n, v);
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) s += v[k];
    uint64_t total;
    uint64_t run = block_exclusive_sum<kNT>(s, tmp, &total) + partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) out[base + k] = (Out)run;
        run += v[k];
    }
}

template <typename Load, typename Out>
hipError_t scan_impl(Load ld, Out *out, const int64_t *n_dev, int64_t n_max, int64_t *total,
                     void *scratch, hipStream_t s) {
    const int64_t nb = (n_max + kChunk - 1) / kChunk;
    uint64_t *partial = static_cast<uint64_t *>(scratch);
    if (nb == 0) {
        // still define the total
        hipLaunchKernelGGL(top_scan_kernel, dim3(1), dim3(kTopNT), 0, s, partial, (int64_t)0, total,
                           (uint32_t *)nullptr, (int64_t)0, (uint32_t *)nullptr,
                           (const uint32_t *)nullptr, (int64_t)0, 1);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((reduce_kernel<Load>), dim3((unsigned)nb), dim3(kNT), 0, s, ld, n_dev, n_max, partial);
    hipLaunchKernelGGL(top_scan_kernel, dim3(1), dim3(kTopNT), 0, s, partial, nb, total, (uint32_t *)nullptr,
                       (int64_t)0, (uint32_t *)nullptr, (const uint32_t *)nullptr, (int64_t)0, 1);
    hipLaunchKernelGGL((downsweep_kernel<Load, Out>), dim3((unsigned)nb), dim3(kNT), 0, s, ld, n_dev,
                       n_max, (const uint64_t *)partial, out);
    return hipGetLastError();
}

// Visible compaction: the downsweep of a scan over the visible flags that
// writes each visible entry's (float32 depth bits, position) to its slot and,
// when range is given, folds the keys into range = [min, max] (positive
// floats: bit order is value order).
__global__ void __launch_bounds__(kNT) compact_visible_kernel(const uint8_t *visible, const uint64_t *depth_key,
                                                              const int64_t *n_dev, int64_t n_max,
                                                              const uint64_t *partial, uint32_t *keys32,
                                                              uint32_t *vals, uint32_t *asc, uint32_t *range) {
    __shared__ uint64_t tmp[kNT / 64 + 1];
    const int64_t n = count_of(n_dev, n_max);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = base + k < n ? visible[base + k] : 0u;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = block_exclusive_sum<kNT>(s, tmp, &total) + partial[blockIdx.x];
    uint32_t kmin = ~0u, kmax = 0u;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (v[k]) {
            const double z = __longlong_as_double((long long)depth_key[base + k]);
            const uint32_t key = __float_as_uint((float)z);   // z > 0: bit order = value order
            keys32[run] = key;
            vals[run] = (uint32_t)(base + k);
            if (asc) asc[run] = (uint32_t)(base + k);
            kmin = min(kmin, key);
            kmax = max(kmax, key);
            ++run;
        }
    }
    if (range) {
        // block minimum and maximum, then one atomic pair per block
        __shared__ uint32_t s_min[kNT / 64], s_max[kNT / 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
        }
        if (lane_id() == 0) {
            s_min[wave_id()] = kmin;
            s_max[wave_id()] = kmax;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
#pragma unroll
            for (int w = 1; w < kNT / 64; ++w) {
                kmin = min(kmin, s_min[w]);
                kmax = max(kmax, s_max[w]);
            }
            if (kmin <= kmax) {
                atomicMin(&range[0], kmin);
                atomicMax(&range[1], kmax);
            }
        }
    }
}

// --- compaction of active-set bits -----------------------------------------
// Each block covers kChunk Gaussians (kChunk/32 bit words).
// Bits at positions >= n (the tail of the last word) are not counted, as the
// compaction does not emit them.
__global__ void __launch_bounds__(kNT) bits_count_kernel(const uint32_t *bits, int64_t n, int64_t nw,
                                                         uint64_t *partial) {
    __shared__ uint64_t tmp[kNT / 64 + 1];
    constexpr int kWords = kChunk / 32;
    const int64_t w0 = (int64_t)blockIdx.x * kWords;
    const uint32_t tail = (n & 31) ? ((1u << (n & 31)) - 1u) : 0xffffffffu;
    uint64_t c = 0;
    for (int k = threadIdx.x; k < kWords; k += kNT)
        if (w0 + k < nw) c += __popc(bits[w0 + k] & (w0 + k == nw - 1 ? tail : 0xffffffffu));
    uint64_t total;
    block_exclusive_sum<kNT>(c, tmp, &total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Thread t of round r handles Gaussian g = block_base + r*kNT + t.  A wave's
// keep bits come from one ballot; a lane's rank is the popcount of the bits
// below it (mbcnt); wave counts are combined through shared memory, so the
// output stays in ascending order.
__global__ void __launch_bounds__(kNT) bits_compact_kernel(const uint32_t *bits, int64_t n,
                                                           const uint64_t *partial, uint32_t *idx) {
    __shared__ uint64_t tmp[kNT / 64 + 1];
    uint64_t run = partial[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int r = 0; r < kItems; ++r) {
        const int64_t g = base + (int64_t)r * kNT + threadIdx.x;
        const bool keep = g < n && ((bits[g >> 5] >> (g & 31)) & 1u);
        const uint64_t ballot = __ballot(keep);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
        const uint64_t wcount = __popcll(ballot);
        if (lane_id() == 0) tmp[wave_id()] = wcount;
        __syncthreads();
        uint64_t before = 0, round_total = 0;
        for (int w = 0; w < kNT / 64; ++w) {
            if (w < wave_id()) before += tmp[w];
            round_total += tmp[w];
        }
        if (keep) idx[run + before + rank] = (uint32_t)g;
        run += round_total;
        __syncthreads();
    }
}

// Population counts of two active-set bit arrays and of their intersection
// (one workgroup; a few hundred thousand words at most, so one pass of
// coalesced loads and a block reduction is enough).  Bits past n in the last
// word are ignored.
constexpr int kOverlapNT = 1024;
__global__ void __launch_bounds__(kOverlapNT) mask_overlap_kernel(const uint32_t *a, const uint32_t *b, int64_t n,
                                                                  int64_t *out) {
    __shared__ uint64_t tmp[kOverlapNT / 64 + 1];
    const int64_t nw = (n + 31) / 32;
    const uint32_t tail = (n & 31) ? ((1u << (n & 31)) - 1u) : 0xffffffffu;
    uint64_t ca = 0, cb = 0, cab = 0;
    for (int64_t w = threadIdx.x; w < nw; w += kOverlapNT) {
        const uint32_t m = w == nw - 1 ? tail : 0xffffffffu;
        const uint32_t x = a[w] & m, y = b[w] & m;
        ca += __popc(x);
        cb += __popc(y);
        cab += __popc(x & y);
    }
    uint64_t ta, tb, tab;
    block_exclusive_sum<kOverlapNT>(ca, tmp, &ta);
    block_exclusive_sum<kOverlapNT>(cb, tmp, &tb);
    block_exclusive_sum<kOverlapNT>(cab, tmp, &tab);
    if (threadIdx.x == 0) {
        out[0] = (int64_t)ta;
        out[1] = (int64_t)tb;
        out[2] = (int64_t)tab;
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n_max) {
    return sizeof(uint64_t) * (size_t)((n_max + kChunk - 1) / kChunk + 1);
}

size_t compact_scratch_bytes(int64_t n) { return scan_scratch_bytes(n); }

hipError_t scan_flags_u8(const uint8_t *in, uint32_t *out, const int64_t *n_dev, int64_t n_max,
                         int64_t *total, void *scratch, hipStream_t s) {
    return scan_impl(LoadU8{in}, out, n_dev, n_max, total, scratch, s);
}

hipError_t scan_u32_to_u64(const uint32_t *in, const uint32_t *gather, uint64_t *out,
                           const int64_t *n_dev, int64_t n_max, int64_t *total, void *scratch,
                           hipStream_t s) {
    return scan_impl(LoadU32{in, gather}, out, n_dev, n_max, total, scratch, s);
}

hipError_t compact_visible(const uint8_t *visible, const uint64_t *depth_key, const int64_t *n_dev, int64_t n_max,
                           int64_t *total, uint32_t *keys32, uint32_t *vals, uint32_t *asc, uint32_t *clear,
                           int64_t n_clear, uint32_t *range, void *scratch, hipStream_t s,
                           const uint32_t *vis_count) {
    static_assert(kChunk % kPreprocessBlock == 0, "whole preprocess workgroups per scan chunk");
    const int64_t nb = (n_max + kChunk - 1) / kChunk;
    uint64_t *partial = static_cast<uint64_t *>(scratch);
    if (vis_count) {
        // the preprocess counted each workgroup's visible entries: sum them per chunk in the scan
        const int64_t n_in = (n_max + kPreprocessBlock - 1) / kPreprocessBlock;
        hipLaunchKernelGGL(top_scan_kernel, dim3(1), dim3(kTopNT), 0, s, partial, nb, total, clear, n_clear, range,
                           vis_count, n_in, kChunk / kPreprocessBlock);
    } else {
        if (nb > 0)
            hipLaunchKernelGGL((reduce_kernel<LoadU8>), dim3((unsigned)nb), dim3(kNT), 0, s, LoadU8{visible}, n_dev,
                               n_max, partial);
        hipLaunchKernelGGL(top_scan_kernel, dim3(1), dim3(kTopNT), 0, s, partial, nb, total, clear, n_clear, range,
                           (const uint32_t *)nullptr, (int64_t)0, 1);
    }
    if (nb > 0)
        hipLaunchKernelGGL(compact_visible_kernel, dim3((unsigned)nb), dim3(kNT), 0, s, visible, depth_key, n_dev,
                           n_max, (const uint64_t *)partial, keys32, vals, asc, range);
    return hipGetLastError();
}

hipError_t compact_bits(const uint32_t *bits, int64_t n, uint32_t *idx, int64_t *count,
                        void *scratch, hipStream_t s) {
    const int64_t nb = (n + kChunk - 1) / kChunk;
    uint64_t *partial = static_cast<uint64_t *>(scratch);
    const int64_t nw = (n + 31) / 32;
    if (nb > 0)
        hipLaunchKernelGGL(bits_count_kernel, dim3((unsigned)nb), dim3(kNT), 0, s, bits, n, nw, partial);
    hipLaunchKernelGGL(top_scan_kernel, dim3(1), dim3(kTopNT), 0, s, partial, nb, count, (uint32_t *)nullptr,
                       (int64_t)0, (uint32_t *)nullptr, (const uint32_t *)nullptr, (int64_t)0, 1);
    if (nb > 0)
        hipLaunchKernelGGL(bits_compact_kernel, dim3((unsigned)nb), dim3(kNT), 0, s, bits, n,
                           (const uint64_t *)partial, idx);
    return hipGetLastError();
}

}  // namespace fdgs

namespace fdgs {

hipError_t launch_mask_overlap(const uint32_t *a, const uint32_t *b, int64_t n, int64_t *out, hipStream_t s) {
    hipLaunchKernelGGL(mask_overlap_kernel, dim3(1), dim3(kOverlapNT), 0, s, a, b, n, out);
    return hipGetLastError();
}

}  // namespace fdgs
