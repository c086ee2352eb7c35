// Device helpers shared by the integer kernels: wave64 and block scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdgs {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// XCD-aware item of block b in a grid of n blocks.  Workgroups go to the
// eight XCDs (each with its own L2) round-robin by block index; here the
// blocks of one XCD take one contiguous range of items, so that neighbouring
// items -- which share cache lines of column-major histograms and of the runs
// a radix pass scatters -- are handled under one L2 and their partial-line
// writes merge there instead of reaching HBM separately.  A bijection of
// [0, n): XCD x takes n / 8 items, one more when x < n % 8.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t n) {
    constexpr int64_t kXcds = 8;
    const int64_t q = n / kXcds, r = n % kXcds, x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}

// Inclusive sum over the 64 lanes of a wavefront.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 64 lanes with DPP row operations (no LDS traffic); the total
// is valid in lane 63.  Steps: xor-1 and xor-2 inside quads, half-row mirror,
// row mirror (every lane now holds its 16-lane row sum), then row broadcasts
// 15 and 31 fold rows 0..3 into row 3.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_add_c(float v) {
    const int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, true);
    return v + __builtin_bit_cast(float, o);
}
// Sum over each row of 16 lanes, valid in every lane of the row: the first
// four steps of the wavefront sum.
__device__ __forceinline__ float row_sum16(float v) {
    v = dpp_add_c<0xB1>(v);          // quad_perm(1,0,3,2)
    v = dpp_add_c<0x4E>(v);          // quad_perm(2,3,0,1)
    v = dpp_add_c<0x141>(v);         // row_half_mirror
    v = dpp_add_c<0x140>(v);         // row_mirror
    return v;
}
__device__ __forceinline__ float wave_sum_to_last(float v) {
    v = dpp_add_c<0xB1>(v);          // quad_perm(1,0,3,2)
    v = dpp_add_c<0x4E>(v);          // quad_perm(2,3,0,1)
    v = dpp_add_c<0x141>(v);         // row_half_mirror
    v = dpp_add_c<0x140>(v);         // row_mirror
    v = dpp_add_c<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_add_c<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

// Exclusive sum over a block of NT threads (NT a multiple of 64, <= 1024).
// `tmp` must hold NT/64 + 1 elements of shared memory.  Returns the thread's
// exclusive prefix; *total receives the block total.  Contains barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T *tmp, T *total) {
    constexpr int NW = NT / 64;
    const T inc = wave_inclusive_sum(v);
    if (lane_id() == 63) tmp[wave_id()] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            const T x = tmp[w];
            tmp[w] = run;
            run += x;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    const T res = tmp[wave_id()] + inc - v;
    *total = tmp[NW];
    __syncthreads();
    return res;
}

}  // namespace fdgs
