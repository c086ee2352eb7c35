// Host emulation of the HIP device API, for checking kernels on the CPU (test
// infrastructure only).  A block runs on std::threads, one per work-item, and
// blocks run one after another, so __shared__ variables can be function
// statics; __syncthreads is a std::barrier over the block; wavefront
// shuffles and ballots go through a per-wavefront exchange buffer with a
// barrier over its 64 work-items; atomics are std::atomic_ref.  A work-item
// that returns drops out of every barrier, as an exited wavefront does.
// Dynamic shared memory (extern __shared__) is provided as g_dyn_lds, sized by
// the launch, so that AddressSanitizer sees its bounds.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define HIP_SYMBOL(x) (&x)

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef void *hipStream_t;
inline hipError_t hipGetLastError() { return hipSuccess; }

struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
struct int2 { int x, y; };
struct int4 { int x, y, z, w; };
struct uint4 { unsigned x, y, z, w; };
struct double2 { double x, y; };
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return uint4{x, y, z, w}; }
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct Idx3 { unsigned x = 0, y = 0, z = 0; };
inline thread_local Idx3 threadIdx;
inline thread_local Idx3 blockIdx;
inline Idx3 blockDim, gridDim;
inline std::barrier<> *g_block_barrier = nullptr;
inline char *g_dyn_lds = nullptr;

struct WaveX {
    std::unique_ptr<std::barrier<>> bar;
    uint64_t v[64];
};
inline std::vector<std::unique_ptr<WaveX>> g_waves;

inline void __syncthreads() { g_block_barrier->arrive_and_wait(); }
inline void __threadfence() {}
inline void __threadfence_block() {}
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() (g_waves[threadIdx.x / 64]->bar->arrive_and_wait())
#define __builtin_amdgcn_update_dpp(a, b, c, d, e, f) (b)

inline WaveX &my_wave() { return *g_waves[threadIdx.x / 64]; }
template <typename T>
inline T wave_exchange(T v, int src_lane) {
    WaveX &w = my_wave();
    const int lane = threadIdx.x & 63;
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    w.bar->arrive_and_wait();
    w.v[lane] = bits;
    w.bar->arrive_and_wait();
    uint64_t got = w.v[(src_lane >= 0 && src_lane < 64) ? src_lane : lane];
    w.bar->arrive_and_wait();
    T r;
    std::memcpy(&r, &got, sizeof(T));
    return r;
}
template <typename T> inline T __shfl_up(T v, int off, int = 64) {
    const int lane = threadIdx.x & 63;
    return wave_exchange(v, lane - off >= 0 ? lane - off : lane);
}
template <typename T> inline T __shfl_xor(T v, int m, int = 64) {
    return wave_exchange(v, (int)((threadIdx.x & 63) ^ m));
}
template <typename T> inline T __shfl(T v, int src, int = 64) { return wave_exchange(v, src); }
inline uint64_t __ballot(int pred) {
    WaveX &w = my_wave();
    const int lane = threadIdx.x & 63;
    w.bar->arrive_and_wait();
    w.v[lane] = pred ? 1 : 0;
    w.bar->arrive_and_wait();
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i) if (w.v[i]) m |= 1ull << i;
    w.bar->arrive_and_wait();
    return m;
}
inline int __popcll(uint64_t x) { return __builtin_popcountll(x); }
// the kernels that read the first lane do so with every lane of the wave active
#define __builtin_amdgcn_readfirstlane(v) wave_exchange((v), 0)
inline int __popc(uint32_t x) { return __builtin_popcount(x); }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline double __longlong_as_double(long long x) { double d; std::memcpy(&d, &x, 8); return d; }
inline long long __double_as_longlong(double d) { long long x; std::memcpy(&x, &d, 8); return x; }

inline uint32_t emu_mbcnt_lo(uint32_t m, uint32_t base) {
    const int l = threadIdx.x & 63;
    const uint32_t below = l >= 32 ? 0xffffffffu : ((1u << l) - 1u);
    return base + (uint32_t)__builtin_popcount(m & below);
}
inline uint32_t emu_mbcnt_hi(uint32_t m, uint32_t base) {
    const int l = threadIdx.x & 63;
    const uint32_t below = l < 32 ? 0u : ((uint32_t)((1ull << (l - 32)) - 1ull));
    return base + (uint32_t)__builtin_popcount(m & below);
}
#define __builtin_amdgcn_mbcnt_lo(m, b) emu_mbcnt_lo((m), (b))
#define __builtin_amdgcn_mbcnt_hi(m, b) emu_mbcnt_hi((m), (b))
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
template <typename T> inline T __hip_atomic_load(const T *p, int, int) {
    return std::atomic_ref<T>(*const_cast<T *>(p)).load();
}
template <typename T, typename U> inline void __hip_atomic_store(T *p, U v, int, int) {
    std::atomic_ref<T>(*p).store((T)v);
}
template <typename T> inline T atomicAdd(T *p, T v) { return std::atomic_ref<T>(*p).fetch_add(v); }
template <typename T> inline T atomicOr(T *p, T v) { return std::atomic_ref<T>(*p).fetch_or(v); }
template <typename T> inline T atomicMin(T *p, T v) {
    std::atomic_ref<T> a(*p); T o = a.load();
    while (v < o && !a.compare_exchange_weak(o, v)) {}
    return o;
}
template <typename T> inline T atomicMax(T *p, T v) {
    std::atomic_ref<T> a(*p); T o = a.load();
    while (v > o && !a.compare_exchange_weak(o, v)) {}
    return o;
}
using std::max;
using std::min;

// One std::thread per work-item of a block, reused for every block of the
// launch: after a block, all work-items meet at an end barrier, work-item 0
// sets up fresh block and wavefront barriers and a fresh dynamic shared buffer,
// and the next block starts.
template <typename... KArgs, typename... Args>
void cpu_launch(void (*k)(KArgs...), dim3 grid, dim3 block, size_t shmem, Args... args) {
    blockDim.x = block.x;
    gridDim.x = grid.x;
    if (grid.x == 0) return;
    std::unique_ptr<std::barrier<>> blk;
    std::vector<char> lds;
    auto setup = [&]() {
        blk = std::make_unique<std::barrier<>>(block.x);
        g_block_barrier = blk.get();
        g_waves.clear();
        for (unsigned w = 0; w < (block.x + 63) / 64; ++w) {
            auto x = std::make_unique<WaveX>();
            x->bar = std::make_unique<std::barrier<>>(std::min(64u, block.x - 64 * w));
            g_waves.push_back(std::move(x));
        }
        lds.assign(shmem ? shmem : 1, 0);
        g_dyn_lds = shmem ? lds.data() : nullptr;
    };
    setup();
    std::barrier<> end_bar(block.x);
    std::vector<std::thread> ts;
    for (unsigned t = 0; t < block.x; ++t)
        ts.emplace_back([&, t]() {
            threadIdx.x = t;
            for (unsigned b = 0; b < grid.x; ++b) {
                blockIdx.x = b;
                k(args...);
                g_waves[t / 64]->bar->arrive_and_drop();
                g_block_barrier->arrive_and_drop();
                end_bar.arrive_and_wait();
                if (t == 0 && b + 1 < grid.x) setup();
                end_bar.arrive_and_wait();
            }
        });
    for (auto &th : ts) th.join();
}
#define hipLaunchKernelGGL(k, grid, block, shmem, stream, ...) cpu_launch(k, dim3(grid), dim3(block), (size_t)(shmem), __VA_ARGS__)
