// Micro-benchmarks of the chip's own rates, against which kernel rates are
// expressed as fractions: LDS reads in the compositor's pattern (every lane of
// a wavefront reading the same 16 bytes, a broadcast) and with lane-distinct
// addresses, and the float32 FMA issue rate of the vector ALUs (non-packed, as
// the library is built).
#include <hip/hip_runtime.h>

#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kLdsNT = 256;
constexpr int kLdsWords = 1024;   // float4 entries (16 KB)

// Each loop step reads 8 float4 per lane and consumes each with two FMAs, so
// the vector ALUs can absorb up to 512 B of LDS data per clock per CU: the
// LDS limits.  broadcast: all lanes of a wavefront read one address.
__global__ void __launch_bounds__(kLdsNT) lds_probe_kernel(int iters, int broadcast, float *out) {
    __shared__ float4 buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kLdsNT)
        buf[i] = make_float4(1e-3f * i, 1.0f, 1e-3f * (i + 1), 1.0f);
    __syncthreads();
    const int lane = broadcast ? 0 : (int)(threadIdx.x & 63);
    int base = (int)(threadIdx.x >> 6) * 64;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            const float4 v = buf[(base + u * 64 + lane) & (kLdsWords - 1)];
            const float4 w = buf[(base + (u + 1) * 64 + lane) & (kLdsWords - 1)];
            a0 = fmaf(v.x, v.y, a0);
            a1 = fmaf(v.z, v.w, a1);
            a2 = fmaf(w.x, w.y, a2);
            a3 = fmaf(w.z, w.w, a3);
        }
        base = (base + 512) & (kLdsWords - 1);
    }
    const float r = (a0 + a1) + (a2 + a3);
    if (r == -1.0f) out[blockIdx.x] = r;   // never true: keeps the reads
}

constexpr int kAluNT = 256;

// Eight independent FMA chains per thread.
__global__ void __launch_bounds__(kAluNT) valu_probe_kernel(int iters, float *out) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = 1e-3f * (float)(threadIdx.x + k);
    const float m = 0.999f, c = 1e-4f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], m, c);
    }
    float r = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) r += x[k];
    if (r == -1.0f) out[blockIdx.x] = r;
}

double time_ms(void (*launch)(hipStream_t, int, float *, int), hipStream_t s, int iters, float *sink, int grid,
               hipError_t *err) {
    hipEvent_t e0, e1;
    *err = hipEventCreate(&e0);
    if (*err != hipSuccess) return 0.0;
    *err = hipEventCreate(&e1);
    if (*err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 0.0;
    }
    launch(s, iters, sink, grid);   // warm-up
    (void)hipEventRecord(e0, s);
    launch(s, iters, sink, grid);
    (void)hipEventRecord(e1, s);
    *err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (*err == hipSuccess) *err = hipEventElapsedTime(&ms, e0, e1);
    if (*err == hipSuccess) *err = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

void lds_bcast(hipStream_t s, int iters, float *sink, int grid) {
    hipLaunchKernelGGL(lds_probe_kernel, dim3(grid), dim3(kLdsNT), 0, s, iters, 1, sink);
}
void lds_distinct(hipStream_t s, int iters, float *sink, int grid) {
    hipLaunchKernelGGL(lds_probe_kernel, dim3(grid), dim3(kLdsNT), 0, s, iters, 0, sink);
}
void valu(hipStream_t s, int iters, float *sink, int grid) {
    hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(kAluNT), 0, s, iters, sink);
}

}  // namespace

hipError_t measure_peaks(float *sink, double *out, hipStream_t s) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int grid = cus * 8;
    const int lds_iters = 4096, alu_iters = 16384;
    const double lds_bytes = (double)grid * kLdsNT * lds_iters * 8 * 16;
    double ms = time_ms(lds_bcast, s, lds_iters, sink, grid, &e);
    if (e != hipSuccess) return e;
    out[0] = lds_bytes / (ms * 1e-3);
    ms = time_ms(lds_distinct, s, lds_iters, sink, grid, &e);
    if (e != hipSuccess) return e;
    out[1] = lds_bytes / (ms * 1e-3);
    ms = time_ms(valu, s, alu_iters, sink, grid, &e);
    if (e != hipSuccess) return e;
    out[2] = (double)grid * kAluNT * alu_iters * 8 / (ms * 1e-3);
    out[3] = (double)cus;
    return hipSuccess;
}

}  // namespace fdgs
