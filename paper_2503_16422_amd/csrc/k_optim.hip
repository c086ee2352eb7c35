// Adam update for the masked fine-tuning of the kept Gaussians (the
// optimisation that compensates for pruning and filtering, Sec. 4.2.1-4.2.2).
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
// One thread per element, four elements per thread when aligned.
#include <hip/hip_runtime.h>
#include <math.h>

#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kBlock = 256;

struct AdamArgs {
    float *p;
    const float *g;
    float *m;
    float *v;
    int64_t n;
    float lr, b1, b2, eps;
    float c1, c2;   // 1 / (1 - b1^t), 1 / (1 - b2^t)
    int32_t vec;    // all four arrays 16-byte aligned
};

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, const AdamArgs &a) {
    m = a.b1 * m + (1.0f - a.b1) * g;
    v = a.b2 * v + (1.0f - a.b2) * g * g;
    p -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

__global__ void __launch_bounds__(kBlock) adam_kernel(AdamArgs a) {
    const int64_t i4 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    if (a.vec && i4 + 3 < a.n) {
        float4 p = *reinterpret_cast<const float4 *>(a.p + i4);
        const float4 g = *reinterpret_cast<const float4 *>(a.g + i4);
        float4 m = *reinterpret_cast<const float4 *>(a.m + i4);
        float4 v = *reinterpret_cast<const float4 *>(a.v + i4);
        adam_one(p.x, g.x, m.x, v.x, a);
        adam_one(p.y, g.y, m.y, v.y, a);
        adam_one(p.z, g.z, m.z, v.z, a);
        adam_one(p.w, g.w, m.w, v.w, a);
        *reinterpret_cast<float4 *>(a.p + i4) = p;
        *reinterpret_cast<float4 *>(a.m + i4) = m;
        *reinterpret_cast<float4 *>(a.v + i4) = v;
    } else {
        const int64_t end = min(i4 + 4, a.n);
        for (int64_t i = i4; i < end; ++i) adam_one(a.p[i], a.g[i], a.m[i], a.v[i], a);
    }
}

}  // namespace

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int32_t step, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    auto al = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    AdamArgs a{p, g, m, v, n, lr, b1, b2, eps, (float)(1.0 / (1.0 - std::pow((double)b1, step))),
               (float)(1.0 / (1.0 - std::pow((double)b2, step))), al(p) && al(g) && al(m) && al(v)};
    const int64_t threads = (n + 3) / 4;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fdgs
