// Pruning with the spatial-temporal variation score (Sec. 4.2.1): the
// temporal variation score of Eq. 5-6 and the volume of each Gaussian, the
// combination of Eq. 7 with the normalised volume, and the selection of the
// highest scores.  The spatial score itself (Eq. 4) is accumulated by the
// compositor.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_gauss.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kBlock = 256;

// Per Gaussian: S^TV = sum_t 1 / (0.5 tanh|p''(t)| + 0.5) with
// p''(t) = ((t - mu_t)^2 / S44^2 - 1 / S44) p(t) (float64), and the volume
// exp(sum of log scales) as a float32 sort key (0 for invalid Gaussians).
__global__ void __launch_bounds__(kBlock) temporal_volume_kernel(KModel m, const double *times, int32_t n_times,
                                                                 float *tv, uint32_t *vol_key, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m.n) return;
    Gauss4 G;
    float s = 0.0f;
    uint32_t key = 0u;
    if (load_gaussian(m, i, G)) {
        const double s44 = sigma44_of(G);
        double acc = 0.0;
        for (int f = 0; f < n_times; ++f) {
            const double d = times[f] - G.mu[3];
            const double p = exp(-d * d / (2.0 * s44));
            const double p2 = (d * d / (s44 * s44) - 1.0 / s44) * p;
            acc += 1.0 / (0.5 * tanh(fabs(p2)) + 0.5);
        }
        s = (float)acc;
        const float vol = (float)exp(G.ls[0] + G.ls[1] + G.ls[2] + G.ls[3]);
        key = __float_as_uint(vol);   // vol >= 0: bit order = value order
    }
    tv[i] = s;
    vol_key[i] = key;
    vals[i] = (uint32_t)i;
}

// out = S^TV gamma spatial, gamma = min(V / V_q, 1)^0.1 with V_q the volume at
// position q of the ascending volumes.
__global__ void __launch_bounds__(kBlock) variation_score_kernel(const float *tv, const uint32_t *vol_key,
                                                                 const uint32_t *sorted_vol, int64_t n, int64_t q,
                                                                 const float *spatial, float *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double vq = (double)__uint_as_float(sorted_vol[q]);
    const double v = (double)__uint_as_float(vol_key[i]);
    double gamma;
    if (vq > 0.0) gamma = pow(fmin(v / vq, 1.0), 0.1);
    else gamma = v > 0.0 ? 1.0 : 0.0;
    out[i] = v > 0.0 ? (float)((double)tv[i] * gamma * (double)spatial[i]) : 0.0f;
}

// Descending order by score through an ascending sort: key = ~bits of the
// score (non-negative floats), scores that are negative or NaN sort as 0.
__global__ void __launch_bounds__(kBlock) prune_keys_kernel(const float *score, int64_t n, uint32_t *keys,
                                                            uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float s = score[i];
    keys[i] = s > 0.0f ? ~__float_as_uint(s) : 0xffffffffu;
    vals[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(kBlock) mark_first_kernel(const uint32_t *sorted_vals, int64_t n_keep,
                                                            uint8_t *flags) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n_keep) flags[sorted_vals[j]] = 1;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_temporal_volume(const KModel &m, const double *times, int32_t n_times, float *tv,
                                  uint32_t *vol_key, uint32_t *vals, hipStream_t s) {
    if (m.n > 0)
        hipLaunchKernelGGL(temporal_volume_kernel, dim3(blocks(m.n)), dim3(kBlock), 0, s, m, times, n_times, tv,
                           vol_key, vals);
    return hipGetLastError();
}

hipError_t launch_variation_score(const float *tv, const uint32_t *vol_key, const uint32_t *sorted_vol, int64_t n,
                                  int64_t q, const float *spatial, float *out, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(variation_score_kernel, dim3(blocks(n)), dim3(kBlock), 0, s, tv, vol_key, sorted_vol, n, q,
                           spatial, out);
    return hipGetLastError();
}

hipError_t launch_prune_keys(const float *score, int64_t n, uint32_t *keys, uint32_t *vals, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(prune_keys_kernel, dim3(blocks(n)), dim3(kBlock), 0, s, score, n, keys, vals);
    return hipGetLastError();
}

hipError_t launch_mark_first(const uint32_t *sorted_vals, int64_t n_keep, uint8_t *flags, hipStream_t s) {
    if (n_keep > 0)
        hipLaunchKernelGGL(mark_first_kernel, dim3(blocks(n_keep)), dim3(kBlock), 0, s, sorted_vals, n_keep, flags);
    return hipGetLastError();
}

}  // namespace fdgs
