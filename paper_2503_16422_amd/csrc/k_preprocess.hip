// Per-Gaussian kernels: temporal slicing (Eq. 1, Eq. 3), the fused
// slice -> project -> shade -> footprint preprocess, and the keyframe
// active-set predicate (Sec. 4.2.2).
//
// The geometry runs in float64.  These kernels are bound by HBM traffic
// (68-260 B per Gaussian against ~400 flops), and CDNA4 issues float64 FMA at
// the same lane rate as non-packed float32, so the wider type is nearly free
// here.  It makes every discrete decision taken per Gaussian (culling, the
// pixel rectangle, the depth order) agree with a float64 evaluation of the
// same formulas, and leaves the stored pixel-space centre accurate to well
// under 1e-5 px.  Colour (SH) is evaluated in float32.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_gauss.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) slice_kernel(KModel m, double t, const uint32_t *idx,
                                                       int64_t count, float *mean3, float *cov3,
                                                       float *p) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= count) return;
    const int64_t g = idx ? (int64_t)idx[j] : j;
    Gauss4 G;
    Sliced S = {};
    if (load_gaussian(m, g, G)) {
        S = slice_gaussian(G, t);
        if (!S.ok) S = Sliced{};
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) mean3[k * count + j] = (float)S.mean3[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) cov3[k * count + j] = (float)S.cov3[k];
    p[j] = (float)S.p;
}

struct PreArgs {
    ViewDesc one;              // the view when V == 1
    const ViewDesc *table;     // device table when V > 1
    int32_t V;
    const int64_t *n_dev;      // device processed count (V == 1 only)
    int64_t n_total;           // processed entries over all views (upper bound when n_dev)
    RenderParams rp;
    double vanilla_level;
    PreprocOut out;
};

// Processed entry j of view vd (local position i = j - vd.p_off).
__device__ __forceinline__ void preprocess_one(const ViewDesc &vd, int64_t j, const PreArgs &a) {
    const int64_t i = j - vd.p_off;
    const int64_t g = vd.idx ? (int64_t)vd.idx[i] : i;
    Gauss4 G;
    bool vis = load_gaussian(vd.m, g, G);
    Sliced S = {};
    Projected Pr = {};
    double opac = 0.0;
    PixRect r = {0, 0, -1, -1};
    if (vis) {
        S = slice_gaussian(G, vd.t);
        vis = S.ok;
    }
    if (vis) {
        Pr = project(vd.cam, S, (double)a.rp.dilation);
        vis = Pr.ok;
    }
    if (vis) {
        const double sigma = 1.0 / (1.0 + exp(-G.logit));
        opac = sigma * S.p;
        if (a.rp.temporal_cull && opac < (double)a.rp.alpha_min) vis = false;
    }
    if (vis) {
        const double q = cut_level(opac, (double)a.rp.alpha_min, a.rp.temporal_cull, a.vanilla_level);
        r = pixel_rect(Pr, q, vd.cam.W, vd.cam.H);
        vis = r.x0 <= r.x1 && r.y0 <= r.y1;
    }
    uint32_t tiles = 0;
    if (vis) {
        const int tx0 = r.x0 / a.rp.tile_w, tx1 = r.x1 / a.rp.tile_w;
        const int ty0 = r.y0 / a.rp.tile_h, ty1 = r.y1 / a.rp.tile_h;
        tiles = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
        const double det = Pr.c00 * Pr.c11 - Pr.c01 * Pr.c01;
        const double ca = Pr.c11 / det, cb = -Pr.c01 / det, cc = Pr.c00 / det;
        // view direction from the camera centre C = -R^T t to the conditional mean
        const double *R = vd.cam.R;
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            d[k] = S.mean3[k] + (R[k] * vd.cam.t[0] + R[3 + k] * vd.cam.t[1] + R[6 + k] * vd.cam.t[2]);
        const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float rgb[3];
        sh_to_rgb(vd.m.sh, vd.m.n, g, vd.m.sh_degree, (float)(d[0] * il), (float)(d[1] * il),
                  (float)(d[2] * il), rgb);
        const float uh = (float)Pr.u, vh = (float)Pr.v;
        Rec2D rec;
        rec.a = make_float4(uh, vh, (float)(Pr.u - (double)uh), (float)(Pr.v - (double)vh));
        rec.b = make_float4((float)ca, (float)cb, (float)cc, (float)opac);
        rec.c = make_float4(rgb[0], rgb[1], rgb[2], (float)Pr.z);
        a.out.rec[j] = rec;
        a.out.depth_key[j] = (uint64_t)__double_as_longlong(Pr.z);
        reinterpret_cast<int4 *>(a.out.rect)[j] = make_int4(r.x0, r.y0, r.x1, r.y1);
    }
    a.out.tiles[j] = tiles;
    a.out.visible[j] = vis ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) preprocess_kernel(PreArgs a) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t P = (a.V == 1 && a.n_dev) ? min(*a.n_dev, a.n_total) : a.n_total;
    if (j >= P) return;
    if (a.V == 1) {
        preprocess_one(a.one, j, a);
        return;
    }
    int lo = 0, hi = a.V - 1;             // last view whose range starts at or before j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.table[mid].p_off <= j) lo = mid; else hi = mid - 1;
    }
    a.out.view_of[j] = (uint32_t)lo;
    preprocess_one(a.table[lo], j, a);
}

struct MaskKArgs {
    KModel m;
    MaskArgs a;
};

__global__ void __launch_bounds__(kBlock) mask_kernel(MaskKArgs k, uint32_t *bits) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool keep = false;
    if (g < k.m.n) {
        Gauss4 G;
        if (load_gaussian(k.m, g, G)) {
            const double s44 = sigma44_of(G);
            for (int f = 0; f < k.a.n_frames && !keep; ++f) {
                const double d = k.a.frames[f] - G.mu[3];
                keep = d * d <= k.a.level * s44;
            }
            if (keep && k.a.mode == FDGS_MASK_TEMPORAL_AND_TILE) {
                bool seen = false;
                for (int kk = 0; kk < 2 && !seen; ++kk) {
                    const Sliced S = slice_gaussian(G, kk == 0 ? k.a.key_lo : k.a.key_hi);
                    if (!S.ok) continue;
                    for (int v = 0; v < k.a.n_views && !seen; ++v) {
                        const KCam cam = k.a.views[v];
                        const Projected P = project(cam, S, k.a.dilation);
                        if (!P.ok) continue;
                        const PixRect r = pixel_rect(P, k.a.rect_level, cam.W, cam.H);
                        seen = r.x0 <= r.x1 && r.y0 <= r.y1;
                    }
                }
                keep = seen;
            }
        }
    }
    const uint64_t ballot = __ballot(keep);
    const int lane = threadIdx.x & 63;
    const int64_t word = g >> 5;
    const int64_t nw = (k.m.n + 31) >> 5;
    if (lane == 0 && word < nw) bits[word] = (uint32_t)(ballot & 0xffffffffu);
    if (lane == 32 && word < nw) bits[word] = (uint32_t)(ballot >> 32);
}

}  // namespace

hipError_t launch_slice(const KModel &m, double t, const uint32_t *idx, int64_t count,
                        float *mean3, float *cov3, float *p, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const unsigned grid = (unsigned)((count + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(slice_kernel, dim3(grid), dim3(kBlock), 0, s, m, t, idx, count, mean3, cov3, p);
    return hipGetLastError();
}

hipError_t launch_preprocess(const ViewDesc *one, const ViewDesc *table, int32_t V, const int64_t *n_dev,
                             int64_t n_total, const RenderParams &rp, const PreprocOut &out, hipStream_t s) {
    if (n_total == 0) return hipSuccess;
    PreArgs a;
    a.one = one ? *one : ViewDesc{};
    a.table = table;
    a.V = V;
    a.n_dev = n_dev;
    a.n_total = n_total;
    a.rp = rp;
    a.vanilla_level = 2.0 * log(1.0 / (double)rp.alpha_min) * (1.0 + 1e-4) + 1e-4;
    a.out = out;
    const unsigned grid = (unsigned)((n_total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(preprocess_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mask_bits(const KModel &m, const MaskArgs &a, uint32_t *bits, hipStream_t s) {
    if (m.n == 0) return hipSuccess;
    MaskKArgs k{m, a};
    const unsigned grid = (unsigned)((m.n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(mask_kernel, dim3(grid), dim3(kBlock), 0, s, k, bits);
    return hipGetLastError();
}

}  // namespace fdgs
