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

#include "dev_cull.h"
#include "dev_gauss.h"
#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kBlock = kPreprocessBlock;
constexpr double kLog2eD = 1.4426950408889634;

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
    PreprocOut out;
};

// Processed entry j of view vd (local position i = j - vd.p_off).  Returns
// whether it is visible; then *rect4 and *ell describe its footprint for the
// tile count.
__device__ __forceinline__ bool preprocess_one(const ViewDesc &vd, int64_t j, const PreArgs &a, int4 *rect4,
                                               CullEllipse *ell) {
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
        const double q = cut_level(opac, (double)a.rp.alpha_min, a.rp.temporal_cull, a.rp.vanilla_level);
        r = pixel_rect(Pr, q, vd.cam.W, vd.cam.H);
        vis = r.x0 <= r.x1 && r.y0 <= r.y1;
    }
    if (vis) {
        const double det = Pr.c00 * Pr.c11 - Pr.c01 * Pr.c01;
        const double ca = Pr.c11 / det, cb = -Pr.c01 / det, cc = Pr.c00 / det;
        // view direction from the camera centre C = -R^T t to the conditional mean
        const double *R = vd.cam.R;
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            d[k] = S.mean3[k] + (R[k] * vd.cam.t[0] + R[3 + k] * vd.cam.t[1] + R[6 + k] * vd.cam.t[2]);
        const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        float rgb[3], coef[48];
        load_sh_model(vd.m, g, coef);
        sh_eval(coef, vd.m.sh_degree, (float)(d[0] * il), (float)(d[1] * il), (float)(d[2] * il), rgb);
        const float uh = (float)Pr.u, vh = (float)Pr.v;
        Rec2D rec;
        rec.a = make_float4(uh, vh, (float)(Pr.u - (double)uh), (float)(Pr.v - (double)vh));
        rec.b = make_float4((float)ca, (float)cb, (float)cc, (float)opac);
        rec.c = make_float4(rgb[0], rgb[1], rgb[2], (float)Pr.z);
        // square completed in y: every term of the compositor's exponent then
        // has one sign, so float32 loses nothing to cancellation however
        // elongated the footprint or far its centre
        const double sl = -Pr.c01 / Pr.c00;
        const float s_hi = (float)sl;
        rec.d = make_float4((float)(-0.5 * kLog2eD / Pr.c00), (float)sqrt(0.5 * kLog2eD * Pr.c00 / det), s_hi,
                            (float)(sl - (double)s_hi));
        a.out.rec[j] = rec;
        a.out.depth_key[j] = (uint64_t)__double_as_longlong(Pr.z);
        const int4 r4 = make_int4(r.x0, r.y0, r.x1, r.y1);
        reinterpret_cast<int4 *>(a.out.rect)[j] = r4;
        *rect4 = r4;
        *ell = cull_ellipse(rec, a.rp);
    }
    a.out.visible[j] = vis ? 1 : 0;
    return vis;
}

// One thread per processed entry; then the workgroup counts its entries'
// tiles row-parallel: the tile rows of the visible entries' rectangles are
// enumerated (block scan of rows per entry) and spread over the threads, each
// evaluating one row's tile columns (the evaluation tile-key emission
// repeats), so a footprint spanning many rows does not hold up a wavefront.
__global__ void __launch_bounds__(kBlock) preprocess_kernel(PreArgs a) {
    __shared__ int4 s_rect[kBlock];
    __shared__ CullEllipse s_ell[kBlock];
    __shared__ uint32_t s_rbase[kBlock], s_cnt[kBlock];
    __shared__ uint32_t s_tmp[kBlock / 64 + 1];
    const int t = threadIdx.x;
    const int64_t j = (int64_t)blockIdx.x * kBlock + t;
    const int64_t P = (a.V == 1 && a.n_dev) ? min(*a.n_dev, a.n_total) : a.n_total;
    bool vis = false;
    int4 r4 = make_int4(0, 0, -1, -1);
    CullEllipse ell = {};
    if (j < P) {
        if (a.V == 1) {
            vis = preprocess_one(a.one, j, a, &r4, &ell);
        } else {
            int lo = 0, hi = a.V - 1;         // last view whose range starts at or before j
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.table[mid].p_off <= j) lo = mid; else hi = mid - 1;
            }
            a.out.view_of[j] = (uint32_t)lo;
            vis = preprocess_one(a.table[lo], j, a, &r4, &ell);
        }
    }
    const int tw = a.rp.tile_w, th = a.rp.tile_h;
    uint32_t rows = 0, direct = 0;
    if (vis) {
        if (ell.a > 0.0f) rows = (uint32_t)(r4.w / th - r4.y / th + 1);
        else direct = count_tiles(ell, r4, tw, th);   // whole rectangle, closed form
    }
    s_rect[t] = r4;
    s_ell[t] = ell;
    s_cnt[t] = direct;
    uint32_t n_rows;
    s_rbase[t] = block_exclusive_sum<kBlock>(rows, s_tmp, &n_rows);   // contains barriers
    for (uint32_t row0 = 0; row0 < n_rows; row0 += kBlock) {
        const uint32_t rho = row0 + (uint32_t)t;
        if (rho < n_rows) {
            int lo = 0, hi = kBlock - 1;      // last entry whose rows start at or before rho
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_rbase[mid] <= rho) lo = mid; else hi = mid - 1;
            }
            const int4 rr = s_rect[lo];
            const int ty = rr.y / th + (int)(rho - s_rbase[lo]);
            int c0, c1;
            if (tile_row_span(s_ell[lo], rr, ty, tw, th, &c0, &c1)) atomicAdd(&s_cnt[lo], (uint32_t)(c1 - c0 + 1));
        }
    }
    __syncthreads();
    if (j < P) a.out.tiles[j] = s_cnt[t];
    if (a.out.vis_count) {                          // uniform
        const int nv = __syncthreads_count(vis);
        if (t == 0) a.out.vis_count[blockIdx.x] = (uint32_t)nv;
    }
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
