// Adjoint of the per-tile compositing (Eq. 2 and Eq. 3 differentiated with
// respect to each record's centre, conic, opacity and colour).
#include <hip/hip_runtime.h>

#include "dev_composite.h"
#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

using namespace comp;

struct BwdArgs {
    RenderParams rp;
    int32_t W, H;
    const uint32_t *ranges;
    const uint32_t *ids;
    const Rec2D *rec;
    const float *T_final;
    const uint32_t *n_contrib;
    const float *dL;
    float *g2d;        // [n_proc][9]: du, dv, d conic a, b, c, d opacity, d rgb
};

// Adjoint, walking each pixel's list back to front from its last contributor.
// The transmittance in front of Gaussian i is recovered as T_{i+1} / (1 - a_i)
// from the stored final T, so no per-pixel list is kept.  With g = dL/dC and
// S the colour accumulated behind i (absolute weights):
//   dL/dc_i = a_i T_i g
//   dL/da_i = T_i c_i.g - (S.g + T_final bg.g) / (1 - a_i)
// then a_i = min(a_max, o_i G_i) -> (o_i, conic, centre).  A thread owns PPT
// pixels of a column of its wavefront's cell (the forward's layout) and adds
// their terms before the per-Gaussian sums are reduced over each row of 16
// lanes (DPP) and added into the tile's LDS accumulators by one lane per row;
// one global add per value and Gaussian leaves the tile after each batch.
// With several cells per tile (and tile culling on) a wavefront walks only the
// records whose footprint ellipse reaches its cell: the others have alpha
// below alpha_min at every one of its pixels and contribute nothing.
template <int TW, int TH, int BATCH, int PPT>
__global__ void __launch_bounds__(TW *TH / PPT) composite_bwd_kernel(BwdArgs a) {
    constexpr int NT = TW * TH / PPT;
    using C = Cells<TW, TH, PPT>;
    // per-wavefront bitmaps of the batch's records that reach its cell (as in the forward)
    constexpr bool kBits = C::NW > 1;
    constexpr int kWords = BATCH / 64;
    __shared__ uint64_t s_bits[kBits ? C::NW * kWords : 1];
    const bool cull = a.rp.tile_cull != 0;
    __shared__ float4 s_xy[BATCH];    // centre (block-centred), log2 opacity, 1 / opacity
    __shared__ float4 s_ex[BATCH];    // s, c0, kx, q: the exponent as the forward stages it
    __shared__ float4 s_rgb[BATCH];
    __shared__ uint32_t s_id[BATCH];
    __shared__ float s_acc[BATCH * 9]; // per-Gaussian gradient sums of the tile
    const int tile = blockIdx.x;
    const int tx = tile % a.rp.tiles_x, ty = tile / a.rp.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64), lane = lane_id();
    const int lx = (wave % C::CX) * C::CW + lane % C::CW, ly0 = (wave / C::CX) * C::CH + (lane / C::CW) * PPT;
    const int px = tx * TW + lx, py0 = ty * TH + ly0;
    const int bx0 = ((tx * TW) & ~(kBlockSize - 1)) + kBlockHalf;   // as in the forward
    const int by0 = ((ty * TH) & ~(kBlockSize - 1)) + kBlockHalf;
    const float fx = (float)(px - bx0) + 0.5f;
    const float ox = (float)bx0, oy = (float)by0;
    const uint32_t start = a.ranges[2 * tile];
    const float amin = a.rp.alpha_min, amax = a.rp.alpha_max;
    const uint32_t amax_bits = __float_as_uint(amax);
    const int64_t plane = (int64_t)a.W * a.H;
    float fy[PPT], g0[PPT], g1[PPT], g2[PPT], T[PPT], S0[PPT], S1[PPT], S2[PPT], bgdot[PPT];
    uint32_t last[PPT];
    uint32_t my_max = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p;
        fy[p] = (float)(py - by0) + 0.5f;
        g0[p] = g1[p] = g2[p] = 0.f;
        T[p] = 1.f;
        last[p] = 0;
        if (px < a.W && py < a.H) {
            const int64_t pix = (int64_t)py * a.W + px;
            g0[p] = a.dL[pix];
            g1[p] = a.dL[plane + pix];
            g2[p] = a.dL[2 * plane + pix];
            T[p] = a.T_final[pix];
            last[p] = a.n_contrib[pix];
        }
        bgdot[p] = T[p] * (a.rp.bg[0] * g0[p] + a.rp.bg[1] * g1[p] + a.rp.bg[2] * g2[p]);   // T_final bg.g
        S0[p] = S1[p] = S2[p] = 0.f;
        my_max = max(my_max, last[p]);
    }
    // block-wide maximum of `last` bounds the walk
    __shared__ uint32_t s_max;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, my_max);
    __syncthreads();
    const uint32_t walk_end = start + s_max;
    for (int j = threadIdx.x; j < BATCH * 9; j += NT) s_acc[j] = 0.0f;
    for (int64_t top = (int64_t)walk_end; top > (int64_t)start; top -= BATCH) {
        const uint32_t lo = (uint32_t)max((int64_t)start, top - BATCH);
        const int cnt = (int)(top - lo);
        __syncthreads();
        for (int k0 = 0; k0 < cnt; k0 += NT) {
            const int k = k0 + (int)threadIdx.x;
            uint32_t cells = 0u;
            if (k < cnt) {
                const uint32_t id = a.ids[lo + k];
                const Rec2D r = a.rec[id];
                const ExpRec q = stage_exp(r, ox, oy);
                s_xy[k] = make_float4(q.gx, q.gy, q.lo, 1.0f / r.b.w);
                s_ex[k] = make_float4(q.s, q.c0, q.kx, q.q);
                s_rgb[k] = r.c;
                s_id[k] = id;
                if constexpr (kBits) {
                    if (cull) cells = reached_cells<TW, TH, PPT>(r, a.rp, tx * TW, ty * TH);
                }
            }
            if (kBits && cull) {
                const int word = k0 / 64 + wave;
#pragma unroll
                for (int w = 0; w < C::NW; ++w) {
                    const uint64_t m = __ballot((cells >> w) & 1u);
                    if (lane == 0 && word < kWords) s_bits[w * kWords + word] = m;
                }
            }
        }
        __syncthreads();
        // one record, back to front; every lane of the wavefront takes part
        auto grad_record = [&](int k) {
            const uint32_t pos = lo + k - start;   // position in the tile list
            const float4 c = s_xy[k];
            const float4 q = s_ex[k];
            const float dx = fx - c.x;
            const float A = exp2_col_a(q.z, c.z, dx), B = exp2_col_t(q.x, q.y, fx);
            float du = 0.f, dv = 0.f, da = 0.f, db = 0.f, dc = 0.f, dop = 0.f;
            float dr = 0.f, dg = 0.f, dbl = 0.f;
            bool hit = false;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                if (pos < last[p]) {
                    const float raw = __builtin_amdgcn_exp2f(exp2_at(q.w, A, B, fy[p]));   // opacity x G
                    const float alpha = clamp_alpha(raw, amax_bits);
                    if (alpha >= amin) {
                        hit = true;
                        const float4 col = s_rgb[k];
                        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);   // 1 / (1 - a_i), ~1 ulp
                        T[p] = T[p] * inv;                 // transmittance in front of i
                        const float w = alpha * T[p];
                        dr = fmaf(w, g0[p], dr);
                        dg = fmaf(w, g1[p], dg);
                        dbl = fmaf(w, g2[p], dbl);
                        const float cg = col.x * g0[p] + col.y * g1[p] + col.z * g2[p];
                        const float sg = S0[p] * g0[p] + S1[p] * g1[p] + S2[p] * g2[p];
                        const float dalpha = T[p] * cg - (sg + bgdot[p]) * inv;
                        S0[p] += col.x * w;
                        S1[p] += col.y * w;
                        S2[p] += col.z * w;
                        if (raw < amax) {
                            // power = -1/2 (a dx^2 + 2 b dx dy + c dy^2); alpha = opacity exp(power)
                            dop = fmaf(raw * c.w, dalpha, dop);       // G = raw / opacity
                            const float dpow = alpha * dalpha;   // d alpha / d power
                            const float dy = fy[p] - c.y;
                            const float vl = exp2_line(q.w, B, fy[p]);   // q (dy + s dx), as in the exponent
                            da = fmaf(-0.5f * dx * dx, dpow, da);
                            db = fmaf(-dx * dy, dpow, db);
                            dc = fmaf(-0.5f * dy * dy, dpow, dc);
                            // d power / d u = -ln 2 d e / d dx with e = lo + kx dx^2 - v^2,
                            // v = q dy + (q s) dx: d e / d dx = 2 kx dx - 2 (q s) v, d e / d dy = -2 q v
                            du = fmaf(-kLn2 * 2.0f * (q.z * dx - q.x * vl), dpow, du);   // (a dx + b dy) dpow
                            dv = fmaf(kLn2 * 2.0f * (q.w * vl), dpow, dv);                // (b dx + c dy) dpow
                        }
                    }
                }
            }
            if (__ballot(hit) != 0ull) {
                // sums over each row of 16 lanes (four DPP steps), then one
                // LDS add per row: four lanes of one instruction per value
                du = row_sum16(du);
                dv = row_sum16(dv);
                da = row_sum16(da);
                db = row_sum16(db);
                dc = row_sum16(dc);
                dop = row_sum16(dop);
                dr = row_sum16(dr);
                dg = row_sum16(dg);
                dbl = row_sum16(dbl);
                if ((lane & 15) == 15) {
                    float *acc = s_acc + k * 9;
                    atomicAdd(acc + 0, du);
                    atomicAdd(acc + 1, dv);
                    atomicAdd(acc + 2, da);
                    atomicAdd(acc + 3, db);
                    atomicAdd(acc + 4, dc);
                    atomicAdd(acc + 5, dop);
                    atomicAdd(acc + 6, dr);
                    atomicAdd(acc + 7, dg);
                    atomicAdd(acc + 8, dbl);
                }
            }
        };
        if (kBits && cull) {
            // only the records whose ellipse reaches this wavefront's cell
            for (int c = (cnt - 1) / 64; c >= 0; --c) {
                const uint64_t word = s_bits[wave * kWords + c];
                uint64_t bits = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(word >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)word);
                while (bits != 0ull) {
                    const int b = 63 - __builtin_clzll(bits);
                    bits &= ~(1ull << b);
                    grad_record(c * 64 + b);
                }
            }
        } else {
            for (int k = cnt - 1; k >= 0; --k) grad_record(k);
        }
        __syncthreads();
        // one global add per (Gaussian, value) for the whole tile
        for (int j = threadIdx.x; j < cnt * 9; j += NT) {
            const float v = s_acc[j];
            if (v != 0.0f) atomicAdd(a.g2d + (int64_t)s_id[j / 9] * 9 + (j % 9), v);
            s_acc[j] = 0.0f;
        }
    }
}

// Pixels per thread in the adjoint: 2 for the 256-pixel tiles, 1 for 8x8.
template <int TW, int TH, int BATCH>
void launch_bwd(const BwdArgs &a, int n_tiles, hipStream_t s) {
    constexpr int PPT = TW * TH > 64 ? 2 : 1;
    hipLaunchKernelGGL((composite_bwd_kernel<TW, TH, BATCH, PPT>), dim3(n_tiles), dim3(TW * TH / PPT), 0, s, a);
}

}  // namespace

hipError_t launch_composite_backward(const RenderParams &rp, int32_t W, int32_t H, int32_t batch,
                                     const uint32_t *ranges, const uint32_t *ids, const Rec2D *rec,
                                     const float *T_final, const uint32_t *n_contrib,
                                     const float *dL_drgb, float *g2d, int64_t /*n_proc_max*/,
                                     hipStream_t s) {
    BwdArgs a{rp, W, H, ranges, ids, rec, T_final, n_contrib, dL_drgb, g2d};
    const int n_tiles = rp.tiles_x * rp.tiles_y;
    FDGS_DISPATCH(launch_bwd, a);
    return hipGetLastError();
}

}  // namespace fdgs
