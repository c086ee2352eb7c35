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
    const uint32_t *order;   // tiles longest list first (workgroup b takes tile order[b]), or NULL: raster order
};

// Adjoint, walking each pixel's list back to front from its last contributor.
// The transmittance in front of Gaussian i is recovered as T_{i+1} / (1 - a_i)
// from the stored final T, so no per-pixel list is kept.  With g = dL/dC, the
// colour behind i seen from just behind it, R_i = (colour behind i + T_final
// bg) . g / T_{i+1}, obeys R_{i-1} = R_i + a_i (c_i . g - R_i) from R = bg . g
// at the last contributor, and
//   dL/dc_i = a_i T_i g,    dL/da_i = T_i (c_i . g - R_i),
// then a_i = min(a_max, o_i G_i) -> (o_i, conic, centre).  With d_i = a_i
// dL/da_i at the pixels where the clamp is inactive (the derivative of alpha
// with respect to the exponent), every conic and centre gradient is a linear
// combination of per-Gaussian sums over the pixels, (dx, dy) = pixel centre -
// Gaussian centre and v = q (dy + s dx) the exponent's scaled distance to the
// footprint's centre line (log2 G = lo + kx dx^2 - v^2):
//   dL/du = -2 ln2 (kx sum d dx - q s sum d v),   dL/dv = 2 ln2 q sum d v,
//   dL/d(a, b, c) = -1/2 sum d dx^2, -sum d dx dy, -1/2 sum d dy^2,
//   dL/do = sum d / o
// (the centre terms in the exponent's own form, which does not cancel for
// needle-shaped footprints).  A pixel adds four of these sums (its column's
// dx gives the rest) and the conversion happens once per Gaussian and tile.
// A thread owns PPT pixels of a column of its wavefront's cell (the forward's
// layout).  The per-Gaussian sums of two records at a time are reduced over
// each row of 16 lanes -- a sum over neighbouring lanes that keeps the first
// record in the even lanes and the second in the odd ones, then three DPP
// steps that keep a lane's parity -- and added into the tile's LDS
// accumulators by two lanes per row; one global add per value and Gaussian
// leaves the tile after each batch.  With several cells per tile (and tile
// culling on) a wavefront walks only the records whose footprint ellipse
// reaches its cell: the others have alpha below alpha_min at every one of its
// pixels and contribute nothing.
template <int CTRL>
__device__ __forceinline__ float dpp_of(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
constexpr int kVals = 9;   // sums of d, d dx, d v, d dx^2, d dx dy, d dy^2; colour r, g, b

template <int TW, int TH, int BATCH, int PPT>
__global__ void __launch_bounds__(TW *TH / PPT) composite_bwd_kernel(BwdArgs a) {
    constexpr int NT = TW * TH / PPT;
    using C = Cells<TW, TH, PPT>;
    // per-wavefront bitmaps of the batch's records that reach its cell (as in the forward)
    constexpr bool kBits = C::NW > 1;
    constexpr int kWords = BATCH / 64;
    __shared__ uint64_t s_bits[kBits ? C::NW * kWords : 1];
    const bool cull = a.rp.tile_cull != 0;
    // per staged record three float4: gx, q s, c0, kx | log2 opacity, q, r, g | b, gy, opacity, id
    __shared__ float4 s_rec[3 * BATCH];
    __shared__ float s_acc[BATCH * kVals];   // per-Gaussian sums of the tile
    // the longest lists first, as in the forward's longest-first schedule: they
    // run beside the rest of the launch instead of alone at its end
    const int tile = a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
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
    float fy[PPT], g0[PPT], g1[PPT], g2[PPT], T[PPT], R[PPT];
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
        R[p] = a.rp.bg[0] * g0[p] + a.rp.bg[1] * g1[p] + a.rp.bg[2] * g2[p];   // bg . g
        my_max = max(my_max, last[p]);
    }
    // block-wide maximum of `last` bounds the walk
    __shared__ uint32_t s_max;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, my_max);
    __syncthreads();
    const uint32_t walk_end = start + s_max;
    for (int j = threadIdx.x; j < BATCH * kVals; j += NT) s_acc[j] = 0.0f;
    const bool odd = (lane & 1) != 0;
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
                s_rec[3 * k] = make_float4(q.gx, q.s, q.c0, q.kx);
                s_rec[3 * k + 1] = make_float4(q.lo, q.q, r.c.x, r.c.y);
                s_rec[3 * k + 2] = make_float4(r.c.z, q.gy, r.b.w, __uint_as_float(id));
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
        // alpha of record k at the thread's pixels: raw = opacity x G, and the
        // clamped alpha where the forward blended it (its position before the
        // pixel's last contributor and alpha >= alpha_min), else 0; also the
        // column offset dx and each pixel's centre-line distance v
        auto alphas = [&](int k, bool real, float &dx, float (&vl)[PPT], float (&raw)[PPT], float (&al)[PPT]) {
            const uint32_t pos = lo + k - start;   // position in the tile list
            const float4 g = s_rec[3 * k];
            const float4 h = s_rec[3 * k + 1];
            dx = fx - g.x;
            const float A = exp2_col_a(g.w, h.x, dx), B = exp2_col_t(g.y, g.z, fx);
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                vl[p] = exp2_line(h.y, B, fy[p]);   // the forward's exponent, term by term
                raw[p] = __builtin_amdgcn_exp2f(fmaf(-vl[p], vl[p], A));
                const float alpha = clamp_alpha(raw[p], amax_bits);
                al[p] = (real && pos < last[p] && alpha >= amin) ? alpha : 0.0f;
            }
        };
        // record k's terms at the thread's pixels, back to front (an alpha of 0
        // leaves T and R unchanged and adds nothing)
        auto grad = [&](int k, float dx, const float (&vl)[PPT], const float (&raw)[PPT], const float (&al)[PPT],
                        float (&v)[kVals]) {
            const float4 h = s_rec[3 * k + 1];
            const float4 e = s_rec[3 * k + 2];   // b, gy, -, id
            float D = 0.f, Dv = 0.f, Dy = 0.f, Dyy = 0.f;
            v[6] = v[7] = v[8] = 0.f;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                T[p] *= __builtin_amdgcn_rcpf(1.0f - al[p]);   // transmittance in front of i
                const float w = al[p] * T[p];
                v[6] = fmaf(w, g0[p], v[6]);
                v[7] = fmaf(w, g1[p], v[7]);
                v[8] = fmaf(w, g2[p], v[8]);
                const float d = fmaf(h.z, g0[p], fmaf(h.w, g1[p], e.x * g2[p])) - R[p];   // c.g - R
                R[p] = fmaf(al[p], d, R[p]);
                const float dpow = raw[p] < amax ? al[p] * (T[p] * d) : 0.0f;
                const float dy = fy[p] - e.y;
                D += dpow;
                Dv = fmaf(vl[p], dpow, Dv);
                Dy = fmaf(dy, dpow, Dy);
                Dyy = fmaf(dy * dy, dpow, Dyy);
            }
            v[0] = D;
            v[1] = dx * D;
            v[2] = Dv;
            v[3] = (dx * dx) * D;
            v[4] = dx * Dy;
            v[5] = Dyy;
        };
        // records k1 (behind) then k2 (in front); with real2 false only k1
        auto pair = [&](int k1, int k2, bool real2) {
            float x1, x2, l1[PPT], l2[PPT], r1[PPT], a1[PPT], r2[PPT], a2[PPT];
            alphas(k1, true, x1, l1, r1, a1);
            alphas(k2, real2, x2, l2, r2, a2);
            bool any = false;
#pragma unroll
            for (int p = 0; p < PPT; ++p) any = any || a1[p] > 0.0f || a2[p] > 0.0f;
            if (__ballot(any) == 0ull) return;
            float v1[kVals], v2[kVals];
            grad(k1, x1, l1, r1, a1, v1);
            grad(k2, x2, l2, r2, a2, v2);
            // sums over neighbouring lane pairs, record 1 kept in the even lanes and
            // record 2 in the odd ones; then sums over lanes of one parity in each
            // row of 16
            float v[kVals];
#pragma unroll
            for (int j = 0; j < kVals; ++j) {
                const float p1 = v1[j] + dpp_of<0xB1>(v1[j]);   // quad_perm(1,0,3,2)
                const float p2 = v2[j] + dpp_of<0xB1>(v2[j]);
                float x = odd ? p2 : p1;
                x += dpp_of<0x4E>(x);                  // quad_perm(2,3,0,1)
                x += dpp_of<0x124>(x);                 // row_ror:4
                x += dpp_of<0x128>(x);                 // row_ror:8
                v[j] = x;
            }
            if ((lane & 14) == 14 && (!odd || real2)) {
                float *acc = s_acc + (odd ? k2 : k1) * kVals;
#pragma unroll
                for (int j = 0; j < kVals; ++j) atomicAdd(acc + j, v[j]);
            }
        };
        if (kBits && cull) {
            // only the records whose ellipse reaches this wavefront's cell, back to front
            for (int c = (cnt - 1) / 64; c >= 0; --c) {
                const uint64_t word = s_bits[wave * kWords + c];
                uint64_t bits = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(word >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)word);
                while (bits != 0ull) {
                    const int b1 = 63 - __builtin_clzll(bits);
                    const uint64_t rest = bits & ~(1ull << b1);
                    const bool two = rest != 0ull;
                    const int b2 = two ? 63 - __builtin_clzll(rest) : b1;
                    bits = two ? rest & ~(1ull << b2) : 0ull;
                    pair(c * 64 + b1, c * 64 + b2, two);
                }
            }
        } else {
            for (int k = cnt - 1; k >= 0; k -= 2) pair(k, k > 0 ? k - 1 : k, k > 0);
        }
        __syncthreads();
        // sums to gradients, one global add per (Gaussian, value) for the whole tile
        for (int k = threadIdx.x; k < cnt; k += NT) {
            float m[kVals];
            bool nz = false;
#pragma unroll
            for (int j = 0; j < kVals; ++j) {
                m[j] = s_acc[k * kVals + j];
                s_acc[k * kVals + j] = 0.0f;
                nz = nz || m[j] != 0.0f;
            }
            if (!nz) continue;
            const float4 g = s_rec[3 * k];       // gx, q s, c0, kx
            const float q = s_rec[3 * k + 1].y;
            const float4 e = s_rec[3 * k + 2];   // b, gy, opacity, id
            const uint32_t id = __float_as_uint(e.w);
            float out[kVals];
            out[0] = -2.0f * kLn2 * (g.w * m[1] - g.y * m[2]);   // d u
            out[1] = 2.0f * kLn2 * q * m[2];                     // d v
            out[2] = -0.5f * m[3];                               // d conic a
            out[3] = -m[4];                                      // d conic b
            out[4] = -0.5f * m[5];                               // d conic c
            out[5] = m[0] / e.z;                                 // d opacity
            out[6] = m[6];
            out[7] = m[7];
            out[8] = m[8];
            float *dst = a.g2d + (int64_t)id * kVals;
#pragma unroll
            for (int j = 0; j < kVals; ++j)
                if (out[j] != 0.0f) atomicAdd(dst + j, out[j]);
        }
    }
}

// Pixels per thread in the adjoint: 1 for 8x8 tiles, else 4 when the forward
// took 4 and 2 otherwise.
struct BwdLaunch {
    BwdArgs a;
    int32_t ppt;
};
template <int TW, int TH, int BATCH>
void launch_bwd(const BwdLaunch &l, int n_tiles, hipStream_t s) {
    if constexpr (TW * TH == 64) {
        hipLaunchKernelGGL((composite_bwd_kernel<TW, TH, BATCH, 1>), dim3(n_tiles), dim3(64), 0, s, l.a);
    } else if (l.ppt == 4) {
        hipLaunchKernelGGL((composite_bwd_kernel<TW, TH, BATCH, 4>), dim3(n_tiles), dim3(TW * TH / 4), 0, s, l.a);
    } else {
        hipLaunchKernelGGL((composite_bwd_kernel<TW, TH, BATCH, 2>), dim3(n_tiles), dim3(TW * TH / 2), 0, s, l.a);
    }
}

}  // namespace

hipError_t launch_composite_backward(const RenderParams &rp, int32_t W, int32_t H, int32_t batch, int32_t ppt,
                                     const uint32_t *ranges, const uint32_t *ids, const Rec2D *rec,
                                     const float *T_final, const uint32_t *n_contrib,
                                     const float *dL_drgb, float *g2d, int64_t /*n_proc_max*/,
                                     const uint32_t *order, hipStream_t s) {
    BwdLaunch l{BwdArgs{rp, W, H, ranges, ids, rec, T_final, n_contrib, dL_drgb, g2d, order}, ppt};
    const int n_tiles = rp.tiles_x * rp.tiles_y;
    FDGS_DISPATCH(launch_bwd, l);
    return hipGetLastError();
}

}  // namespace fdgs
