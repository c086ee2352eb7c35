// Per-tile front-to-back compositing (Eq. 2 with alpha from Eq. 3).
//
// One workgroup per screen tile; a thread owns 1, 2 or 4 pixels of a column.
// The tile's depth-ordered list is walked in batches: the workgroup stages a
// batch of records in LDS (the exponent's staged form relative to the block
// centre, colour), then every pixel evaluates the batch.  A pixel
// stops before the Gaussian that would take its transmittance below t_min;
// the workgroup leaves the list as soon as every pixel has stopped.  No MFMA:
// per (pixel, Gaussian) pair the work is an exponential and a dozen FMAs, not
// a contraction.
//
// Precision: the centre is stored as a float pair (hi + lo) and re-centred on
// the centre of the tile's 32x32 block while staging, and the exponent is
// evaluated with its square completed (every term of one sign), so alpha is
// within a few 1e-6 (relative) of its float64 value for any footprint.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_composite.h"
#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

using namespace comp;

struct CompArgs {
    RenderParams rp;
    int32_t W, H;
    const uint32_t *ranges;
    const uint32_t *ids;
    const Rec2D *rec;
    float *out_rgb;
    float *out_T;
    uint32_t *n_contrib;
    unsigned long long *pairs;   // optional counters: evaluated pairs, then blended pairs
    int32_t ppt;                 // pixels per thread (host-side dispatch only)
    int32_t V;                   // views sharing the launch
    const uint32_t *order;       // longest-first schedule: (view, tile) items, longest list first
    int32_t n_items;             // V x tiles per view
    uint8_t *contrib;            // kMark: per processed entry, set to 1 when blended
    float *weight;               // kWeight: per processed entry, += sum of alpha T
};

// What a compositor instance records beyond colour and transmittance.
enum CompMode {
    kPlain = 0,   // nothing
    kState = 1,   // last contributor per pixel (for the adjoint)
    kCount = 2,   // last contributor and the evaluated-pair count (profiling)
    kMark = 3,    // flags every record some pixel blends (visibility masks)
    kWeight = 4,  // adds every record's blend weights alpha T over the pixels (pruning score)
};

// One (view, tile) item; s_rec is the workgroup's LDS staging array of
// 3 x BATCH float4.  Every thread of the workgroup calls it.
template <int TW, int TH, int BATCH, int PPT, int MODE>
__device__ __forceinline__ void composite_item(const CompArgs &a, int item, float4 *s_rec) {
    constexpr int NT = TW * TH / PPT;
    static_assert(NT % 64 == 0, "whole wavefronts per tile");
    using C = Cells<TW, TH, PPT>;
    // per-wavefront bitmaps of the batch's records that reach its cell (with
    // several cells per tile; a single wavefront per tile walks every record,
    // branching per pixel)
    constexpr bool kBits = C::NW > 1;
    constexpr bool kBranchy = PPT == 1 && !kBits;
    const bool cull = a.rp.tile_cull != 0;   // without tile culling every record reaches every cell
    constexpr int kWords = BATCH / 64;
    __shared__ uint64_t s_bits[kBits ? C::NW * kWords : 1];
    const int n_tiles = a.rp.tiles_x * a.rp.tiles_y;
    const int view = item / n_tiles;
    const int tile = item - view * n_tiles;
    const int tx = tile % a.rp.tiles_x, ty = tile / a.rp.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64), lane = (int)threadIdx.x % 64;
    const int lx = (wave % C::CX) * C::CW + lane % C::CW, ly0 = (wave / C::CX) * C::CH + (lane / C::CW) * PPT;
    const int px = tx * TW + lx, py0 = ty * TH + ly0;
    // offsets from the centre of the enclosing 32x32 block (the same for every
    // tile shape, so a pixel's arithmetic does not depend on the tiling)
    const int bx0 = ((tx * TW) & ~(kBlockSize - 1)) + kBlockHalf, by0 = ((ty * TH) & ~(kBlockSize - 1)) + kBlockHalf;
    const float fx = (float)(px - bx0) + 0.5f;
    const float ox = (float)bx0, oy = (float)by0;
    const uint32_t start = a.ranges[2 * item], end = a.ranges[2 * item + 1];
    const float amin = a.rp.alpha_min, tmin = a.rp.t_min;
    const uint32_t amax_bits = __float_as_uint(a.rp.alpha_max);
    constexpr bool COUNT = MODE == kCount;
    constexpr bool LAST = MODE == kState || MODE == kCount;
    constexpr bool MARK = MODE == kMark;
    constexpr bool WEIGHT = MODE == kWeight;
    constexpr float kInf = __builtin_huge_valf();
    // thr[p]: the transmittance a blend must keep; t_min while the pixel is
    // live, +inf once it has stopped (or lies outside the image), so a stopped
    // pixel fails every later test and its T stays the T at the stop.
    float fy[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], thr[PPT];
    uint32_t last[PPT], stop[PPT], blends[PPT];
    bool all_done = true;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        fy[p] = (float)(py0 + p - by0) + 0.5f;
        T[p] = 1.0f;
        C0[p] = C1[p] = C2[p] = 0.0f;
        last[p] = 0;
        blends[p] = 0;
        // evaluated pairs (profiling): the branchy walk evaluates its list up to
        // its stop; the select-based walk counts the records it evaluates live
        stop[p] = kBranchy ? end - start : 0u;
        const bool inside = px < a.W && py0 + p < a.H;
        thr[p] = inside ? tmin : kInf;
        all_done = all_done && !inside;
    }
    for (uint32_t base = start; base < end; base += BATCH) {
        if constexpr (!kBranchy) {
            bool left = false;
#pragma unroll
            for (int p = 0; p < PPT; ++p) left = left || thr[p] < kInf;
            all_done = !left;
        }
        if (__syncthreads_count(!all_done) == 0) break;
        const int cnt = (int)min((uint32_t)BATCH, end - base);
        // staging: thread t stages records t, t + NT, ... of the batch; with several
        // cells per tile, each wavefront also records, per target wavefront, which
        // of its 64 records reach that wavefront's cell (one ballot per cell)
        for (int k0 = 0; k0 < cnt; k0 += NT) {
            const int k = k0 + (int)threadIdx.x;
            uint32_t cells = 0u;
            if (k < cnt) {
                const uint32_t id = a.ids[base + k];
                const Rec2D r = a.rec[id];
                const ExpRec q = stage_exp(r, ox, oy);
                if constexpr (kBits) {
                    if (cull) cells = reached_cells<TW, TH, PPT>(r, a.rp, tx * TW, ty * TH);
                }
                s_rec[3 * k] = make_float4(q.gx, q.s, q.c0, q.kx);
                s_rec[3 * k + 1] = make_float4(q.lo, q.q, r.c.x, r.c.y);
                s_rec[3 * k + 2] = make_float4(r.c.z, __uint_as_float(id), 0.0f, 0.0f);
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
        if constexpr (kBranchy) {
            if (!all_done) {
                for (int k = 0; k < cnt; ++k) {
                    const float4 g = s_rec[3 * k];
                    const float4 h = s_rec[3 * k + 1];
                    const float dx = fx - g.x;
                    const uint32_t pos = base + k - start + 1;
                    // one pixel: branch, so a wavefront skips the blend when no lane takes it
                    const float e = exp2_at(h.y, exp2_col_a(g.w, h.x, dx), exp2_col_t(g.y, g.z, fx), fy[0]);
                    const float alpha = clamp_alpha(__builtin_amdgcn_exp2f(e), amax_bits);
                    if (alpha < amin) continue;
                    const float test = after(T[0], alpha);
                    if (test < thr[0]) {
                        thr[0] = kInf;
                        if constexpr (COUNT) stop[0] = pos;
                        all_done = true;
                        break;
                    }
                    const float w = T[0] - test;   // the blend weight, as in the multi-pixel walk
                    C0[0] = fmaf(h.z, w, C0[0]);
                    C1[0] = fmaf(h.w, w, C1[0]);
                    C2[0] = fmaf(s_rec[3 * k + 2].x, w, C2[0]);
                    T[0] = test;
                    if constexpr (LAST) last[0] = pos;
                    if constexpr (COUNT) ++blends[0];
                    if constexpr (MARK) {
                        // lanes here blended record k: the lowest one flags it
                        if (lane_id() == __builtin_ctzll(__ballot(1)))
                            a.contrib[__float_as_uint(s_rec[3 * k + 2].y)] = 1;
                    }
                    if constexpr (WEIGHT) atomicAdd(&a.weight[__float_as_uint(s_rec[3 * k + 2].y)], w);
                }
            }
        } else if (__ballot(!all_done) != 0ull) {
            // select-based updates (several pixels per thread, or one pixel and
            // several cells per tile): no branches or lane masks per pixel, and
            // control flow uniform over the wavefront (lanes whose pixels
            // stopped run along with w = 0), so the wavefront sums see every lane
            // alpha of record k at the thread's pixels (clamped to the float with bit
            // pattern cap: alpha_max, or 0 to make the record a no-op)
            auto alphas = [&](int k, float (&al)[PPT], uint32_t cap) {
                const float4 g = s_rec[3 * k];
                const float4 h = s_rec[3 * k + 1];
                const float dx = fx - g.x;
                const float A = exp2_col_a(g.w, h.x, dx), B = exp2_col_t(g.y, g.z, fx);
#pragma unroll
                for (int p = 0; p < PPT; ++p)
                    al[p] = clamp_alpha(__builtin_amdgcn_exp2f(exp2_at(h.y, A, B, fy[p])), cap);
            };
            // blend record k with those alphas (counted: whether it is an evaluated pair)
            auto apply = [&](int k, const float (&al)[PPT], bool counted) {
                const float4 h = s_rec[3 * k + 1];
                const float cb = s_rec[3 * k + 2].x;
                const uint32_t pos = base + k - start + 1;
                bool blended = false;
                float wsum = 0.0f;
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    // blend when alpha reaches alpha_min and the pixel keeps at least
                    // thr (t_min while live); stop when alpha reaches alpha_min but the
                    // transmittance would fall below thr.  The two conditions combine
                    // as lane masks; the new transmittance is one select and the
                    // weight alpha T is its drop, so a skipped or stopped pair
                    // (weight 0) costs nothing more
                    const float alpha = al[p];
                    const float test = after(T[p], alpha);
                    const bool hit = alpha >= amin;
                    const bool ok = hit && test >= thr[p];
                    const float Tn = ok ? test : T[p];
                    const float w = T[p] - Tn;
                    C0[p] = fmaf(h.z, w, C0[p]);
                    C1[p] = fmaf(h.w, w, C1[p]);
                    C2[p] = fmaf(cb, w, C2[p]);
                    if constexpr (LAST) last[p] = ok ? pos : last[p];
                    if constexpr (COUNT) {
                        stop[p] += (counted && thr[p] < kInf) ? 1u : 0u;
                        blends[p] += ok ? 1u : 0u;
                    }
                    T[p] = Tn;
                    thr[p] = hit != ok ? kInf : thr[p];   // alpha reached alpha_min, T would fall below thr
                    if constexpr (MARK) blended = blended || ok;
                    if constexpr (WEIGHT) wsum += w;
                }
                if constexpr (WEIGHT) {
                    // one wave sum, one atomic per record and wavefront
                    const float tot = wave_sum_to_last(wsum);
                    if (lane == 63 && tot != 0.0f) atomicAdd(&a.weight[__float_as_uint(s_rec[3 * k + 2].y)], tot);
                }
                if constexpr (MARK) {
                    const uint64_t m = __ballot(blended);
                    if (m != 0ull && lane == __builtin_ctzll(m)) a.contrib[__float_as_uint(s_rec[3 * k + 2].y)] = 1;
                }
            };
            // two records per step: both alphas first (they do not depend on the
            // transmittance), so the second record's LDS reads and exponentials
            // overlap the first's blend.  With one record left the second is the
            // same record with every alpha 0, which changes nothing.
            auto blend2 = [&](int k1, int k2, bool two) {
                float a1[PPT], a2[PPT];
                alphas(k1, a1, amax_bits);
                alphas(k2, a2, two ? amax_bits : 0u);
                apply(k1, a1, true);
                apply(k2, a2, two);
            };
            // whether some pixel of the wavefront is still live
            auto live = [&]() {
                bool left = false;
#pragma unroll
                for (int p = 0; p < PPT; ++p) left = left || thr[p] < kInf;
                return __ballot(left) != 0ull;
            };
            if (kBits && cull) {
                // only the records whose ellipse reaches this wavefront's cell, in
                // order; the liveness test every 8 of them
                int since = 0;
                bool more = true;
                for (int c = 0; c < cnt && more; c += 64) {
                    const uint64_t word = s_bits[wave * kWords + c / 64];
                    uint64_t bits = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(word >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)word);
                    while (bits != 0ull) {
                        const int k1 = c + (int)__builtin_ctzll(bits);
                        const uint64_t rest = bits & (bits - 1ull);   // without k1
                        const bool two = rest != 0ull;
                        const int k2 = two ? c + (int)__builtin_ctzll(rest) : k1;
                        bits = rest & (rest - 1ull);                  // 0 when rest is 0
                        blend2(k1, k2, two);
                        since += 2;
                        if (since >= 8) {
                            since = 0;
                            if (!live()) {
                                more = false;
                                break;
                            }
                        }
                    }
                }
            } else {
                // groups of 8 records, leaving the batch once no pixel of the wavefront is live
                for (int k0 = 0; k0 < cnt; k0 += 8) {
                    const int kn = min(cnt, k0 + 8);
                    for (int k = k0; k < kn; k += 2) blend2(k, min(k + 1, kn - 1), k + 1 < kn);
                    if (!live()) break;
                }
            }
        }
    }
    const int64_t plane = (int64_t)a.W * a.H;
    float *out_rgb = a.out_rgb + (int64_t)view * 3 * plane;
    uint32_t evaluated = 0, blended = 0;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int py = py0 + p;
        if (px < a.W && py < a.H) {
            const int64_t pix = (int64_t)py * a.W + px;
            out_rgb[pix] = C0[p] + T[p] * a.rp.bg[0];
            out_rgb[plane + pix] = C1[p] + T[p] * a.rp.bg[1];
            out_rgb[2 * plane + pix] = C2[p] + T[p] * a.rp.bg[2];
            if (a.out_T) a.out_T[view * plane + pix] = T[p];
            if constexpr (LAST) {
                if (a.n_contrib) a.n_contrib[view * plane + pix] = last[p];
            }
            evaluated += stop[p];
            blended += blends[p];
        }
    }
    if constexpr (COUNT) {
        const unsigned long long w = wave_sum((unsigned long long)evaluated);
        const unsigned long long b = wave_sum((unsigned long long)blended);
        if (lane_id() == 0) {
            atomicAdd(a.pairs, w);
            atomicAdd(a.pairs + 1, b);
        }
    }
}

// One workgroup per (view, tile) item.  Raster schedule (ORDERED false):
// workgroup b renders item b (tiles in raster order, views in turn).
// Longest-first schedule (ORDERED true): workgroup b renders item a.order[b],
// the items sorted by list length, longest first.  A launch lasts at least as
// long as its longest lists; dispatched first, they run beside the rest of
// the launch instead of alone at its end (headline frame: 110 -> 92 us at LDS
// batch 512).  Workgroups go to the XCDs in turn, so the longest lists are
// spread over all of them.  With up to two pixels per thread the register
// budget is held to eight wavefronts per SIMD (where the LDS allows as many);
// four pixels need more registers than that.
template <int TW, int TH, int BATCH, int PPT, int MODE, bool ORDERED>
__global__ void __launch_bounds__(TW *TH / PPT) __attribute__((amdgpu_waves_per_eu(PPT == 4 ? 1 : 8)))
composite_kernel(CompArgs a) {
    // per staged record three float4 at one address: gx, s, c0, kx |
    // log2 opacity, q, r, g | b, id, -, - (the exponent's staged form)
    __shared__ float4 s_rec[3 * BATCH];
    const int item = ORDERED ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
    composite_item<TW, TH, BATCH, PPT, MODE>(a, item, s_rec);
}

// Visibility flags (bytes) to LSB-first bit words: one ballot per wavefront.
__global__ void __launch_bounds__(256) flags_to_bits_kernel(const uint8_t *flags, int64_t n, uint32_t *bits) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t m = __ballot(g < n && flags[g] != 0);
    const int lane = lane_id();
    const int64_t word = g >> 5;
    if ((lane == 0 || lane == 32) && word < (n + 31) / 32)
        bits[word] = lane == 0 ? (uint32_t)(m & 0xffffffffu) : (uint32_t)(m >> 32);
}

// Orders the V x tiles items by the length of their lists, longest first, in
// classes a quarter of an octave wide (bit length and the two bits after the
// leading one; one workgroup; order inside a class is arbitrary, which only
// affects scheduling).
constexpr int kOrderNT = 1024;
__global__ void __launch_bounds__(kOrderNT) tile_order_kernel(const uint32_t *ranges, int32_t n_items,
                                                              uint32_t *order) {
    constexpr int kClasses = 33 * 4;
    __shared__ uint32_t s_cnt[kClasses];
    if (threadIdx.x < kClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    auto cls = [&](int i) {
        const uint32_t len = ranges[2 * i + 1] - ranges[2 * i];
        const int b = len ? 32 - __clz(len) : 0;   // bit length, 0 (empty) .. 32
        return b * 4 + (b >= 3 ? (int)((len >> (b - 3)) & 3u) : 0);
    };
    for (int i = threadIdx.x; i < n_items; i += kOrderNT) atomicAdd(&s_cnt[cls(i)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int c = kClasses - 1; c >= 0; --c) {
            const uint32_t k = s_cnt[c];
            s_cnt[c] = run;
            run += k;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_items; i += kOrderNT) order[atomicAdd(&s_cnt[cls(i)], 1u)] = (uint32_t)i;
}

template <int TW, int TH, int BATCH, int PPT, int MODE>
void launch_fwd_sched(const CompArgs &a, int n_items, hipStream_t s) {
    constexpr int NT = TW * TH / PPT;
    if (a.order) {
        hipLaunchKernelGGL((composite_kernel<TW, TH, BATCH, PPT, MODE, true>), dim3(n_items), dim3(NT), 0, s, a);
    } else {
        hipLaunchKernelGGL((composite_kernel<TW, TH, BATCH, PPT, MODE, false>), dim3(n_items), dim3(NT), 0, s, a);
    }
}

template <int TW, int TH, int BATCH, int PPT>
void launch_fwd_ppt(const CompArgs &a, int n_tiles, hipStream_t s) {
    if (a.contrib)
        launch_fwd_sched<TW, TH, BATCH, PPT, kMark>(a, n_tiles, s);
    else if (a.weight)
        launch_fwd_sched<TW, TH, BATCH, PPT, kWeight>(a, n_tiles, s);
    else if (a.pairs)
        launch_fwd_sched<TW, TH, BATCH, PPT, kCount>(a, n_tiles, s);
    else if (a.n_contrib)
        launch_fwd_sched<TW, TH, BATCH, PPT, kState>(a, n_tiles, s);
    else
        launch_fwd_sched<TW, TH, BATCH, PPT, kPlain>(a, n_tiles, s);
}

// Pixels per thread: 1 for 8x8 tiles (one wavefront per tile), a.ppt (1, 2
// or 4) for the 256-pixel tiles.
template <int TW, int TH, int BATCH>
void launch_fwd(const CompArgs &a, int n_tiles, hipStream_t s) {
    if constexpr (TW * TH == 64) {
        launch_fwd_ppt<TW, TH, BATCH, 1>(a, n_tiles, s);
    } else {
        if (a.ppt == 1) launch_fwd_ppt<TW, TH, BATCH, 1>(a, n_tiles, s);
        else if (a.ppt == 2) launch_fwd_ppt<TW, TH, BATCH, 2>(a, n_tiles, s);
        else launch_fwd_ppt<TW, TH, BATCH, 4>(a, n_tiles, s);
    }
}

}  // namespace

hipError_t launch_composite(const RenderParams &rp, int32_t W, int32_t H, int32_t V, int32_t batch,
                            const uint32_t *ranges, const uint32_t *ids, const Rec2D *rec,
                            float *out_rgb, float *out_T, uint32_t *n_contrib,
                            uint64_t *pair_counter, int32_t ppt, uint32_t *sched, uint8_t *contrib,
                            float *weight, hipStream_t s) {
    if (ppt != 1 && ppt != 2 && ppt != 4) return hipErrorInvalidValue;
    const int n_tiles = rp.tiles_x * rp.tiles_y * V;
    const bool side = contrib || weight;   // visibility or score pass: no state, no counters
    CompArgs a{rp, W, H, ranges, ids, rec, out_rgb, out_T, side ? nullptr : n_contrib,
               side ? nullptr : reinterpret_cast<unsigned long long *>(pair_counter), ppt, V,
               sched, n_tiles, contrib, contrib ? nullptr : weight};
    FDGS_DISPATCH(launch_fwd, a);
    return hipGetLastError();
}

hipError_t launch_tile_order(const uint32_t *ranges, int32_t n_items, uint32_t *order, hipStream_t s) {
    if (n_items > 0) hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(kOrderNT), 0, s, ranges, n_items, order);
    return hipGetLastError();
}

hipError_t launch_flags_to_bits(const uint8_t *flags, int64_t n, uint32_t *bits, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(flags_to_bits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, flags, n, bits);
    return hipGetLastError();
}

}  // namespace fdgs
