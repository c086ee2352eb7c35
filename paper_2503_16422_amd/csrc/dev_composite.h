// Device helpers shared by the compositor and its adjoint: the staged form of
// a record's conic and opacity, the base-2 exponent both kernels evaluate, the
// wavefront-per-cell thread layout with the cells a record reaches, and the
// tile-shape / LDS-batch dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_cull.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace comp {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;

// Pixel offsets are taken from the centre of the 32x32 pixel block that holds
// the tile (the same block for every tile shape, so a pixel's arithmetic does
// not depend on the tiling): a thread's fx, fy lie in [-15.5, 15.5].
constexpr int kBlockSize = 32;
constexpr int kBlockHalf = 16;

// Staged exponent of a record for the block centred at (ox, oy) (absolute
// pixels).  With the square completed in y (Rec2D::d),
//   log2(opacity G) = lo + kx dx^2 - v^2,   v = q (dy + s dx) = q fy + s' fx + c0,
// s' = q s and c0 = -q (gy + s gx) taken in float64 from the centre's float
// pair and the float pair of s: both variable terms are <= 0 (kx < 0), and v,
// the scaled distance to the footprint's centre line, is formed from
// block-sized numbers, so the float32 exponent is accurate to a few 1e-6 of
// its value even for a needle whose centre lies thousands of pixels away.
struct ExpRec {
    float gx, gy;   // centre relative to the block centre
    float q;        // sqrt(-ky)
    float s, c0;    // scaled centre line: v = q fy + s fx + c0
    float kx, lo;
};
__device__ __forceinline__ ExpRec stage_exp(const Rec2D &r, float ox, float oy) {
    const double gx = ((double)r.a.x - (double)ox) + (double)r.a.z;
    const double gy = ((double)r.a.y - (double)oy) + (double)r.a.w;
    const double sl = (double)r.d.z + (double)r.d.w;
    const double q = (double)r.d.y;
    ExpRec e;
    e.gx = (float)gx;
    e.gy = (float)gy;
    e.q = r.d.y;
    e.s = (float)(q * sl);
    e.c0 = (float)(-q * (gy + sl * gx));
    e.kx = r.d.x;
    e.lo = __log2f(r.b.w);
    return e;
}

// The terms that depend on the thread's column only (computed once for the
// thread's PPT pixels): A = kx dx^2 + lo and t = s fx + c0; then per pixel
// v = q fy + t and e = A - v^2.  Every kernel evaluates exactly these
// expressions, so forward, adjoint and all tile shapes take identical alpha
// decisions.
__device__ __forceinline__ float exp2_col_a(float kx, float lo, float dx) { return fmaf(kx * dx, dx, lo); }
__device__ __forceinline__ float exp2_col_t(float s, float c0, float fx) { return fmaf(s, fx, c0); }
__device__ __forceinline__ float exp2_line(float q, float t, float fy) { return fmaf(q, fy, t); }
__device__ __forceinline__ float exp2_at(float q, float A, float t, float fy) {
    const float v = exp2_line(q, t, fy);
    return fmaf(-v, v, A);
}
// min(alpha_max, v) for v = exp2(...) >= +0 (or a NaN): non-negative floats
// order as their bit patterns, so one unsigned minimum gives fminf's result
// (alpha_max for +inf and for a NaN of either sign) without the operand
// canonicalisation fminf needs.
__device__ __forceinline__ float clamp_alpha(float v, uint32_t amax_bits) {
    return __uint_as_float(min(__float_as_uint(v), amax_bits));
}
// Transmittance after blending alpha in front of T.
__device__ __forceinline__ float after(float T, float alpha) { return fmaf(-alpha, T, T); }

// Thread layout of both compositors: each wavefront owns a CW x CH block
// ("cell") of the tile and each of its threads PPT consecutive pixels of one
// column of the cell (TW x TH / PPT threads); the column's dx terms and the
// LDS reads of a record are shared by the thread's PPT pixels.  Cells are 16
// pixels wide where the tile allows, so several wavefronts split a tile into
// blocks that a record's footprint often misses: with several pixels per
// thread, the staging marks in one bitmap per wavefront the records whose
// ellipse reaches its cell, and the wavefront walks only those (a scalar bit
// scan per record).
template <int TW, int TH, int PPT>
struct Cells {
    static constexpr int CW = (TW >= 16 && TH >= 4 * PPT) ? 16 : TW;
    static constexpr int CH = 64 * PPT / CW;
    static constexpr int CX = TW / CW;
    static constexpr int NW = CX * (TH / CH);
    static_assert(TW % CW == 0 && TH % CH == 0 && NW * 64 * PPT == TW * TH, "whole cells per tile");
};

// Bit w set when the record's footprint ellipse reaches a pixel of wavefront
// w's cell of the tile with origin (x0, y0) (every bit when tile culling is
// off, or the ellipse is not usable for it).  One column span per band of
// cell rows, then a range test per cell of the band.
template <int TW, int TH, int PPT>
__device__ __forceinline__ uint32_t reached_cells(const Rec2D &r, const RenderParams &rp, int x0, int y0) {
    using C = Cells<TW, TH, PPT>;
    const CullEllipse e = cull_ellipse(r, rp);
    uint32_t m = 0;
#pragma unroll 1
    for (int band = 0; band < C::NW / C::CX; ++band) {
        const int r0 = y0 + band * C::CH;
        int p0 = x0, p1 = x0 + TW - 1;
        if (!ellipse_band_columns(e, r0, r0 + C::CH - 1, x0, x0 + TW - 1, &p0, &p1)) continue;
#pragma unroll
        for (int cx = 0; cx < C::CX; ++cx) {
            const int c0 = x0 + cx * C::CW;
            if (p0 <= c0 + C::CW - 1 && p1 >= c0) m |= 1u << (band * C::CX + cx);
        }
    }
    return m;
}

}  // namespace comp
}  // namespace fdgs

// Instantiates LAUNCH<TW, TH, BATCH>(ARGS, n_tiles, s) for the supported tile
// shapes and LDS batches; returns hipErrorInvalidValue from the enclosing
// function for others.
#define FDGS_DISPATCH(LAUNCH, ARGS)                                                             \
    do {                                                                                        \
        const int key = rp.tile_w * 1000 + rp.tile_h;                                           \
        bool ok = true;                                                                         \
        if (key == 8008) {                                                                      \
            if (batch == 64) LAUNCH<8, 8, 64>(ARGS, n_tiles, s);                                \
            else if (batch == 128) LAUNCH<8, 8, 128>(ARGS, n_tiles, s);                         \
            else if (batch == 256) LAUNCH<8, 8, 256>(ARGS, n_tiles, s);                         \
            else ok = false;                                                                    \
        } else if (key == 16016) {                                                              \
            if (batch == 64) LAUNCH<16, 16, 64>(ARGS, n_tiles, s);                              \
            else if (batch == 128) LAUNCH<16, 16, 128>(ARGS, n_tiles, s);                       \
            else if (batch == 256) LAUNCH<16, 16, 256>(ARGS, n_tiles, s);                       \
            else ok = false;                                                                    \
        } else if (key == 32008) {                                                              \
            if (batch == 64) LAUNCH<32, 8, 64>(ARGS, n_tiles, s);                               \
            else if (batch == 128) LAUNCH<32, 8, 128>(ARGS, n_tiles, s);                        \
            else if (batch == 256) LAUNCH<32, 8, 256>(ARGS, n_tiles, s);                        \
            else ok = false;                                                                    \
        } else if (key == 32016) {                                                              \
            if (batch == 64) LAUNCH<32, 16, 64>(ARGS, n_tiles, s);                              \
            else if (batch == 128) LAUNCH<32, 16, 128>(ARGS, n_tiles, s);                       \
            else if (batch == 256) LAUNCH<32, 16, 256>(ARGS, n_tiles, s);                       \
            else ok = false;                                                                    \
        } else if (key == 32032) {                                                              \
            if (batch == 64) LAUNCH<32, 32, 64>(ARGS, n_tiles, s);                              \
            else if (batch == 128) LAUNCH<32, 32, 128>(ARGS, n_tiles, s);                       \
            else if (batch == 256) LAUNCH<32, 32, 256>(ARGS, n_tiles, s);                       \
            else if (batch == 512) LAUNCH<32, 32, 512>(ARGS, n_tiles, s);                       \
            else if (batch == 1024) LAUNCH<32, 32, 1024>(ARGS, n_tiles, s);                     \
            else ok = false;                                                                    \
        } else {                                                                                \
            ok = false;                                                                         \
        }                                                                                       \
        if (!ok) return hipErrorInvalidValue;                                                   \
    } while (0)

