// Tile culling by the footprint ellipse.
//
// A record is drawn at pixel centre (X, Y) only if the compositor's alpha
// reaches alpha_min there, i.e. inside the ellipse
//   a dx^2 + 2 b dx dy + c dy^2 <= q,   (dx, dy) = (X - u, Y - v),
// of its conic at the cut level q.  Listing a record in every tile of its
// bounding rectangle also lists it in the rectangle's tiles the ellipse
// misses (a rotated, elongated footprint leaves most of them empty).  Here
// each tile row of the rectangle gets the columns the ellipse reaches: over
// the row's band of pixel-centre heights the ellipse spans x from its left
// boundary's minimum to its right boundary's maximum, both in closed form, so
// a record costs one evaluation per tile row.  Skipped tiles hold no pixel
// the compositor would blend, so the image is unchanged.
//
// Conservativeness.  The ellipse is taken from the very float32 values the
// compositor reads (centre, conic, opacity).  The compositor's float32
// exponent errs by a few roundings of its largest term, at most kappa times
// the quadratic form for a conic of condition number kappa, so the level
// grows by 2e-6 kappa_b (relative; kappa_b = (a + c)^2 / det >= kappa) and a
// few 1e-6.  The span itself is evaluated in float32 with the square root's
// argument raised by 1e-6 of its terms and the span widened by 1e-4 of its
// terms plus 1e-3 px, far above the float32 rounding of those steps; the
// centre offsets are added in float64.  Conics with kappa_b above 4e5, or not
// positive definite in float32, keep every tile of the rectangle.
//
// The per-Gaussian tile count (preprocess) and the instance emission
// (duplicate) call the same functions on the same inputs with contraction
// off, so both see the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "fdgs_internal.h"

namespace fdgs {

struct CullEllipse {
    double u, v;      // centre, px
    float a, b;       // conic's xx and xy terms; a == 0 marks "keep the whole rectangle"
    float ia;         // 1 / a
    float det;        // a c - b^2
    float q;          // level incl. margins
    float dyx;        // dy of the rightmost point; the leftmost lies at -dyx
};

// Cut level from the record's float32 opacity, as the rectangle's level is
// from the float64 one (2 ln(opacity / alpha_min) with its margin when culling
// by opacity, else the fixed level).
__device__ inline CullEllipse cull_ellipse(const Rec2D &r, const RenderParams &rp) {
#pragma clang fp contract(off)
    CullEllipse e;
    e.u = (double)r.a.x + (double)r.a.z;
    e.v = (double)r.a.y + (double)r.a.w;
    e.a = 0.0f;
    e.b = 0.0f;
    e.ia = 0.0f;
    e.det = 0.0f;
    e.q = 0.0f;
    e.dyx = 0.0f;
    if (!rp.tile_cull) return e;
    const float a = r.b.x, b = r.b.y, c = r.b.z;
    const float det = (float)((double)a * (double)c - (double)b * (double)b);   // exact products
    if (!(a > 0.0f) || !(c > 0.0f) || !(det > 0.0f)) return e;
    const float kb = (a + c) * (a + c) / det;
    if (!(kb <= 4e5f)) return e;
    float q;
    if (rp.temporal_cull) {
        const float ratio = fmaxf(r.b.w / rp.alpha_min, 1.0f);
        q = 2.0f * logf(ratio) * (1.0f + 1e-4f) + 1e-4f;
    } else {
        q = (float)rp.vanilla_level;
    }
    q = q * (1.0f + 2e-6f * kb + 4e-6f) + 4e-6f;
    e.a = a;
    e.b = b;
    e.ia = 1.0f / a;
    e.det = det;
    e.q = q;
    e.dyx = -b * sqrtf(q / (c * det));
    return e;
}

// Pixel columns [*p0, *p1] that the ellipse reaches over pixel rows
// [r0, r1], clipped to [x0, x1]; false when it reaches none.
__device__ inline bool ellipse_row_span(const CullEllipse &e, int r0, int r1, int x0, int x1, int *p0,
                                        int *p1) {
#pragma clang fp contract(off)
    if (!(e.a > 0.0f)) {
        *p0 = x0;
        *p1 = x1;
        return true;
    }
    const float d0 = (float)(((double)r0 + 0.5) - e.v), d1 = (float)(((double)r1 + 0.5) - e.v);
    // left boundary x_l(dy) is convex with its minimum at -dyx, the right one
    // concave with its maximum at +dyx: clamp those heights into the band
    const float dl = fminf(fmaxf(-e.dyx, d0), d1);
    const float dr = fminf(fmaxf(e.dyx, d0), d1);
    const float aq = e.a * e.q;
    const float tl = e.det * (dl * dl), tr = e.det * (dr * dr);
    const float sl = sqrtf(fmaxf((aq - tl) + 1e-6f * (aq + tl), 0.0f));
    const float sr = sqrtf(fmaxf((aq - tr) + 1e-6f * (aq + tr), 0.0f));
    const float bl = e.b * dl, br = e.b * dr;
    const float ol = (-bl - sl) * e.ia - (1e-4f * (fabsf(bl) + sl) * e.ia + 1e-3f);
    const float orr = (-br + sr) * e.ia + (1e-4f * (fabsf(br) + sr) * e.ia + 1e-3f);
    // pixel px is reached when u + ol <= px + 0.5 <= u + orr
    const double cl = fmax(ceil((e.u + (double)ol) - 0.5), (double)x0);
    const double cr = fmin(floor((e.u + (double)orr) - 0.5), (double)x1);
    if (!(cl <= cr)) return false;
    *p0 = (int)cl;
    *p1 = (int)cr;
    return true;
}

// Pixel columns [*p0, *p1] (within [x0, x1]) that the ellipse may reach over
// rows [r0, r1]; false when it reaches no pixel centre of the block.  Every
// point at height dy has a quadratic form of at least (det / a) dy^2, so a
// band whose nearest height to the centre already exceeds the level holds no
// such pixel; otherwise the band's column span decides.
__device__ inline bool ellipse_band_columns(const CullEllipse &e, int r0, int r1, int x0, int x1, int *p0,
                                            int *p1) {
#pragma clang fp contract(off)
    if (!(e.a > 0.0f)) {
        *p0 = x0;
        *p1 = x1;
        return true;
    }
    const float d0 = (float)(((double)r0 + 0.5) - e.v), d1 = (float)(((double)r1 + 0.5) - e.v);
    const float dn = (d0 <= 0.0f && d1 >= 0.0f) ? 0.0f : fminf(fabsf(d0), fabsf(d1));
    const float aq = e.a * e.q, tn = e.det * (dn * dn);
    if ((aq - tn) + 1e-6f * (aq + tn) < 0.0f) return false;
    return ellipse_row_span(e, r0, r1, x0, x1, p0, p1);
}

// Tile columns [*c0, *c1] of tile row ty for a record with pixel rectangle
// rect (x0, y0, x1, y1); false when the row is empty.
__device__ inline bool tile_row_span(const CullEllipse &e, int4 rect, int ty, int tw, int th, int *c0, int *c1) {
    const int r0 = max(ty * th, rect.y), r1 = min(ty * th + th - 1, rect.w);
    int p0, p1;
    if (!ellipse_row_span(e, r0, r1, rect.x, rect.z, &p0, &p1)) return false;
    *c0 = p0 / tw;
    *c1 = p1 / tw;
    return true;
}

// Tiles listed for a record with pixel rectangle `rect` (non-empty).
__device__ inline uint32_t count_tiles(const CullEllipse &e, int4 rect, int tw, int th) {
    const int ty0 = rect.y / th, ty1 = rect.w / th;
    if (!(e.a > 0.0f)) return (uint32_t)((rect.z / tw - rect.x / tw + 1) * (ty1 - ty0 + 1));
    uint32_t n = 0;
    for (int ty = ty0; ty <= ty1; ++ty) {
        int c0, c1;
        if (tile_row_span(e, rect, ty, tw, th, &c0, &c1)) n += (uint32_t)(c1 - c0 + 1);
    }
    return n;
}

}  // namespace fdgs
