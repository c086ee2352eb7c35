// Device helpers shared by the compositor and its adjoint: the staged form of
// a record's conic and opacity, the base-2 exponent both kernels evaluate, and
// the tile-shape / LDS-batch dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include "fdgs_internal.h"

namespace fdgs {
namespace comp {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.69314718055994531f;

// Staged form of a record's conic and opacity: base-2 exponent coefficients
// and log2(opacity), so that
//   opacity * exp(-1/2 d^T conic d) = exp2(ka dx^2 + kb dx dy + kc dy^2 + lo).
__device__ __forceinline__ float4 staged_conic(const Rec2D &r) {
    return make_float4(-0.5f * kLog2e * r.b.x, -kLog2e * r.b.y, -0.5f * kLog2e * r.b.z, __log2f(r.b.w));
}

// Base-2 exponent of opacity x 2D Gaussian at offset (dx, dy):
//   e = ((ka dx) dx + lo) + dy (kb dx + kc dy).
// The dx-only terms are computed once per column when a thread owns several
// pixels of one column; every kernel evaluates exactly this expression, so
// forward, adjoint and all tile shapes take identical alpha decisions.
__device__ __forceinline__ float exp2_col_a(float4 q, float dx) { return fmaf(q.x * dx, dx, q.w); }
__device__ __forceinline__ float exp2_col_b(float4 q, float dx) { return q.y * dx; }
__device__ __forceinline__ float exp2_at(float4 q, float A, float B, float dy) {
    return fmaf(dy, fmaf(q.z, dy, B), A);
}
__device__ __forceinline__ float gauss_exp2(float4 q, float dx, float dy) {
    return exp2_at(q, exp2_col_a(q, dx), exp2_col_b(q, dx), dy);
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
            else ok = false;                                                                    \
        } else {                                                                                \
            ok = false;                                                                         \
        }                                                                                       \
        if (!ok) return hipErrorInvalidValue;                                                   \
    } while (0)

