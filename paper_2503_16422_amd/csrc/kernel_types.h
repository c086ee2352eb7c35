// Types passed by value to kernels: camera, model pointers, the 2D record
// the compositor consumes and the render parameters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdgs {

// Camera as passed to kernels (by value).
struct KCam {
    double R[9];
    double t[3];
    double fx, fy, cx, cy, znear;
    int32_t W, H;
};

// Model pointers as passed to kernels.
struct KModel {
    const float *mean, *log_scale, *q_left, *q_right, *logit, *sh;
    int64_t n;
    int32_t sh_degree;
    const uint32_t *sh_index;   // optional: SH from sh_code[sh_index[g]] (48 floats per entry)
    const float *sh_code;
    int64_t n_code;
};

// Per visible Gaussian record consumed by the compositor (64 B, 16-B aligned).
//   a: u_hi, v_hi, u_lo, v_lo    (pixel-space centre as a float pair)
//   b: conic a, b, c, opacity    (Sigma_2D^{-1} = [[a, b], [b, c]]; sigma * p(t))
//   c: r, g, b, depth (float32)
//   d: kx, q, s_hi, s_lo         (the exponent with the square completed in y,
//                                 from the float64 Sigma_2D:
//                                 log2(opacity G) = log2(opacity) + kx dx^2 - q^2 (dy + s dx)^2,
//                                 kx = -log2(e) / (2 Sigma_xx), q^2 = log2(e) Sigma_xx / (2 det),
//                                 s = -Sigma_xy / Sigma_xx = s_hi + s_lo)
struct alignas(16) Rec2D {
    float4 a, b, c, d;
};

struct RenderParams {
    int32_t tile_w, tile_h, tiles_x, tiles_y;
    float bg[3];
    float alpha_min, alpha_max, t_min, dilation;
    int32_t temporal_cull;
    int32_t tile_cull;      // list a record only in the tiles its ellipse reaches
    double vanilla_level;   // cut level without opacity culling, incl. margin
};

}  // namespace fdgs
