// Device math for one 4D Gaussian, shared by the forward and adjoint
// kernels: parameter loading, the 4D rotation, temporal slicing (Eq. 1,
// Eq. 3), the local-affine projection, the pixel footprint and the SH colour.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "fdgs_internal.h"

namespace fdgs {

struct Gauss4 {
    double mu[4];
    double ls[4];
    double ql[4];
    double qr[4];
    double logit;
};

__device__ __forceinline__ bool load_gaussian(const KModel &m, int64_t g, Gauss4 &G) {
    const int64_t n = m.n;
    if (g < 0 || g >= n) return false;   // an out-of-range index draws nothing
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        G.mu[k] = (double)m.mean[k * n + g];
        G.ls[k] = (double)m.log_scale[k * n + g];
        G.ql[k] = (double)m.q_left[k * n + g];
        G.qr[k] = (double)m.q_right[k * n + g];
        ok = ok && isfinite(G.mu[k]) && isfinite(G.ls[k]) && isfinite(G.ql[k]) && isfinite(G.qr[k]);
    }
    G.logit = (double)m.logit[g];
    ok = ok && isfinite(G.logit);
    const double nl = G.ql[0] * G.ql[0] + G.ql[1] * G.ql[1] + G.ql[2] * G.ql[2] + G.ql[3] * G.ql[3];
    const double nr = G.qr[0] * G.qr[0] + G.qr[1] * G.qr[1] + G.qr[2] * G.qr[2] + G.qr[3] * G.qr[3];
    return ok && nl >= 1e-12 && nr >= 1e-12;
}

// M = R diag(s), with R the matrix of x -> q_l * x * q_r (unit quaternions),
// i.e. the product of q_l's left-multiplication matrix and q_r's
// right-multiplication matrix.
__device__ __forceinline__ void scaled_rotation(const Gauss4 &G, double M[4][4]) {
    double a[4], p[4];
    const double il = 1.0 / sqrt(G.ql[0] * G.ql[0] + G.ql[1] * G.ql[1] + G.ql[2] * G.ql[2] + G.ql[3] * G.ql[3]);
    const double ir = 1.0 / sqrt(G.qr[0] * G.qr[0] + G.qr[1] * G.qr[1] + G.qr[2] * G.qr[2] + G.qr[3] * G.qr[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) { a[k] = G.ql[k] * il; p[k] = G.qr[k] * ir; }
    const double L[4][4] = {{a[0], -a[1], -a[2], -a[3]},
                            {a[1], a[0], -a[3], a[2]},
                            {a[2], a[3], a[0], -a[1]},
                            {a[3], -a[2], a[1], a[0]}};
    const double Rr[4][4] = {{p[0], -p[1], -p[2], -p[3]},
                             {p[1], p[0], p[3], -p[2]},
                             {p[2], -p[3], p[0], p[1]},
                             {p[3], p[2], -p[1], p[0]}};
    double s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = exp(G.ls[k]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += L[i][k] * Rr[k][j];
            M[i][j] = acc * s[j];
        }
}

struct Sliced {
    double mean3[3];
    double cov3[6];   // xx xy xz yy yz zz
    double p;
    bool ok;
};

// Eq. 1 and Eq. 3 at time t.  With M = R diag(s), A = M[0:3,:] and u = M[3,:]:
// Sigma_44 = u.u, Sigma_{1:3,4} = A u and the conditional covariance
// Sigma_{1:3,1:3} - A u u^T A^T / Sigma_44 equals B B^T with
// B = A - (A u) u^T / Sigma_44 (a projector form that stays positive
// semi-definite under rounding).
__device__ __forceinline__ Sliced slice_gaussian(const Gauss4 &G, double t) {
    double M[4][4];
    scaled_rotation(G, M);
    Sliced S;
    const double s44 = M[3][0] * M[3][0] + M[3][1] * M[3][1] + M[3][2] * M[3][2] + M[3][3] * M[3][3];
    double b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        b[i] = M[i][0] * M[3][0] + M[i][1] * M[3][1] + M[i][2] * M[3][2] + M[i][3] * M[3][3];
    const double dt = t - G.mu[3];
    const double inv = 1.0 / s44;
    double B[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        S.mean3[i] = G.mu[i] + b[i] * inv * dt;
#pragma unroll
        for (int k = 0; k < 4; ++k) B[i][k] = M[i][k] - b[i] * inv * M[3][k];
    }
    int c = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            S.cov3[c++] = B[i][0] * B[j][0] + B[i][1] * B[j][1] + B[i][2] * B[j][2] + B[i][3] * B[j][3];
    S.p = exp(-0.5 * dt * dt * inv);
    S.ok = s44 > 0.0 && isfinite(s44) && isfinite(S.mean3[0]) && isfinite(S.mean3[1]) &&
           isfinite(S.mean3[2]);
    return S;
}

__device__ __forceinline__ double sigma44_of(const Gauss4 &G) {
    double M[4][4];
    scaled_rotation(G, M);
    return M[3][0] * M[3][0] + M[3][1] * M[3][1] + M[3][2] * M[3][2] + M[3][3] * M[3][3];
}

struct Projected {
    double u, v, z;
    double c00, c01, c11;   // Sigma_2D
    bool ok;
};

// Local-affine projection of the conditional Gaussian (the usual EWA
// splatting Jacobian at the conditional mean) plus the dilation term.
__device__ __forceinline__ Projected project(const KCam &cam, const Sliced &S, double dilation) {
    Projected P;
    const double *R = cam.R;
    const double x = R[0] * S.mean3[0] + R[1] * S.mean3[1] + R[2] * S.mean3[2] + cam.t[0];
    const double y = R[3] * S.mean3[0] + R[4] * S.mean3[1] + R[5] * S.mean3[2] + cam.t[1];
    const double z = R[6] * S.mean3[0] + R[7] * S.mean3[1] + R[8] * S.mean3[2] + cam.t[2];
    P.z = z;
    P.ok = z > cam.znear && isfinite(z);
    const double zs = P.ok ? z : 1.0;
    const double j00 = cam.fx / zs, j02 = -cam.fx * x / (zs * zs);
    const double j11 = cam.fy / zs, j12 = -cam.fy * y / (zs * zs);
    double T0[3], T1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T0[j] = j00 * R[j] + j02 * R[6 + j];
        T1[j] = j11 * R[3 + j] + j12 * R[6 + j];
    }
    const double *c = S.cov3;
    const double Sm[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
    double V0[3], V1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        V0[i] = Sm[i][0] * T0[0] + Sm[i][1] * T0[1] + Sm[i][2] * T0[2];
        V1[i] = Sm[i][0] * T1[0] + Sm[i][1] * T1[1] + Sm[i][2] * T1[2];
    }
    P.c00 = T0[0] * V0[0] + T0[1] * V0[1] + T0[2] * V0[2] + dilation;
    P.c01 = T0[0] * V1[0] + T0[1] * V1[1] + T0[2] * V1[2];
    P.c11 = T1[0] * V1[0] + T1[1] * V1[1] + T1[2] * V1[2] + dilation;
    P.u = cam.fx * x / zs + cam.cx;
    P.v = cam.fy * y / zs + cam.cy;
    const double det = P.c00 * P.c11 - P.c01 * P.c01;
    P.ok = P.ok && det > 0.0 && isfinite(det) && isfinite(P.u) && isfinite(P.v);
    return P;
}

struct PixRect {
    int x0, y0, x1, y1;
};

// Pixel centres (px + 0.5, py + 0.5) inside the axis-aligned box of the
// ellipse d^T Sigma_2D^{-1} d <= q (half-extents sqrt(q Sxx), sqrt(q Syy)),
// clipped to the image; empty when x0 > x1 or y0 > y1.
__device__ __forceinline__ PixRect pixel_rect(const Projected &P, double q, int W, int H) {
    const double hx = sqrt(q * fmax(P.c00, 0.0));
    const double hy = sqrt(q * fmax(P.c11, 0.0));
    auto clip = [](double a, double hi) { return fmin(fmax(a, -1.0), hi + 1.0); };
    PixRect r;
    r.x0 = max((int)ceil(clip(P.u - hx - 0.5, W)), 0);
    r.x1 = min((int)floor(clip(P.u + hx - 0.5, W)), W - 1);
    r.y0 = max((int)ceil(clip(P.v - hy - 0.5, H)), 0);
    r.y1 = min((int)floor(clip(P.v + hy - 0.5, H)), H - 1);
    return r;
}

// Mahalanobis level beyond which alpha < alpha_min, with a small margin so
// the rectangle stays conservative for the float32 alpha of the compositor.
__device__ __forceinline__ double cut_level(double opac, double alpha_min, int cull,
                                            double vanilla_level) {
    if (!cull) return vanilla_level;
    const double ratio = fmax(opac / alpha_min, 1.0);
    return 2.0 * log(ratio) * (1.0 + 1e-4) + 1e-4;
}

// Real spherical harmonics up to degree 3 (Condon-Shortley phase, index
// k = l*l + l + m) at unit direction d = (x, y, z).
struct ShConst {
    static constexpr float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
    static constexpr float c1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
    static constexpr float c2a = 1.0925484305920792f;   // sqrt(15/pi)/2
    static constexpr float c2b = 0.31539156525252005f;  // sqrt(5/pi)/4
    static constexpr float c2c = 0.54627421529603959f;  // sqrt(15/pi)/4
    static constexpr float c3a = 0.59004358992664352f;  // sqrt(35/(2 pi))/4
    static constexpr float c3b = 2.8906114426405538f;   // sqrt(105/pi)/2
    static constexpr float c3c = 0.45704579946446572f;  // sqrt(21/(2 pi))/4
    static constexpr float c3d = 0.37317633259011540f;  // sqrt(7/pi)/4
    static constexpr float c3e = 1.4453057213202769f;   // sqrt(105/pi)/4
};

__device__ __forceinline__ void sh_basis(float x, float y, float z, float Y[16]) {
    using C = ShConst;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = C::c0;
    Y[1] = -C::c1 * y;
    Y[2] = C::c1 * z;
    Y[3] = -C::c1 * x;
    Y[4] = C::c2a * x * y;
    Y[5] = -C::c2a * y * z;
    Y[6] = C::c2b * (2.0f * zz - xx - yy);
    Y[7] = -C::c2a * x * z;
    Y[8] = C::c2c * (xx - yy);
    Y[9] = -C::c3a * y * (3.0f * xx - yy);
    Y[10] = C::c3b * x * y * z;
    Y[11] = -C::c3c * y * (4.0f * zz - xx - yy);
    Y[12] = C::c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -C::c3c * x * (4.0f * zz - xx - yy);
    Y[14] = C::c3e * z * (xx - yy);
    Y[15] = -C::c3a * x * (xx - 3.0f * yy);
}

// Partial derivatives of the polynomials above with respect to x, y, z.
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float dX[16], float dY[16],
                                              float dZ[16]) {
    using C = ShConst;
    const float xx = x * x, yy = y * y, zz = z * z;
    dX[0] = 0.f; dY[0] = 0.f; dZ[0] = 0.f;
    dX[1] = 0.f; dY[1] = -C::c1; dZ[1] = 0.f;
    dX[2] = 0.f; dY[2] = 0.f; dZ[2] = C::c1;
    dX[3] = -C::c1; dY[3] = 0.f; dZ[3] = 0.f;
    dX[4] = C::c2a * y; dY[4] = C::c2a * x; dZ[4] = 0.f;
    dX[5] = 0.f; dY[5] = -C::c2a * z; dZ[5] = -C::c2a * y;
    dX[6] = -2.0f * C::c2b * x; dY[6] = -2.0f * C::c2b * y; dZ[6] = 4.0f * C::c2b * z;
    dX[7] = -C::c2a * z; dY[7] = 0.f; dZ[7] = -C::c2a * x;
    dX[8] = 2.0f * C::c2c * x; dY[8] = -2.0f * C::c2c * y; dZ[8] = 0.f;
    dX[9] = -6.0f * C::c3a * x * y; dY[9] = -3.0f * C::c3a * (xx - yy); dZ[9] = 0.f;
    dX[10] = C::c3b * y * z; dY[10] = C::c3b * x * z; dZ[10] = C::c3b * x * y;
    dX[11] = 2.0f * C::c3c * x * y; dY[11] = -C::c3c * (4.0f * zz - xx - 3.0f * yy); dZ[11] = -8.0f * C::c3c * y * z;
    dX[12] = -6.0f * C::c3d * x * z; dY[12] = -6.0f * C::c3d * y * z; dZ[12] = C::c3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
    dX[13] = -C::c3c * (4.0f * zz - 3.0f * xx - yy); dY[13] = 2.0f * C::c3c * x * y; dZ[13] = -8.0f * C::c3c * x * z;
    dX[14] = 2.0f * C::c3e * x * z; dY[14] = -2.0f * C::c3e * y * z; dZ[14] = C::c3e * (xx - yy);
    dX[15] = -3.0f * C::c3a * (xx - yy); dY[15] = 6.0f * C::c3a * x * y; dZ[15] = 0.f;
}

// rgb = max(0, sum_k sh_k Y_k(d) + 0.5) per channel; raw[] gets the value
// before the clamp.
// The (degree + 1)^2 x 3 SH coefficients of Gaussian g (coef[k * 3 + ch]);
// the others are set to 0.  All loads are issued before any is used.
__device__ __forceinline__ void load_sh(const float *sh, int64_t n, int64_t g, int degree, float coef[48]) {
    const int nk = (degree + 1) * (degree + 1);
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) coef[k * 3 + ch] = k < nk ? sh[((int64_t)(k * 3 + ch)) * n + g] : 0.0f;
}

__device__ __forceinline__ void sh_eval(const float coef[48], int degree, float dx, float dy, float dz,
                                        float rgb[3], float raw[3] = nullptr) {
    float Y[16];
    sh_basis(dx, dy, dz, Y);
    const int nk = (degree + 1) * (degree + 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < nk) acc += Y[k] * coef[k * 3 + ch];
        if (raw) raw[ch] = acc + 0.5f;
        rgb[ch] = fmaxf(acc + 0.5f, 0.0f);
    }
}

// Coefficients of Gaussian g from the model: its SH planes or, for a
// quantised model, its codebook entry (48 contiguous floats, 16-B aligned).
__device__ __forceinline__ void load_sh_model(const KModel &m, int64_t g, float coef[48]) {
    if (m.sh_index) {
        const int64_t e = min((int64_t)m.sh_index[g], m.n_code - 1);
        const float4 *src = reinterpret_cast<const float4 *>(m.sh_code + e * 48);
        const int nk = (m.sh_degree + 1) * (m.sh_degree + 1);
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const float4 v = src[q];
            coef[4 * q] = v.x;
            coef[4 * q + 1] = v.y;
            coef[4 * q + 2] = v.z;
            coef[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int i = 0; i < 48; ++i)
            if (i / 3 >= nk) coef[i] = 0.0f;
    } else {
        load_sh(m.sh, m.n, g, m.sh_degree, coef);
    }
}

__device__ __forceinline__ void sh_to_rgb(const float *sh, int64_t n, int64_t g, int degree,
                                          float dx, float dy, float dz, float rgb[3],
                                          float raw[3] = nullptr) {
    float coef[48];
    load_sh(sh, n, g, degree, coef);
    sh_eval(coef, degree, dx, dy, dz, rgb, raw);
}

}  // namespace fdgs
