// Adjoint of the per-Gaussian preprocess: from the per-Gaussian 2D gradients
// (centre, conic, opacity, colour) back to the 4D parameters (mean, log-scale,
// both quaternions, opacity logit, SH).  The forward quantities are recomputed
// in float64 from the parameters; each thread owns one processed Gaussian, so
// gradients are accumulated with plain read-modify-writes (the processed set
// holds each Gaussian once).
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_gauss.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kBlock = 128;

struct BArgs {
    KModel m;
    const uint32_t *idx;
    const int64_t *n_dev;
    int64_t n_max;
    KCam cam;
    double t;
    double dilation;
    const uint32_t *vis_list;   // processed positions of the visible Gaussians, ascending
    const int64_t *n_vis_dev;   // their count (device)
    const float *g2d;
    fdgs_grads grads;
};

// One thread per visible Gaussian, through the forward's ascending list of
// visible positions: no lane idles on a culled Gaussian, and neighbouring
// threads read and update neighbouring entries of the parameter planes.
__global__ void __launch_bounds__(kBlock) preprocess_bwd_kernel(BArgs a) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t P = a.n_dev ? min(*a.n_dev, a.n_max) : a.n_max;
    if (j >= min(*a.n_vis_dev, P)) return;
    const int64_t i = a.vis_list[j];
    if (i >= P) return;
    const int64_t n = a.m.n;
    const int64_t g = a.idx ? (int64_t)a.idx[i] : i;
    if (g >= n) return;
    Gauss4 G;
    if (!load_gaussian(a.m, g, G)) return;
    const float *gi = a.g2d + i * 9;
    const double du = gi[0], dv = gi[1];
    const double dca = gi[2], dcb = gi[3], dcc = gi[4];
    const double dop = gi[5];
    const double drgb[3] = {gi[6], gi[7], gi[8]};

    // ---- forward recompute (float64) ----
    const double nl = sqrt(G.ql[0] * G.ql[0] + G.ql[1] * G.ql[1] + G.ql[2] * G.ql[2] + G.ql[3] * G.ql[3]);
    const double nr = sqrt(G.qr[0] * G.qr[0] + G.qr[1] * G.qr[1] + G.qr[2] * G.qr[2] + G.qr[3] * G.qr[3]);
    double qa[4], qp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { qa[k] = G.ql[k] / nl; qp[k] = G.qr[k] / nr; }
    const double L[4][4] = {{qa[0], -qa[1], -qa[2], -qa[3]},
                            {qa[1], qa[0], -qa[3], qa[2]},
                            {qa[2], qa[3], qa[0], -qa[1]},
                            {qa[3], -qa[2], qa[1], qa[0]}};
    const double Rr[4][4] = {{qp[0], -qp[1], -qp[2], -qp[3]},
                             {qp[1], qp[0], qp[3], -qp[2]},
                             {qp[2], -qp[3], qp[0], qp[1]},
                             {qp[3], qp[2], -qp[1], qp[0]}};
    double s[4], R4[4][4], M[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = exp(G.ls[k]);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += L[r][k] * Rr[k][c];
            R4[r][c] = acc;
            M[r][c] = acc * s[c];
        }
    const double s44 = M[3][0] * M[3][0] + M[3][1] * M[3][1] + M[3][2] * M[3][2] + M[3][3] * M[3][3];
    const double inv = 1.0 / s44;
    double b[3], mean3[3], B[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        b[r] = M[r][0] * M[3][0] + M[r][1] * M[3][1] + M[r][2] * M[3][2] + M[r][3] * M[3][3];
    const double dt = a.t - G.mu[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        mean3[r] = G.mu[r] + b[r] * inv * dt;
#pragma unroll
        for (int k = 0; k < 4; ++k) B[r][k] = M[r][k] - b[r] * inv * M[3][k];
    }
    double S3[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            S3[r][c] = B[r][0] * B[c][0] + B[r][1] * B[c][1] + B[r][2] * B[c][2] + B[r][3] * B[c][3];
    const double p = exp(-0.5 * dt * dt * inv);
    const double sig = 1.0 / (1.0 + exp(-G.logit));

    const double *Rc = a.cam.R;
    const double x = Rc[0] * mean3[0] + Rc[1] * mean3[1] + Rc[2] * mean3[2] + a.cam.t[0];
    const double y = Rc[3] * mean3[0] + Rc[4] * mean3[1] + Rc[5] * mean3[2] + a.cam.t[1];
    const double z = Rc[6] * mean3[0] + Rc[7] * mean3[1] + Rc[8] * mean3[2] + a.cam.t[2];
    const double fx = a.cam.fx, fy = a.cam.fy;
    const double iz = 1.0 / z, iz2 = iz * iz;
    double T[2][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T[0][j] = fx * iz * Rc[j] - fx * x * iz2 * Rc[6 + j];
        T[1][j] = fy * iz * Rc[3 + j] - fy * y * iz2 * Rc[6 + j];
    }
    double V[3][2];   // S3 T^T
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) V[r][c] = S3[r][0] * T[c][0] + S3[r][1] * T[c][1] + S3[r][2] * T[c][2];
    const double c00 = T[0][0] * V[0][0] + T[0][1] * V[1][0] + T[0][2] * V[2][0] + a.dilation;
    const double c01 = T[0][0] * V[0][1] + T[0][1] * V[1][1] + T[0][2] * V[2][1];
    const double c11 = T[1][0] * V[0][1] + T[1][1] * V[1][1] + T[1][2] * V[2][1] + a.dilation;
    const double det = c00 * c11 - c01 * c01;
    const double qa_ = c11 / det, qb_ = -c01 / det, qc_ = c00 / det;   // conic

    // ---- colour ----
    double vdir[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        vdir[k] = mean3[k] + (Rc[k] * a.cam.t[0] + Rc[3 + k] * a.cam.t[1] + Rc[6 + k] * a.cam.t[2]);
    const double vlen = sqrt(vdir[0] * vdir[0] + vdir[1] * vdir[1] + vdir[2] * vdir[2]);
    const double dirx = vdir[0] / vlen, diry = vdir[1] / vlen, dirz = vdir[2] / vlen;
    float coef[48], rgb[3], raw[3];
    load_sh(a.m.sh, n, g, a.m.sh_degree, coef);
    sh_eval(coef, a.m.sh_degree, (float)dirx, (float)diry, (float)dirz, rgb, raw);
    float Y[16], dYx[16], dYy[16], dYz[16];
    sh_basis((float)dirx, (float)diry, (float)dirz, Y);
    sh_basis_grad((float)dirx, (float)diry, (float)dirz, dYx, dYy, dYz);
    const int nk = (a.m.sh_degree + 1) * (a.m.sh_degree + 1);
    double ddir[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float draw = raw[ch] < 0.0f ? 0.0f : (float)drgb[ch];
        if (draw == 0.0f) continue;
        // one channel's gradient plane entries: all loads first, then the stores
        float gsh[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) gsh[k] = k < nk ? a.grads.sh[((int64_t)(k * 3 + ch)) * n + g] : 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k >= nk) continue;
            a.grads.sh[((int64_t)(k * 3 + ch)) * n + g] = gsh[k] + Y[k] * draw;
            const float c = coef[k * 3 + ch] * draw;
            ddir[0] += c * dYx[k];
            ddir[1] += c * dYy[k];
            ddir[2] += c * dYz[k];
        }
    }
    double dmean3[3];
    {
        const double dd = dirx * ddir[0] + diry * ddir[1] + dirz * ddir[2];
        dmean3[0] = (ddir[0] - dirx * dd) / vlen;
        dmean3[1] = (ddir[1] - diry * dd) / vlen;
        dmean3[2] = (ddir[2] - dirz * dd) / vlen;
    }

    // ---- conic -> Sigma_2D -> (T, Sigma3) ----
    // gradient w.r.t. the symmetric conic matrix: [[da, db/2], [db/2, dc]]
    const double Gq[2][2] = {{dca, 0.5 * dcb}, {0.5 * dcb, dcc}};
    const double Q[2][2] = {{qa_, qb_}, {qb_, qc_}};
    double QG[2][2], GS[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) QG[r][c] = Q[r][0] * Gq[0][c] + Q[r][1] * Gq[1][c];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) GS[r][c] = -(QG[r][0] * Q[0][c] + QG[r][1] * Q[1][c]);
    double GS3[3][3];   // T^T GS T
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int w = 0; w < 2; ++w) acc += T[u][r] * GS[u][w] * T[w][c];
            GS3[r][c] = acc;
        }
    double GT[2][3];    // 2 GS T S3
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int k = 0; k < 3; ++k) acc += GS[r][u] * T[u][k] * S3[k][c];
            GT[r][c] = 2.0 * acc;
        }
    double GJ[2][3];    // GT Rc^T
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) GJ[r][c] = GT[r][0] * Rc[3 * c] + GT[r][1] * Rc[3 * c + 1] + GT[r][2] * Rc[3 * c + 2];
    double dxc[3];
    dxc[0] = du * fx * iz + GJ[0][2] * (-fx * iz2);
    dxc[1] = dv * fy * iz + GJ[1][2] * (-fy * iz2);
    dxc[2] = -du * fx * x * iz2 - dv * fy * y * iz2 + GJ[0][0] * (-fx * iz2) + GJ[0][2] * (2.0 * fx * x * iz2 * iz) +
             GJ[1][1] * (-fy * iz2) + GJ[1][2] * (2.0 * fy * y * iz2 * iz);
#pragma unroll
    for (int k = 0; k < 3; ++k) dmean3[k] += Rc[k] * dxc[0] + Rc[3 + k] * dxc[1] + Rc[6 + k] * dxc[2];

    // ---- opacity ----
    const double dsig = dop * p, dp = dop * sig;
    const double dlogit = dsig * sig * (1.0 - sig);

    // ---- Eq. 1 / Eq. 3 adjoint ----
    double dmu[4] = {dmean3[0], dmean3[1], dmean3[2], 0.0};
    double db_[3], dinv = 0.0, ddt = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        db_[r] = dmean3[r] * inv * dt;
        dinv += dmean3[r] * b[r] * dt;
        ddt += dmean3[r] * b[r] * inv;
    }
    ddt += dp * p * (-dt * inv);
    dinv += dp * p * (-0.5 * dt * dt);
    double GB[3][4];   // 2 GS3 B
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            GB[r][k] = 2.0 * (GS3[r][0] * B[0][k] + GS3[r][1] * B[1][k] + GS3[r][2] * B[2][k]);
    double dM[4][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) dM[r][k] = GB[r][k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) acc += GB[r][k] * b[r];
        dM[3][k] = -acc * inv;
        dinv -= acc * M[3][k];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += GB[r][k] * M[3][k];
        db_[r] -= acc * inv;
    }
    const double ds44 = -dinv * inv * inv;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            dM[r][k] += db_[r] * M[3][k];
            dM[3][k] += db_[r] * M[r][k];
        }
#pragma unroll
    for (int k = 0; k < 4; ++k) dM[3][k] += 2.0 * ds44 * M[3][k];
    dmu[3] = -ddt;

    // ---- M = R diag(s), R = L(q_l) R(q_r) ----
    double dR[4][4], dls[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dR[r][c] = dM[r][c] * s[c];
            acc += dM[r][c] * R4[r][c];
        }
        dls[c] = acc * s[c];
    }
    double dL[4][4], dRr[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double accL = 0.0, accR = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                accL += dR[r][k] * Rr[c][k];   // dR Rr^T
                accR += L[k][r] * dR[k][c];    // L^T dR
            }
            dL[r][c] = accL;
            dRr[r][c] = accR;
        }
    double dqa[4], dqp[4];
    dqa[0] = dL[0][0] + dL[1][1] + dL[2][2] + dL[3][3];
    dqa[1] = -dL[0][1] + dL[1][0] - dL[2][3] + dL[3][2];
    dqa[2] = -dL[0][2] + dL[1][3] + dL[2][0] - dL[3][1];
    dqa[3] = -dL[0][3] - dL[1][2] + dL[2][1] + dL[3][0];
    dqp[0] = dRr[0][0] + dRr[1][1] + dRr[2][2] + dRr[3][3];
    dqp[1] = -dRr[0][1] + dRr[1][0] + dRr[2][3] - dRr[3][2];
    dqp[2] = -dRr[0][2] - dRr[1][3] + dRr[2][0] + dRr[3][1];
    dqp[3] = -dRr[0][3] + dRr[1][2] - dRr[2][1] + dRr[3][0];
    const double pa = qa[0] * dqa[0] + qa[1] * dqa[1] + qa[2] * dqa[2] + qa[3] * dqa[3];
    const double pp = qp[0] * dqp[0] + qp[1] * dqp[1] + qp[2] * dqp[2] + qp[3] * dqp[3];
    // all current values first, then the stores (the planes may alias as far as the compiler knows)
    float gm[4], gl[4], gqa[4], gqp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        gm[k] = a.grads.mean[k * n + g];
        gl[k] = a.grads.log_scale[k * n + g];
        gqa[k] = a.grads.q_left[k * n + g];
        gqp[k] = a.grads.q_right[k * n + g];
    }
    const float go = a.grads.opacity_logit[g];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a.grads.mean[k * n + g] = gm[k] + (float)dmu[k];
        a.grads.log_scale[k * n + g] = gl[k] + (float)dls[k];
        a.grads.q_left[k * n + g] = gqa[k] + (float)((dqa[k] - qa[k] * pa) / nl);
        a.grads.q_right[k * n + g] = gqp[k] + (float)((dqp[k] - qp[k] * pp) / nr);
    }
    a.grads.opacity_logit[g] = go + (float)dlogit;
}

}  // namespace

hipError_t launch_preprocess_backward(const KModel &m, const uint32_t *idx, const int64_t *n_dev,
                                      int64_t n_max, const KCam &cam, double t,
                                      const RenderParams &rp, const uint32_t *vis_list,
                                      const int64_t *n_vis_dev, const float *g2d, const fdgs_grads &grads,
                                      hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    BArgs a{m, idx, n_dev, n_max, cam, t, (double)rp.dilation, vis_list, n_vis_dev, g2d, grads};
    const unsigned grid = (unsigned)((n_max + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(preprocess_bwd_kernel, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace fdgs
