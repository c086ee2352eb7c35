/*
 * FP64 brute-force compositing for the oracle (TEST INFRASTRUCTURE ONLY; the
 * product library never links this file).
 *
 * Eq. 2 / Eq. 3 evaluated per pixel: the caller passes the Gaussians already
 * sorted by (depth, index); for every pixel the whole list is walked front to
 * back.  Pixel (px, py) is sampled at (px + 0.5, py + 0.5).
 *
 *   power = -1/2 d^T conic d          (conic = Sigma_2D^{-1} = [[a, b], [b, c]])
 *   alpha = min(alpha_max, opacity * exp(power))
 *   alpha <  alpha_min          -> the Gaussian is skipped
 *   T * (1 - alpha) < t_min     -> the walk stops before this Gaussian
 *   otherwise C += rgb * alpha * T,  T *= (1 - alpha)
 *   output C + T * bg and T.
 *
 * Rect mode skips a Gaussian at a pixel outside its conservative pixel
 * rectangle, where alpha < alpha_min is guaranteed; it visits the same
 * contributors in the same order, so its result is identical to brute force.
 *
 * Flags (per pixel, OR-ed): 1 an alpha within rel_alpha of alpha_min,
 * 2 a transmittance test within rel_t of t_min, 4 two consecutive
 * contributors whose depths differ, but by at most rel_depth * depth (exactly
 * equal depths are ordered by index, which is not ambiguous).
 *
 * Blend weights (optional, per Gaussian, summed over pixels): alpha_i T_i of
 * every blend, the ray contribution that Eq. 4 sums over all pixels.
 *
 * Weight slack (optional, per Gaussian, summed over the flagged pixels only):
 * how far a float32 walk, which may take any of a flagged pixel's
 * near-threshold decisions the other way, can move the Gaussian's weight at
 * that pixel: its own weight there (the walk may stop before it or skip it)
 * plus the largest weight such a walk can give it (its alpha, if it may pass
 * alpha_min, times the largest transmittance in front of it: the product of
 * (1 - alpha) over the Gaussians surely above alpha_min, without any stop).
 *
 * Contributions (optional, per Gaussian, OR-ed over pixels): 1 blended at a
 * pixel whose flags were still 0 after this Gaussian's own decisions (a float32
 * renderer takes the same decisions, so it blends it too); 2 blended at some
 * pixel, or reaching alpha >= alpha_min (1 - rel_alpha) anywhere in the list of
 * a pixel that ends flagged (a float32 renderer may blend it there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t n;
    const double *u, *v, *ca, *cb, *cc, *opac, *rgb, *depth; /* rgb: n x 3 */
    const int32_t *rect;                                     /* n x 4 (x0,y0,x1,y1) or NULL */
    int32_t *contrib;                                        /* n, OR-ed contribution bits, or NULL */
    double *weight;                                          /* n, summed alpha T, or NULL */
    double *weight_slack;                                    /* n, see above, or NULL */
    double bg[3];
    double alpha_min, alpha_max, t_min;
    double rel_alpha, rel_t, rel_depth;
} oracle_scene;

static void shade_pixel(const oracle_scene *s, const int64_t *list, int64_t nlist,
                        int32_t px, int32_t py, double *out_rgb, double *out_t,
                        int32_t *out_flag)
{
    const double sx = px + 0.5, sy = py + 0.5;
    double T = 1.0, C0 = 0.0, C1 = 0.0, C2 = 0.0;
    double prev_depth = -INFINITY;
    int32_t flag = 0;
    for (int64_t k = 0; k < nlist; ++k) {
        const int64_t i = list[k];
        if (s->rect) {
            const int32_t *r = s->rect + 4 * i;
            if (px < r[0] || px > r[2] || py < r[1] || py > r[3]) continue;
        }
        const double dx = sx - s->u[i], dy = sy - s->v[i];
        const double power = -0.5 * (s->ca[i] * dx * dx + 2.0 * s->cb[i] * dx * dy + s->cc[i] * dy * dy);
        double alpha = s->opac[i] * exp(power);
        if (alpha > s->alpha_max) alpha = s->alpha_max;
        if (fabs(alpha - s->alpha_min) <= s->rel_alpha * s->alpha_min) flag |= 1;
        if (alpha < s->alpha_min) continue;
        const double test = T * (1.0 - alpha);
        if (fabs(test - s->t_min) <= s->rel_t * s->t_min) flag |= 2;
        if (test < s->t_min) break;
        {   /* equal depths are ordered by index on both sides; only near-equal ones are ambiguous */
            const double gap = s->depth[i] - prev_depth;
            if (gap > 0.0 && gap <= s->rel_depth * fabs(s->depth[i])) flag |= 4;
        }
        prev_depth = s->depth[i];
        if (s->contrib) {
            const int32_t bits = flag == 0 ? 3 : 2;
            #pragma omp atomic update
            s->contrib[i] |= bits;
        }
        const double w = alpha * T;
        if (s->weight) {
            #pragma omp atomic update
            s->weight[i] += w;
        }
        C0 += s->rgb[3 * i + 0] * w;
        C1 += s->rgb[3 * i + 1] * w;
        C2 += s->rgb[3 * i + 2] * w;
        T = test;
    }
    if (s->weight_slack && flag != 0) {
        double Tr = 1.0, Th = 1.0;
        int stopped = 0;
        for (int64_t k = 0; k < nlist; ++k) {
            const int64_t i = list[k];
            if (s->rect) {
                const int32_t *r = s->rect + 4 * i;
                if (px < r[0] || px > r[2] || py < r[1] || py > r[3]) continue;
            }
            const double dx = sx - s->u[i], dy = sy - s->v[i];
            const double power = -0.5 * (s->ca[i] * dx * dx + 2.0 * s->cb[i] * dx * dy + s->cc[i] * dy * dy);
            double alpha = s->opac[i] * exp(power);
            if (alpha > s->alpha_max) alpha = s->alpha_max;
            double w_ref = 0.0;   /* this pixel's weight in the walk above */
            if (!stopped && alpha >= s->alpha_min) {
                const double test = Tr * (1.0 - alpha);
                if (test < s->t_min) {
                    stopped = 1;
                } else {
                    w_ref = alpha * Tr;
                    Tr = test;
                }
            }
            const double w_max = alpha >= s->alpha_min * (1.0 - s->rel_alpha) ? alpha * (1.0 + s->rel_alpha) * Th : 0.0;
            if (w_ref + w_max > 0.0) {
                #pragma omp atomic update
                s->weight_slack[i] += w_ref + w_max;
            }
            if (alpha >= s->alpha_min * (1.0 + s->rel_alpha)) Th *= 1.0 - alpha * (1.0 - s->rel_alpha);
        }
    }
    if (s->contrib && flag != 0) {
        /* a flagged pixel: any Gaussian near or above alpha_min may be blended by a float32 walk */
        for (int64_t k = 0; k < nlist; ++k) {
            const int64_t i = list[k];
            if (s->rect) {
                const int32_t *r = s->rect + 4 * i;
                if (px < r[0] || px > r[2] || py < r[1] || py > r[3]) continue;
            }
            const double dx = sx - s->u[i], dy = sy - s->v[i];
            const double power = -0.5 * (s->ca[i] * dx * dx + 2.0 * s->cb[i] * dx * dy + s->cc[i] * dy * dy);
            const double alpha = s->opac[i] * exp(power);
            if (alpha >= s->alpha_min * (1.0 - s->rel_alpha)) {
                #pragma omp atomic update
                s->contrib[i] |= 2;
            }
        }
    }
    out_rgb[0] = C0 + T * s->bg[0];
    out_rgb[1] = C1 + T * s->bg[1];
    out_rgb[2] = C2 + T * s->bg[2];
    *out_t = T;
    *out_flag = flag;
}

/*
 * Shade npix pixels (px[k], py[k]).  In rect mode the pixels must be grouped
 * by row (all pixels of a row contiguous); for each row the list is first
 * narrowed to the Gaussians whose rectangle spans that row, in order.
 * Returns 0, or -1 on allocation failure.
 */
int oracle_composite(const oracle_scene *s, int64_t npix, const int32_t *px, const int32_t *py,
                     double *out_rgb, double *out_t, int32_t *out_flag)
{
    if (!s->rect) {
        int64_t *all = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
        if (!all) return -1;
        for (int64_t i = 0; i < s->n; ++i) all[i] = i;
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < npix; ++k)
            shade_pixel(s, all, s->n, px[k], py[k], out_rgb + 3 * k, out_t + k, out_flag + k);
        free(all);
        return 0;
    }
    /* row groups */
    int64_t ngroups = 0;
    int64_t *gstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npix + 1));
    if (!gstart) return -1;
    for (int64_t k = 0; k < npix; ++k)
        if (k == 0 || py[k] != py[k - 1]) gstart[ngroups++] = k;
    gstart[ngroups] = npix;
    int failed = 0;
    #pragma omp parallel
    {
        int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
        if (!list) {
            #pragma omp atomic write
            failed = 1;
        }
        #pragma omp for schedule(dynamic, 1)
        for (int64_t g = 0; g < ngroups; ++g) {
            if (!list) continue;
            const int32_t row = py[gstart[g]];
            int64_t nl = 0;
            for (int64_t i = 0; i < s->n; ++i) {
                const int32_t *r = s->rect + 4 * i;
                if (row >= r[1] && row <= r[3]) list[nl++] = i;
            }
            for (int64_t k = gstart[g]; k < gstart[g + 1]; ++k)
                shade_pixel(s, list, nl, px[k], py[k], out_rgb + 3 * k, out_t + k, out_flag + k);
        }
        free(list);
    }
    free(gstart);
    return failed ? -1 : 0;
}

int oracle_num_threads(void)
{
    int n = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
