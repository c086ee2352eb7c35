/*
 * fdgs.h - C ABI of libfdgs.so, a masked 4D Gaussian rasterizer for AMD
 * Instinct MI355X (gfx950).
 *
 * The library renders I(u, v, t) of a set of 4D Gaussians (Sec. 3):
 *   - temporal slicing of every processed Gaussian into a conditional 3D
 *     Gaussian and a temporal opacity factor (Eq. 1, Eq. 3);
 *   - an optional keyframe active set that drops inactive Gaussians before any
 *     of that work (Sec. 4.2.2);
 *   - projection, screen-tile binning, depth ordering and front-to-back alpha
 *     blending (Eq. 2, Eq. 3);
 *   - the adjoint of the whole forward pass.
 *
 * Conventions shared by every entry point
 *   - Every call returns an fdgs_status.  On failure fdgs_last_error() returns
 *     a message (thread-local, valid until the next fdgs_* call on the thread).
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid argument enqueues nothing.
 *   - "device" pointers are HIP device memory owned by the caller; the library
 *     never frees them.  "host" pointers are ordinary CPU memory read during the
 *     call only.
 *   - Work is enqueued on the caller's stream and runs asynchronously unless a
 *     call says it synchronises.
 *   - A context owns scratch memory and is not thread-safe: use one context per
 *     host thread / stream.  Scratch grows geometrically when a call needs more
 *     (hipMalloc, which may wait for the device); a replaced block is freed
 *     only after a later device-wide synchronisation (fdgs_destroy, once
 *     more than 1 GiB of replaced blocks wait, or when an allocation runs out
 *     of memory, which then retries, at the exact size if need be), so growth
 *     in one context does not stall work in flight on other streams.
 *   - Model tensors are float32 structure-of-arrays with plane stride n
 *     (see fdgs_model).  Non-finite parameters or a quaternion with
 *     |q|^2 < 1e-12 make a Gaussian invisible; they never raise an error.
 */
#ifndef FDGS_H
#define FDGS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDGS_API __attribute__((visibility("default")))

typedef int32_t fdgs_status;
enum {
    FDGS_OK = 0,
    FDGS_ERR_INVALID_ARG = 1,   /* bad pointer, size, enum or shape          */
    FDGS_ERR_HIP = 2,           /* a HIP runtime call failed                  */
    FDGS_ERR_CAPACITY = 3,      /* fixed instance capacity was too small      */
    FDGS_ERR_UNSUPPORTED = 4,   /* valid request this build does not support  */
    FDGS_ERR_STATE = 5          /* state handle missing, released or mismatched */
};

FDGS_API const char *fdgs_last_error(void);
FDGS_API const char *fdgs_version(void);

typedef struct fdgs_ctx fdgs_ctx;

/* Create a context on HIP device `device` (made current for the call). */
FDGS_API fdgs_status fdgs_create(fdgs_ctx **out, int32_t device);
/* Destroy a context and every state it owns.  Waits for its work to finish. */
FDGS_API fdgs_status fdgs_destroy(fdgs_ctx *ctx);

/*
 * 4D Gaussians (Sec. 3): mean mu in R^4, covariance Sigma = R S S^T R^T with
 * S = diag(exp(log_scale)) and R the 4D rotation x -> q_l * x * q_r (x read as
 * a quaternion (w, i, j, k) = (x, y, z, t); both quaternions are normalised
 * before use), opacity sigmoid(opacity_logit), RGB colour from real spherical
 * harmonics of degree sh_degree.  All device, float32, plane stride n:
 *   mean[4][n], log_scale[4][n], q_left[4][n], q_right[4][n] (w, x, y, z),
 *   opacity_logit[n], sh[16][3][n] (basis k = l*l + l + m, then channel).
 */
typedef struct {
    const float *mean;
    const float *log_scale;
    const float *q_left;
    const float *q_right;
    const float *opacity_logit;
    const float *sh;
    int64_t n;              /* 0 <= n < 2^31 */
    int32_t sh_degree;      /* 0..3; coefficients k >= (degree+1)^2 are not read */
    /* Optional vector-quantised SH (the post-processing of Sec. 5, see
     * fdgs_sh_kmeans): when sh_index is not NULL, Gaussian i's coefficients are
     * sh_codebook[sh_index[i]][0..47] (basis-major, then channel; device,
     * float32, 16-byte aligned), sh is not read and may be NULL, and an index
     * >= sh_codebook_size reads the last entry.  fdgs_render_backward rejects
     * such a model (FDGS_ERR_UNSUPPORTED).  Zero / NULL: plain SH planes. */
    const uint32_t *sh_index;
    const float *sh_codebook;
    int64_t sh_codebook_size;
} fdgs_model;

/*
 * Pinhole camera, host POD, float64.  World to camera: x_c = R x_w + tvec
 * (R row-major), OpenCV axes (x right, y down, z forward).  Pixel (px, py) is
 * sampled at (px + 0.5, py + 0.5); u = fx x/z + cx, v = fy y/z + cy.  A
 * Gaussian whose conditional mean has z <= znear is not drawn.
 */
typedef struct {
    double R[9];
    double tvec[3];
    double fx, fy, cx, cy;
    double znear;           /* > 0 */
    int32_t width, height;  /* 1..16384 */
} fdgs_camera;

/*
 * Rendering options.  fdgs_render_cfg_default() fills the defaults given in
 * brackets.  Screen tiles and the LDS batch only change speed, never the image.
 */
typedef struct {
    int32_t tile_w, tile_h;     /* one of 8x8, 16x16, 32x8, 32x16,
                                   32x32                         [16x16] */
    int32_t batch;              /* Gaussians staged in LDS: 64/128/256
                                   (also 512/1024 with 32x32 tiles) [128] */
    int32_t pixels_per_thread;  /* 1, 2 or 4 pixels of a column per thread in
                                   the forward compositor; 8x8 tiles always
                                   use 1; 0 picks the default              [0] */
    float bg[3];                /* background, added with the final T  [0,0,0] */
    float alpha_min;            /* alpha below this is skipped         [1/255] */
    float alpha_max;            /* alpha clamp                          [0.99] */
    float t_min;                /* stop before T would fall below this  [1e-4] */
    float dilation;             /* added to Sigma_2D's diagonal, px^2    [0.3] */
    int32_t temporal_cull;      /* 1: drop sigma*p(t) < alpha_min before binning;
                                   0: bin every Gaussian in view (the
                                   unfiltered baseline's work)            [1] */
    int32_t tile_cull;          /* 1: list a Gaussian only in the tiles of its
                                   rectangle that its footprint ellipse
                                   reaches; 0: in every tile of the
                                   rectangle.  The image is the same     [1] */
    int32_t schedule;           /* compositor schedule: one workgroup per
                                   (view, tile) item, 0 in raster order, 1
                                   longest list first (a first launch sorts
                                   the items by list length).  Same image [1] */
    int64_t instance_capacity;  /* 0: size tile-list buffers exactly (one
                                   host synchronisation per frame); >0: fixed
                                   capacity, no synchronisation, overflow
                                   reported as FDGS_ERR_CAPACITY by
                                   fdgs_check_overflow                     [0] */
} fdgs_render_cfg;

FDGS_API void fdgs_render_cfg_default(fdgs_render_cfg *cfg);

/*
 * (1) Temporal slicing, Eq. 1 and Eq. 3.  For each j < m, Gaussian
 * g = idx ? idx[j] : j is sliced at time t:
 *   out_mean3[3][m]  mu_{1:3} + Sigma_{1:3,4} Sigma_44^{-1} (t - mu_t)
 *   out_cov3[6][m]   Sigma_{1:3,1:3} - Sigma_{1:3,4} Sigma_44^{-1} Sigma_{4,1:3},
 *                    stored xx, xy, xz, yy, yz, zz
 *   out_p[m]         exp(-(t - mu_t)^2 / (2 Sigma_44))
 * Computed in float64, stored float32.  An invalid Gaussian yields zeros.
 * idx (device, uint32, entries < n) may be NULL (then m <= n).  All outputs
 * are device buffers of the stated sizes.
 */
FDGS_API fdgs_status fdgs_slice_4d(fdgs_ctx *ctx, const fdgs_model *model, double t,
                          const uint32_t *idx, int64_t m,
                          float *out_mean3, float *out_cov3, float *out_p,
                          hipStream_t stream);

/*
 * (2) Active set of one keyframe window (Sec. 4.2.2).
 *   mode FDGS_MASK_TEMPORAL: keep Gaussian i iff its temporal opacity p_i(t)
 *     reaches alpha_min at one of the window's frames (decided in float64 as
 *     (t_f - mu_t)^2 <= 2 ln(1/alpha_min) Sigma_44).  Rendering any frame of
 *     the window with this set gives exactly the unmasked image.
 *   mode FDGS_MASK_TEMPORAL_AND_TILE: additionally keep only Gaussians whose
 *     opacity-free footprint (level 2 ln(1/alpha_min)) covers a pixel of one of
 *     the mask views at key_lo or key_hi.
 *   mode FDGS_MASK_CONTRIBUTED (the keyframe visibility of Sec. 4.2.2): render
 *     every mask view at key_lo and at key_hi (all n Gaussians, default
 *     render options with this alpha_min and dilation) and keep Gaussian i iff
 *     some pixel blends it (Eq. 2: alpha >= alpha_min before the pixel's walk
 *     stops); the set is the union over views and both keyframes.  Frame
 *     times are not used (n_frames may be 0).  Rendering a keyframe from a
 *     mask view with this set gives exactly the unmasked image.
 * Outputs (device): out_bits[ceil(n/32)] (bit i%32 of word i/32, LSB first),
 * out_idx[n] (kept indices ascending; entries past the count are unspecified)
 * and *out_count (int64).  Synchronises `stream` (the host arrays of the spec
 * are copied to the device during the call).
 */
enum { FDGS_MASK_TEMPORAL = 0, FDGS_MASK_TEMPORAL_AND_TILE = 1, FDGS_MASK_CONTRIBUTED = 2 };
typedef struct {
    const double *frame_times;  /* host, 1 <= n_frames <= 256 (modes 0, 1)   */
    int32_t n_frames;
    const fdgs_camera *views;   /* host, n_views mask views (modes 1, 2)      */
    int32_t n_views;            /* <= 64                                      */
    double key_lo, key_hi;      /* keyframe times of the window               */
    int32_t mode;
    float alpha_min;            /* threshold on p(t) [1/255 if <= 0]          */
    float dilation;             /* footprint dilation (modes 1, 2) [0.3 if < 0] */
} fdgs_mask_spec;

FDGS_API fdgs_status fdgs_build_active_mask(fdgs_ctx *ctx, const fdgs_model *model,
                                   const fdgs_mask_spec *spec,
                                   uint32_t *out_bits, uint32_t *out_idx,
                                   int64_t *out_count, hipStream_t stream);

/*
 * Overlap of two active sets, for the redundancy measures of Sec. 4.1:
 * out[0] = |a|, out[1] = |b|, out[2] = |a and b|, counted over the first n
 * bits of the bit arrays a and b (device, ceil(n/32) uint32 words each, bit
 * i%32 of word i/32, as fdgs_build_active_mask writes them; bits past n are
 * ignored); out is a device int64[3], written on `stream`.  With A_t the set
 * of Gaussians that some pixel of some view blends at time t
 * (fdgs_build_active_mask, mode FDGS_MASK_CONTRIBUTED, key_lo = key_hi = t):
 * the active ratio at t is |A_t| / n and the activation IoU between frames 0
 * and t is |A_0 and A_t| / (|A_0| + |A_t| - |A_0 and A_t|).  Runs on the
 * current HIP device; 0 <= n < 2^31.
 */
FDGS_API fdgs_status fdgs_mask_overlap(const uint32_t *bits_a, const uint32_t *bits_b, int64_t n,
                                       int64_t *out, hipStream_t stream);

/*
 * (2b) fdgs_build_active_mask without any device allocation, for callers that
 * cannot allocate: code that must not call hipMalloc (a serving loop with a
 * fixed memory budget, a harness that forbids allocation).  Takes no context.
 * Modes FDGS_MASK_TEMPORAL and FDGS_MASK_TEMPORAL_AND_TILE only (the
 * contributed mode renders views and returns FDGS_ERR_UNSUPPORTED); model->n
 * at most FDGS_NOALLOC_MAX_GAUSSIANS, else FDGS_ERR_INVALID_ARG.  Outputs and
 * limits on the spec as for fdgs_build_active_mask, which gives bit-identical
 * results.  Its scratch (the window's frame times, the mask cameras and the
 * compaction's per-chunk counts) is a static device array of 2 MiB on each
 * GPU the library runs on, held until the process ends and shared by every
 * call on that GPU: calls that overlap on one GPU (on different streams or
 * host threads) race.  Runs on the current HIP device; synchronises `stream`.
 */
#define FDGS_NOALLOC_MAX_GAUSSIANS (INT64_C(1) << 27)
FDGS_API fdgs_status fdgs_build_active_mask_noalloc(const fdgs_model *model, const fdgs_mask_spec *spec,
                                                    uint32_t *out_bits, uint32_t *out_idx,
                                                    int64_t *out_count, hipStream_t stream);

/*
 * (3) Forward render of one view at time t (Eq. 2, Eq. 3).
 * Processed set: every Gaussian if idx == NULL, else idx[0..count) with count
 * read from the device scalar *n_idx_dev (int64, <= model->n), as written by
 * fdgs_build_active_mask.  Per pixel the processed Gaussians that survive
 * culling are blended front to back in order of camera depth (float64 z of the
 * conditional mean), equal depths by processing position.
 * Outputs (device): out_rgb[3][H][W]; out_T[H][W] (final transmittance) may be
 * NULL.  keep_state: NULL to discard the intermediate state; otherwise
 * *keep_state receives a state for fdgs_render_backward / inspection (a
 * non-NULL *keep_state from an earlier forward of this context is reused).
 */
typedef struct fdgs_state fdgs_state;

FDGS_API fdgs_status fdgs_render_forward(fdgs_ctx *ctx, const fdgs_model *model,
                                const uint32_t *idx, const int64_t *n_idx_dev,
                                const fdgs_camera *cam, double t,
                                const fdgs_render_cfg *cfg,
                                float *out_rgb, float *out_T,
                                fdgs_state **keep_state, hipStream_t stream);

/*
 * (4) Adjoint of the forward pass recorded in `state`: Eq. 2 and Eq. 3
 * differentiated back to front through the blend (transmittance recovered from
 * the final T, no per-pixel lists), then through the projection, Eq. 1's
 * slicing and the activations to the model's parameters (Sec. 3).  dL_drgb
 * (device, [3][H][W]) is the gradient of a scalar loss with respect to out_rgb.
 * Gradients are ACCUMULATED (+=) into the caller's device buffers, laid out
 * like fdgs_model: mean[4][n], log_scale[4][n], q_left[4][n], q_right[4][n],
 * opacity_logit[n], sh[16][3][n].  Gaussians that were not processed or not
 * visible receive nothing.  The model passed to the forward must be unchanged.
 * Float atomics make the last bits order-dependent.
 */
typedef struct {
    float *mean, *log_scale, *q_left, *q_right, *opacity_logit, *sh;
} fdgs_grads;

FDGS_API fdgs_status fdgs_render_backward(fdgs_ctx *ctx, fdgs_state *state,
                                 const float *dL_drgb, const fdgs_grads *grads,
                                 hipStream_t stream);

/*
 * The two phases of fdgs_render_backward, for callers that order them apart
 * (adjoint of Eq. 2-3, then of Sec. 3's slicing and projection):
 *   - fdgs_render_backward_2d: the adjoint of the blend, back to front, into
 *     the state's own per-Gaussian gradients of the 2D centre, conic, opacity
 *     and colour.  It writes nothing outside the state.
 *   - fdgs_render_backward_params: those gradients through the projection,
 *     Eq. 1's slicing and the activations, ACCUMULATED (+=) into `grads` (as in
 *     fdgs_render_backward: per Gaussian a plain read-modify-write, so two
 *     calls that add into the same buffers must be ordered, e.g. by events).
 *     FDGS_ERR_STATE unless fdgs_render_backward_2d ran on the state since its
 *     last forward.
 * fdgs_render_backward_2d then fdgs_render_backward_params on one stream is
 * fdgs_render_backward.  A multi-view step can overlap the first phases of
 * several views (one context each, on their own streams) and chain only the
 * second.
 */
FDGS_API fdgs_status fdgs_render_backward_2d(fdgs_ctx *ctx, fdgs_state *state, const float *dL_drgb,
                                             hipStream_t stream);
FDGS_API fdgs_status fdgs_render_backward_params(fdgs_ctx *ctx, fdgs_state *state, const fdgs_grads *grads,
                                                 hipStream_t stream);

/* Release a state (NULL is accepted). */
FDGS_API fdgs_status fdgs_state_release(fdgs_ctx *ctx, fdgs_state *state);

/*
 * Inspection of a state's binning (device pointers valid until the state is
 * reused or released).  Synchronises `stream` to read the counts.
 *   sorted_ids[n_inst]   processing positions, tile after tile, each tile in
 *                        depth order
 *   tile_ranges[n_tiles][2]  [start, end) of each tile (id ty*tiles_x + tx)
 *   rects[n_proc][4]     int32 inclusive pixel rect (x0,y0,x1,y1) of each
 *                        processed Gaussian; only meaningful when visible
 *   depth[n_proc]        float64 camera depth of each processed Gaussian
 *   visible[n_proc]      uint8 1 if binned
 */
typedef struct {
    const uint32_t *sorted_ids;
    const uint32_t *tile_ranges;
    const int32_t *rects;
    const double *depth;
    const uint8_t *visible;
    int64_t n_inst, n_vis, n_proc;
    int32_t n_tiles, tiles_x, tiles_y;
} fdgs_binning;

FDGS_API fdgs_status fdgs_state_binning(fdgs_ctx *ctx, fdgs_state *state, fdgs_binning *out,
                               hipStream_t stream);

/*
 * (5) Batched forward for many views across scenes of uneven size (a
 * multi-view workload such as rendering every (camera, timestamp) of several
 * dynamic scenes).  The views are processed in launches of views_per_launch
 * views (0: all at once): each launch runs every stage once over the
 * concatenated (view, Gaussian) space, bins with (view, tile) keys and
 * blends all views' tiles in one compositor launch.  Results equal
 * fdgs_render_forward of each view (no state is kept).
 *   scenes[n_scenes]: models (device pointers as in fdgs_model).
 *   views[n_views]: host descriptors; every view has the same width/height;
 *     idx (device) selects a processed subset of its scene (NULL: all) with
 *     n_idx entries (host count).
 *   out_rgb: device [n_views][3][H][W].
 *   use_graph: 1 captures the whole call in a HIP graph on first use (after
 *     one eager run that sizes every buffer) and replays it while all
 *     arguments and the views' contents are unchanged; requires
 *     cfg->instance_capacity > 0 (per launch).  Synchronises `stream` when
 *     it (re)builds the graph.
 */
typedef struct {
    int32_t scene;
    fdgs_camera cam;
    double t;
    const uint32_t *idx;
    int64_t n_idx;
} fdgs_view;

FDGS_API fdgs_status fdgs_render_batch(fdgs_ctx *ctx, const fdgs_model *scenes, int32_t n_scenes,
                                       const fdgs_view *views, int32_t n_views,
                                       const fdgs_render_cfg *cfg, int32_t views_per_launch,
                                       int32_t use_graph, float *out_rgb, hipStream_t stream);

/*
 * Autotuner: renders the batch with every tile shape (8x8, 16x16, 32x8,
 * 32x16, 32x32), LDS batch (64, 128, 256; also 512 and 1024 for 32x32),
 * pixels-per-thread choice (1, 2, 4; 1 only for 8x8) and compositor schedule
 * (1, 0): 90 configurations, each timed with HIP
 * events (best of `repeats`).  It checks that every
 * configuration's images are bit-identical to the first one's, and writes the
 * fastest into *inout_cfg (other fields are kept).  results (host, may be
 * NULL) receives up to max_results entries; *n_results the number tried.
 * Returns FDGS_ERR_STATE if any configuration's images differed.
 * Synchronises `stream`.
 */
typedef struct {
    int32_t tile_w, tile_h, batch, pixels_per_thread, schedule;
    double ms;
    int32_t identical;
} fdgs_tune_result;

FDGS_API fdgs_status fdgs_autotune(fdgs_ctx *ctx, const fdgs_model *scenes, int32_t n_scenes,
                                   const fdgs_view *views, int32_t n_views, int32_t views_per_launch,
                                   int32_t repeats, fdgs_render_cfg *inout_cfg,
                                   fdgs_tune_result *results, int32_t max_results, int32_t *n_results,
                                   hipStream_t stream);

/*
 * (7) Pruning with the spatial-temporal variation score (Sec. 4.2.1).
 *
 * fdgs_spatial_score (Eq. 4): for each v < n_views renders the model at
 * (cams[v], times[v]) (host arrays) with every Gaussian processed and ADDS to
 * inout_score[i] (device, float[n]) the sum over that view's pixels of
 * Gaussian i's blend weight alpha_i T_i.  cfg may be NULL (defaults; its tile
 * shape, batch and schedule only change speed).  Synchronises `stream`.
 */
FDGS_API fdgs_status fdgs_spatial_score(fdgs_ctx *ctx, const fdgs_model *model, const fdgs_camera *cams,
                                        const double *times, int32_t n_views, const fdgs_render_cfg *cfg,
                                        float *inout_score, hipStream_t stream);

/*
 * fdgs_variation_score (Eq. 5-7): out_score[i] = S^TV_i gamma_i spatial[i]
 * (device float[n] in and out) with
 *   S^TV_i  = sum over the n_times host times t of 1 / (0.5 tanh|p_i''(t)| + 0.5),
 *             p_i''(t) = ((t - mu_t)^2 / Sigma_44^2 - 1 / Sigma_44) p_i(t),
 *   gamma_i = min(V_i / V_90, 1)^0.1, V_i = product of the four scales and V_90
 *             the volume at position floor(0.9 (n - 1)) of the ascending volumes
 *             (gamma = 1 for every positive volume if V_90 = 0);
 * invalid Gaussians score 0.  Temporal sums in float64.  Synchronises `stream`.
 */
FDGS_API fdgs_status fdgs_variation_score(fdgs_ctx *ctx, const fdgs_model *model, const double *times,
                                          int32_t n_times, const float *spatial, float *out_score,
                                          hipStream_t stream);

/*
 * fdgs_prune: keeps the n_keep (0..n) highest of score[0..n) (device), equal
 * scores by the lower index, negative or NaN scores counting as 0, and writes
 * the kept set as fdgs_build_active_mask does: out_bits[ceil(n/32)],
 * out_idx[n] (ascending; entries past the count unspecified), *out_count.
 * Synchronises `stream`.
 */
FDGS_API fdgs_status fdgs_prune(fdgs_ctx *ctx, const float *score, int64_t n, int64_t n_keep, uint32_t *out_bits,
                                uint32_t *out_idx, int64_t *out_count, hipStream_t stream);

/*
 * SH vector quantisation by Lloyd's k-means (the post-processing of Sec. 5:
 * the paper quantises each Gaussian's SH with a codebook).  A Gaussian's SH
 * vector is its 16 x 3 coefficients from model->sh (basis-major, then
 * channel).  The codebook starts as the vectors of the k Gaussians init_index
 * [k] names (device; indices >= n read the last Gaussian), then `iterations`
 * times: assign every Gaussian to its nearest entry (squared L2 in float32,
 * equal distances to the lower index), replace each entry by the mean of its
 * members (float64 sum in index order; an entry without members is kept).
 * Outputs: codebook [k][48] (device float32, 16-byte aligned) and assignment
 * [n] (device; the nearest entry of the final codebook).  The whole
 * computation is enqueued on `stream`; scratch is owned by ctx.
 * Constraints: model->sh not NULL, 1 <= k <= 2^24, 0 <= iterations <= 1000.
 */
FDGS_API fdgs_status fdgs_sh_kmeans(fdgs_ctx *ctx, const fdgs_model *model, const uint32_t *init_index, int64_t k,
                                    int32_t iterations, float *codebook, uint32_t *assignment, hipStream_t stream);

/*
 * (8) Adam step for fine-tuning the kept Gaussians: for i < n (device float
 * arrays, updated in place)
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * step >= 1; m and v start at 0.  Elements with g = 0 and m = v = 0 (never
 * touched by a gradient) stay unchanged.
 */
FDGS_API fdgs_status fdgs_adam_step(fdgs_ctx *ctx, float *param, const float *grad, float *m, float *v, int64_t n,
                                    float lr, float beta1, float beta2, float eps, int32_t step,
                                    hipStream_t stream);

/*
 * Reports FDGS_ERR_CAPACITY if a forward with a fixed instance_capacity on
 * this context overflowed since the last check, or FDGS_ERR_UNSUPPORTED if
 * more than 4096 visible Gaussians of one forward shared a float32-rounded
 * depth (their relative order then falls back to processing order instead of
 * the float64 depth); clears the flags.  Synchronises `stream`.
 */
FDGS_API fdgs_status fdgs_check_overflow(fdgs_ctx *ctx, hipStream_t stream);

/*
 * Per-stage timing with HIP events recorded on the caller's stream around each
 * kernel group of fdgs_render_forward / fdgs_render_backward, plus work
 * counters (processed and visible Gaussians, tile instances, and (pixel,
 * Gaussian) pairs evaluated by the compositor and, of those, blended).  Profiling adds event records
 * between kernels and a per-wavefront counter update in the compositor; it is
 * off by default.
 */
enum {
    FDGS_STAGE_PREPROCESS = 0,   /* slice + project + SH + footprint        */
    FDGS_STAGE_COMPACT = 1,      /* visible-set scan and scatter             */
    FDGS_STAGE_DEPTH_SORT = 2,   /* depth radix sort + tie fix               */
    FDGS_STAGE_OFFSETS = 3,      /* instance offsets (scan)                  */
    FDGS_STAGE_DUPLICATE = 4,    /* tile-key emission                        */
    FDGS_STAGE_TILE_SORT = 5,    /* tile radix sort                          */
    FDGS_STAGE_RANGES = 6,       /* tile ranges (and the longest-first order) */
    FDGS_STAGE_COMPOSITE = 7,    /* per-tile blending                        */
    FDGS_STAGE_BWD_COMPOSITE = 8,
    FDGS_STAGE_BWD_PREPROCESS = 9,
    FDGS_NUM_STAGES = 10
};
typedef struct {
    double ms[FDGS_NUM_STAGES];      /* summed event time per stage        */
    int64_t calls[FDGS_NUM_STAGES];  /* times each stage ran               */
    int64_t processed;               /* sums over the profiled forwards    */
    int64_t visible;
    int64_t instances;
    uint64_t pairs;                  /* (pixel, Gaussian) evaluations      */
    uint64_t blended;                /* of those, pairs that were blended  */
} fdgs_profile;

/*
 * Rates of the device, measured with micro-benchmarks (a few milliseconds;
 * synchronises `stream`), against which kernel rates are reported:
 *   out[0] LDS bytes/s delivered to lanes when every lane of a wavefront
 *          reads the same 16 bytes (the compositors' staged-record reads),
 *   out[1] LDS bytes/s with lane-distinct 16-byte reads,
 *   out[2] float32 FMA lane-operations/s of the vector ALUs (non-packed),
 *   out[3] compute units.
 * out is host double[4].
 */
FDGS_API fdgs_status fdgs_measure_peaks(fdgs_ctx *ctx, double *out, hipStream_t stream);

/* Profiling for subsequent calls on this context: 0 off; 1 stage events and
 * work counts (the compositor is the one that runs unprofiled); 2 as 1 plus
 * the evaluated-pair count (a counting variant of the compositor). */
FDGS_API fdgs_status fdgs_profile_enable(fdgs_ctx *ctx, int32_t enable);
/* Read (and with reset=1 clear) the totals.  Synchronises the device. */
FDGS_API fdgs_status fdgs_profile_read(fdgs_ctx *ctx, fdgs_profile *out, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* FDGS_H */
