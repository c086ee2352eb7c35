// C ABI of libfdgs: argument validation, scratch management and the order in
// which the kernels of one render are enqueued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fdgs_internal.h"

using namespace fdgs;

namespace {

thread_local std::string g_err;

constexpr int kMaskMaxFrames = 256;   // frame times of one keyframe window
constexpr int kMaskMaxViews = 64;     // mask cameras

fdgs_status fail(fdgs_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FDGS_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// Blocks replaced by a larger one.  Kernels enqueued before the growth (on
// whatever stream the caller gave) may still read the old block, so it is not
// freed at once: it waits here until a device-wide synchronisation that
// starts after its retirement -- fdgs_destroy, a growth that finds more than
// kRetiredLimit bytes waiting, or an allocation that runs out of memory -- so
// that a growth does not stall every stream of the process.  Growth is geometric (1.5x), so a buffer retires a
// few blocks at most.
std::mutex g_retired_mu;
std::vector<std::pair<int, void *>> g_retired;   // (device, block)
size_t g_retired_bytes = 0;
constexpr size_t kRetiredLimit = size_t(1) << 30;

hipError_t free_retired() {
    std::vector<std::pair<int, void *>> mine;
    {
        std::lock_guard<std::mutex> lk(g_retired_mu);
        mine.swap(g_retired);
        g_retired_bytes = 0;
    }
    if (mine.empty()) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    // every block taken here was retired before this synchronisation started
    std::vector<int> devs;
    for (const auto &r : mine)
        if (std::find(devs.begin(), devs.end(), r.first) == devs.end()) devs.push_back(r.first);
    for (int d : devs) {
        const hipError_t f = hipSetDevice(d) == hipSuccess ? hipDeviceSynchronize() : hipErrorInvalidDevice;
        if (e == hipSuccess) e = f;
    }
    for (const auto &r : mine) {
        (void)hipSetDevice(r.first);
        const hipError_t f = hipFree(r.second);
        if (e == hipSuccess) e = f;
    }
    (void)hipSetDevice(cur);
    return e;
}

hipError_t ensure(Buf &b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (bytes <= b.cap) return hipSuccess;
    const size_t want = std::max(bytes, b.cap + b.cap / 2);
    if (b.p) {
        bool flush = false;
        int dev = 0;
        const hipError_t de = hipGetDevice(&dev);
        if (de != hipSuccess) return de;
        {
            std::lock_guard<std::mutex> lk(g_retired_mu);
            g_retired.emplace_back(dev, b.p);
            g_retired_bytes += b.cap;
            flush = g_retired_bytes > kRetiredLimit;
        }
        b.p = nullptr;
        b.cap = 0;
        if (flush) {
            const hipError_t e = free_retired();
            if (e != hipSuccess) return e;
        }
    }
    size_t got = want;
    hipError_t e = hipMalloc(&b.p, got);
    if (e == hipErrorOutOfMemory) {
        // out of memory: free the retired blocks (a device synchronisation), then
        // try again, at the exact size if the geometric one still does not fit
        (void)hipGetLastError();
        bool waiting = false;
        {
            std::lock_guard<std::mutex> lk(g_retired_mu);
            waiting = !g_retired.empty();
        }
        e = waiting ? free_retired() : hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipMalloc(&b.p, got);
        if (e == hipErrorOutOfMemory && want > bytes) {
            (void)hipGetLastError();
            got = bytes;
            e = hipMalloc(&b.p, got);
        }
    }
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.cap = got;
    return hipSuccess;
}

void release(Buf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

constexpr int32_t kDefaultPpt = 2;
constexpr int64_t kBucketMaxN = int64_t(1) << 20;   // largest processed count ordered by buckets

bool valid_tile(int w, int h) {
    return (w == 8 && h == 8) || (w == 16 && h == 16) || (w == 32 && (h == 8 || h == 16 || h == 32));
}

int bits_for(int64_t v) {   // bits needed to represent values in [0, v)
    int b = 0;
    while (b < 63 && (int64_t(1) << b) < v) ++b;
    return b;
}

}  // namespace

struct fdgs_state {
    fdgs_ctx *owner = nullptr;
    bool has_forward = false;
    bool has_g2d = false;   // a backward's first phase ran since the last forward
    bool ordered = false;   // sched holds the last forward's tiles longest list first
    // per processed Gaussian
    Buf rec, depth_key, rect, tiles, visible, vis_pos, order_k, order_v, order_k2, order_v2, offsets, view_of;
    Buf bucket;        // depth buckets: counts, cursors, starts, key range
    Buf vis_count;     // visible entries per preprocess workgroup
    // per instance
    Buf tkeys, tids, tkeys2, tids2;
    // per tile / pixel
    Buf ranges, T_final, n_contrib;
    Buf sched;         // uint32[V x tiles]: the compositor's longest-first item order
    Buf counts;        // int64[4]: n_vis, n_inst
    Buf g2d;
    Buf scratch;
    // what the forward used
    fdgs_model model{};
    const uint32_t *idx = nullptr;
    const int64_t *n_idx_dev = nullptr;
    KCam cam{};
    double t = 0.0;
    RenderParams rp{};
    int32_t batch = 128;
    int32_t ppt = 2;   // pixels per thread of the forward (the adjoint takes 4 when it did, else 2)
    int64_t n_max = 0;
    int64_t capacity = 0;
    uint32_t *sorted_ids = nullptr;   // points into tids or tids2
    uint32_t *vis_list = nullptr;     // visible positions in ascending order (vis_pos), for the adjoint
    uint32_t *sorted_keys = nullptr;
    int32_t W = 0, H = 0;

    void free_all() {
        for (Buf *b : {&rec, &depth_key, &rect, &tiles, &visible, &vis_pos, &order_k, &order_v, &order_k2,
                       &order_v2, &offsets, &view_of, &bucket, &vis_count, &tkeys, &tids, &tkeys2, &tids2, &ranges, &sched,
                       &T_final, &n_contrib, &counts, &g2d, &scratch})
            release(*b);
    }
};

struct PendingStage {
    int stage;
    hipEvent_t e0, e1;
};

struct fdgs_ctx {
    int32_t device = 0;
    fdgs_state scratch_state;
    std::vector<fdgs_state *> states;
    Buf overflow;                  // int32 device flag
    Buf mask_frames, mask_views, mask_scratch;
    Buf mask_flags, mask_img;      // contributed-mode visibility bytes and the keyframe image
    Buf prune_a, prune_b, prune_c, prune_d, prune_e, prune_times;   // score / prune work
    Buf vq_scratch;                // k-means keys, values, cluster ranges, radix scratch
    int64_t *host_counts = nullptr;  // pinned
    // profiling
    int prof = 0;                  // 0 off, 1 stage events and counts, 2 also evaluated pairs
    Buf prof_acc;                  // uint64[5]: processed, visible, instances, pairs, blended pairs
    std::vector<hipEvent_t> free_events;
    std::vector<PendingStage> pending;
    double ms[FDGS_NUM_STAGES] = {};
    int64_t calls[FDGS_NUM_STAGES] = {};
    bool capturing = false;        // inside hipStreamBeginCapture / EndCapture
    // batched rendering
    fdgs_state batch_state;
    std::vector<Buf> batch_tables;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;   // graphs are captured here (the caller's may be the null stream)
    std::vector<unsigned char> graph_key;
    Buf tune_ref, tune_img, tune_diff;
    Buf probe_sink;                // fdgs_measure_peaks

    hipEvent_t get_event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {

// Records HIP events around one stage when profiling is on.
struct StageTimer {
    fdgs_ctx *c;
    int stage;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    StageTimer(fdgs_ctx *c_, int stage_, hipStream_t s_) : c(c_), stage(stage_), s(s_) {
        if (c->prof && !c->capturing && (e0 = c->get_event())) (void)hipEventRecord(e0, s);
    }
    ~StageTimer() {
        if (!c->prof || c->capturing || !e0) return;
        hipEvent_t e1 = c->get_event();
        if (!e1) return;
        (void)hipEventRecord(e1, s);
        c->pending.push_back(PendingStage{stage, e0, e1});
    }
};

}  // namespace

extern "C" {

const char *fdgs_last_error(void) { return g_err.c_str(); }

const char *fdgs_version(void) { return "fdgs 0.1 (gfx950)"; }

void fdgs_render_cfg_default(fdgs_render_cfg *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->tile_w = 16;
    cfg->tile_h = 16;
    cfg->batch = 128;
    cfg->alpha_min = 1.0f / 255.0f;
    cfg->alpha_max = 0.99f;
    cfg->t_min = 1e-4f;
    cfg->dilation = 0.3f;
    cfg->temporal_cull = 1;
    cfg->tile_cull = 1;
    cfg->schedule = 1;
    cfg->instance_capacity = 0;
}

fdgs_status fdgs_create(fdgs_ctx **out, int32_t device) {
    if (!out) return fail(FDGS_ERR_INVALID_ARG, "fdgs_create: out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(FDGS_ERR_INVALID_ARG, "fdgs_create: device %d not in [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    fdgs_ctx *c = new (std::nothrow) fdgs_ctx();
    if (!c) return fail(FDGS_ERR_HIP, "fdgs_create: out of host memory");
    c->device = device;
    c->scratch_state.owner = c;
    c->batch_state.owner = c;
    hipError_t e = ensure(c->overflow, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(c->overflow.p, 0, sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->host_counts, 4 * sizeof(int64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        release(c->overflow);
        delete c;
        return fail(FDGS_ERR_HIP, "fdgs_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return FDGS_OK;
}

fdgs_status fdgs_destroy(fdgs_ctx *ctx) {
    if (!ctx) return FDGS_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    (void)free_retired();
    for (fdgs_state *s : ctx->states) {
        s->free_all();
        delete s;
    }
    ctx->scratch_state.free_all();
    ctx->batch_state.free_all();
    for (Buf &b : ctx->batch_tables) release(b);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    release(ctx->tune_ref);
    release(ctx->tune_img);
    release(ctx->tune_diff);
    release(ctx->overflow);
    release(ctx->mask_frames);
    release(ctx->mask_views);
    release(ctx->mask_scratch);
    release(ctx->mask_flags);
    release(ctx->mask_img);
    release(ctx->probe_sink);
    for (Buf *b : {&ctx->prune_a, &ctx->prune_b, &ctx->prune_c, &ctx->prune_d, &ctx->prune_e, &ctx->prune_times,
                   &ctx->vq_scratch})
        release(*b);
    release(ctx->prof_acc);
    for (auto &p : ctx->pending) {
        (void)hipEventDestroy(p.e0);
        (void)hipEventDestroy(p.e1);
    }
    for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->host_counts) (void)hipHostFree(ctx->host_counts);
    delete ctx;
    return FDGS_OK;
}

}  // extern "C"

namespace {

fdgs_status check_model(const fdgs_model *m, const char *fn) {
    if (!m) return fail(FDGS_ERR_INVALID_ARG, "%s: model is NULL", fn);
    if (m->n < 0 || m->n >= (int64_t(1) << 31))
        return fail(FDGS_ERR_INVALID_ARG, "%s: model n=%lld out of range", fn, (long long)m->n);
    if (m->sh_degree < 0 || m->sh_degree > 3)
        return fail(FDGS_ERR_INVALID_ARG, "%s: sh_degree %d not in 0..3", fn, m->sh_degree);
    if (m->n > 0 && (!m->mean || !m->log_scale || !m->q_left || !m->q_right || !m->opacity_logit ||
                     (!m->sh && !m->sh_index)))
        return fail(FDGS_ERR_INVALID_ARG, "%s: a model pointer is NULL", fn);
    if (m->sh_index) {
        if (!m->sh_codebook || m->sh_codebook_size < 1)
            return fail(FDGS_ERR_INVALID_ARG, "%s: sh_index needs sh_codebook and sh_codebook_size >= 1", fn);
        if (reinterpret_cast<uintptr_t>(m->sh_codebook) % 16 != 0)
            return fail(FDGS_ERR_INVALID_ARG, "%s: sh_codebook must be 16-byte aligned", fn);
    }
    return FDGS_OK;
}

fdgs_status check_camera(const fdgs_camera *c, const char *fn) {
    if (!c) return fail(FDGS_ERR_INVALID_ARG, "%s: camera is NULL", fn);
    if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
        return fail(FDGS_ERR_INVALID_ARG, "%s: image %dx%d out of range", fn, c->width, c->height);
    if (!(c->znear > 0.0) || !std::isfinite(c->znear))
        return fail(FDGS_ERR_INVALID_ARG, "%s: znear must be > 0", fn);
    const double v[] = {c->fx, c->fy, c->cx, c->cy};
    for (double x : v)
        if (!std::isfinite(x)) return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite intrinsics", fn);
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(c->R[k])) return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite R", fn);
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->tvec[k])) return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite tvec", fn);
    if (!(c->fx > 0.0) || !(c->fy > 0.0)) return fail(FDGS_ERR_INVALID_ARG, "%s: focal must be > 0", fn);
    return FDGS_OK;
}

fdgs_status check_cfg(const fdgs_render_cfg *cfg, const char *fn) {
    if (!cfg) return fail(FDGS_ERR_INVALID_ARG, "%s: cfg is NULL", fn);
    if (!valid_tile(cfg->tile_w, cfg->tile_h))
        return fail(FDGS_ERR_INVALID_ARG, "%s: tile %dx%d not one of 8x8, 16x16, 32x8, 32x16, 32x32", fn, cfg->tile_w,
                    cfg->tile_h);
    if (cfg->batch != 64 && cfg->batch != 128 && cfg->batch != 256 &&
        !((cfg->batch == 512 || cfg->batch == 1024) && cfg->tile_w == 32 && cfg->tile_h == 32))
        return fail(FDGS_ERR_INVALID_ARG, "%s: batch %d not one of 64, 128, 256 (or 512 with 32x32 tiles)", fn,
                    cfg->batch);
    if (cfg->schedule != 0 && cfg->schedule != 1)
        return fail(FDGS_ERR_INVALID_ARG, "%s: schedule %d not one of 0, 1", fn, cfg->schedule);
    if (cfg->pixels_per_thread != 0 && cfg->pixels_per_thread != 1 && cfg->pixels_per_thread != 2 &&
        cfg->pixels_per_thread != 4)
        return fail(FDGS_ERR_INVALID_ARG, "%s: pixels_per_thread %d not one of 0, 1, 2, 4", fn,
                    cfg->pixels_per_thread);
    if (!(cfg->alpha_min > 0.0f) || !(cfg->alpha_max > cfg->alpha_min) || !(cfg->alpha_max < 1.0f))
        return fail(FDGS_ERR_INVALID_ARG, "%s: need 0 < alpha_min < alpha_max < 1", fn);
    if (!(cfg->t_min > 0.0f) || !(cfg->t_min < 1.0f))
        return fail(FDGS_ERR_INVALID_ARG, "%s: need 0 < t_min < 1", fn);
    if (!(cfg->dilation >= 0.0f) || !std::isfinite(cfg->dilation))
        return fail(FDGS_ERR_INVALID_ARG, "%s: dilation must be finite and >= 0", fn);
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(cfg->bg[k])) return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite bg", fn);
    if (cfg->instance_capacity < 0 || cfg->instance_capacity > 0xffffffffll)
        return fail(FDGS_ERR_INVALID_ARG, "%s: instance_capacity out of range", fn);
    return FDGS_OK;
}

KModel kmodel(const fdgs_model *m) {
    return KModel{m->mean,  m->log_scale, m->q_left,   m->q_right,     m->opacity_logit,
                  m->sh,    m->n,         m->sh_degree, m->sh_index,   m->sh_codebook,
                  m->sh_index ? m->sh_codebook_size : 0};
}

KCam kcam(const fdgs_camera *c) {
    KCam k;
    std::memcpy(k.R, c->R, sizeof k.R);
    std::memcpy(k.t, c->tvec, sizeof k.t);
    k.fx = c->fx;
    k.fy = c->fy;
    k.cx = c->cx;
    k.cy = c->cy;
    k.znear = c->znear;
    k.W = c->width;
    k.H = c->height;
    return k;
}

fdgs_state *find_state(fdgs_ctx *ctx, fdgs_state *s) {
    for (fdgs_state *x : ctx->states)
        if (x == s) return x;
    return nullptr;
}

fdgs_status run_forward(fdgs_ctx *ctx, fdgs_state *S, const ViewDesc *one, const ViewDesc *table, int32_t V,
                        const int64_t *n_dev, int64_t n_total, int32_t W, int32_t H, const fdgs_render_cfg *cfg,
                        float *out_rgb, float *out_T, bool need_state, hipStream_t stream,
                        uint8_t *contrib = nullptr, float *weight = nullptr);

}  // namespace

extern "C" {

fdgs_status fdgs_slice_4d(fdgs_ctx *ctx, const fdgs_model *model, double t, const uint32_t *idx, int64_t m,
                          float *out_mean3, float *out_cov3, float *out_p, hipStream_t stream) {
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: ctx is NULL");
    if (fdgs_status st = check_model(model, "fdgs_slice_4d")) return st;
    if (!std::isfinite(t)) return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: t is not finite");
    if (m < 0 || m >= (int64_t(1) << 31)) return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: m out of range");
    if (!idx && m > model->n) return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: m > n without idx");
    if (m > 0 && (!out_mean3 || !out_cov3 || !out_p))
        return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: an output pointer is NULL");
    if (m > 0 && idx && model->n == 0) return fail(FDGS_ERR_INVALID_ARG, "fdgs_slice_4d: idx into empty model");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_slice(kmodel(model), t, idx, m, out_mean3, out_cov3, out_p, stream));
    return FDGS_OK;
}

}  // extern "C"

namespace {

// Validation shared by the mask entry points; fills the effective alpha_min
// and dilation.
fdgs_status check_mask_args(const fdgs_model *model, const fdgs_mask_spec *spec, const uint32_t *out_bits,
                            const uint32_t *out_idx, const int64_t *out_count, float *amin_out, float *dil_out,
                            const char *fn) {
    if (fdgs_status st = check_model(model, fn)) return st;
    if (!spec) return fail(FDGS_ERR_INVALID_ARG, "%s: spec is NULL", fn);
    if (spec->mode != FDGS_MASK_TEMPORAL && spec->mode != FDGS_MASK_TEMPORAL_AND_TILE &&
        spec->mode != FDGS_MASK_CONTRIBUTED)
        return fail(FDGS_ERR_INVALID_ARG, "%s: unknown mode %d", fn, spec->mode);
    if (spec->mode != FDGS_MASK_CONTRIBUTED) {
        if (spec->n_frames < 1 || spec->n_frames > kMaskMaxFrames || !spec->frame_times)
            return fail(FDGS_ERR_INVALID_ARG, "%s: need 1..%d frame times", fn, kMaskMaxFrames);
        for (int f = 0; f < spec->n_frames; ++f)
            if (!std::isfinite(spec->frame_times[f]))
                return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite frame time", fn);
    }
    if (spec->mode != FDGS_MASK_TEMPORAL) {
        if (spec->n_views < 1 || spec->n_views > kMaskMaxViews || !spec->views)
            return fail(FDGS_ERR_INVALID_ARG, "%s: modes 1 and 2 need 1..%d views", fn, kMaskMaxViews);
        for (int v = 0; v < spec->n_views; ++v)
            if (fdgs_status st = check_camera(&spec->views[v], fn)) return st;
        if (!std::isfinite(spec->key_lo) || !std::isfinite(spec->key_hi))
            return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite keyframe time", fn);
    }
    if (!out_bits || !out_idx || !out_count) return fail(FDGS_ERR_INVALID_ARG, "%s: an output is NULL", fn);
    const float amin = spec->alpha_min > 0.0f ? spec->alpha_min : 1.0f / 255.0f;
    if (!(amin < 1.0f)) return fail(FDGS_ERR_INVALID_ARG, "%s: alpha_min must be < 1", fn);
    *amin_out = amin;
    *dil_out = spec->dilation >= 0.0f ? spec->dilation : 0.3f;
    return FDGS_OK;
}

// Modes TEMPORAL and TEMPORAL_AND_TILE: copies the window's frame times and
// mask cameras into frames_dev / views_dev (device, room for the spec's
// counts), runs the predicate and compacts the bits with compact_scratch
// (compact_scratch_bytes(n)); synchronises the stream, since the host arrays
// are copied asynchronously.
fdgs_status enqueue_window_mask(const fdgs_model *model, const fdgs_mask_spec *spec, float amin, float dil,
                                double *frames_dev, KCam *views_dev, void *compact_scratch, uint32_t *out_bits,
                                uint32_t *out_idx, int64_t *out_count, hipStream_t stream) {
    HIP_TRY(hipMemcpyAsync(frames_dev, spec->frame_times, sizeof(double) * spec->n_frames, hipMemcpyHostToDevice,
                           stream));
    KCam views[kMaskMaxViews];
    const int32_t n_views = spec->mode == FDGS_MASK_TEMPORAL_AND_TILE ? spec->n_views : 0;
    for (int v = 0; v < n_views; ++v) views[v] = kcam(&spec->views[v]);
    if (n_views > 0)
        HIP_TRY(hipMemcpyAsync(views_dev, views, sizeof(KCam) * n_views, hipMemcpyHostToDevice, stream));
    MaskArgs a;
    a.frames = frames_dev;
    a.n_frames = spec->n_frames;
    a.views = views_dev;
    a.n_views = n_views;
    a.key_lo = spec->key_lo;
    a.key_hi = spec->key_hi;
    a.mode = spec->mode;
    a.level = 2.0 * std::log(1.0 / (double)amin);
    a.rect_level = a.level * (1.0 + 1e-4) + 1e-4;
    a.dilation = dil;
    HIP_TRY(launch_mask_bits(kmodel(model), a, out_bits, stream));
    HIP_TRY(compact_bits(out_bits, model->n, out_idx, out_count, compact_scratch, stream));
    // the host arrays were copied asynchronously: finish before returning
    HIP_TRY(hipStreamSynchronize(stream));
    return FDGS_OK;
}

}  // namespace

extern "C" {

fdgs_status fdgs_build_active_mask(fdgs_ctx *ctx, const fdgs_model *model, const fdgs_mask_spec *spec,
                                   uint32_t *out_bits, uint32_t *out_idx, int64_t *out_count,
                                   hipStream_t stream) {
    const char *fn = "fdgs_build_active_mask";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    float amin = 0.0f, dil = 0.0f;
    if (fdgs_status st = check_mask_args(model, spec, out_bits, out_idx, out_count, &amin, &dil, fn)) return st;
    HIP_TRY(hipSetDevice(ctx->device));
    const int64_t n = model->n;
    if (spec->mode == FDGS_MASK_CONTRIBUTED) {
        // the union over views and both keyframes of the Gaussians some pixel blends
        fdgs_render_cfg cfg;
        fdgs_render_cfg_default(&cfg);
        cfg.alpha_min = amin;
        cfg.dilation = dil;
        cfg.pixels_per_thread = 2;
        int64_t px_max = 1;
        for (int v = 0; v < spec->n_views; ++v)
            px_max = std::max<int64_t>(px_max, (int64_t)spec->views[v].width * spec->views[v].height);
        HIP_TRY(ensure(ctx->mask_flags, (size_t)((n + 3) / 4) * 4 + 4));
        HIP_TRY(ensure(ctx->mask_img, sizeof(float) * 3 * (size_t)px_max));
        HIP_TRY(launch_fill_u32(ctx->mask_flags.as<uint32_t>(), (n + 3) / 4, 0u, stream));
        const double keys[2] = {spec->key_lo, spec->key_hi};
        for (int k = 0; k < (spec->key_hi == spec->key_lo ? 1 : 2); ++k) {
            for (int v = 0; v < spec->n_views; ++v) {
                ViewDesc one;
                one.m = kmodel(model);
                one.cam = kcam(&spec->views[v]);
                one.t = keys[k];
                one.idx = nullptr;
                one.p_off = 0;
                one.n_proc = n;
                if (fdgs_status st = run_forward(ctx, &ctx->scratch_state, &one, nullptr, 1, nullptr, n,
                                                 spec->views[v].width, spec->views[v].height, &cfg,
                                                 ctx->mask_img.as<float>(), nullptr, false, stream,
                                                 ctx->mask_flags.as<uint8_t>()))
                    return st;
            }
        }
        HIP_TRY(launch_flags_to_bits(ctx->mask_flags.as<uint8_t>(), n, out_bits, stream));
        HIP_TRY(ensure(ctx->mask_scratch, compact_scratch_bytes(n)));
        HIP_TRY(compact_bits(out_bits, n, out_idx, out_count, ctx->mask_scratch.p, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return FDGS_OK;
    }
    HIP_TRY(ensure(ctx->mask_frames, sizeof(double) * spec->n_frames));
    if (spec->mode == FDGS_MASK_TEMPORAL_AND_TILE) HIP_TRY(ensure(ctx->mask_views, sizeof(KCam) * spec->n_views));
    HIP_TRY(ensure(ctx->mask_scratch, compact_scratch_bytes(n)));
    return enqueue_window_mask(model, spec, amin, dil, ctx->mask_frames.as<double>(), ctx->mask_views.as<KCam>(),
                               ctx->mask_scratch.p, out_bits, out_idx, out_count, stream);
}

}  // extern "C"

namespace {

// Scratch of fdgs_build_active_mask_noalloc: one array per GPU, held until the
// process ends.  Host code never passes `scratch` itself (in host code the
// name is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device.
//   [0, 2 KiB)        frame times (double[256])
//   [2 KiB, 12 KiB)   mask cameras (KCam[64], 144 B each)
//   [12 KiB, 2 MiB)   per-chunk counts of the compaction (compact_scratch_bytes(n): 8 B per
//                     1024 Gaussians, 1 MiB at the maximum of 2^27)
constexpr size_t kNoAllocFrames = 0;
constexpr size_t kNoAllocViews = 2048;
constexpr size_t kNoAllocCompact = 12288;
constexpr size_t kNoAllocBytes = size_t(2) << 20;
static_assert(sizeof(double) * kMaskMaxFrames <= kNoAllocViews - kNoAllocFrames, "frame times fit");
static_assert(sizeof(KCam) * kMaskMaxViews <= kNoAllocCompact - kNoAllocViews, "mask cameras fit");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
fdgs_status noalloc_scratch(void **out, const char *fn) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FDGS_ERR_UNSUPPORTED, "%s: device %d out of range", fn, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FDGS_ERR_HIP, "%s: no device address for the scratch array", fn);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FDGS_OK;
}

}  // namespace

extern "C" {

fdgs_status fdgs_measure_peaks(fdgs_ctx *ctx, double *out, hipStream_t stream) {
    const char *fn = "fdgs_measure_peaks";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (!out) return fail(FDGS_ERR_INVALID_ARG, "%s: out is NULL", fn);
    HIP_TRY(hipSetDevice(ctx->device));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HIP_TRY(ensure(ctx->probe_sink, sizeof(float) * 8 * (size_t)std::max(cus, 1)));
    HIP_TRY(measure_peaks(ctx->probe_sink.as<float>(), out, stream));
    return FDGS_OK;
}

fdgs_status fdgs_mask_overlap(const uint32_t *bits_a, const uint32_t *bits_b, int64_t n, int64_t *out,
                              hipStream_t stream) {
    const char *fn = "fdgs_mask_overlap";
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(FDGS_ERR_INVALID_ARG, "%s: n out of range", fn);
    if (!out || (n > 0 && (!bits_a || !bits_b))) return fail(FDGS_ERR_INVALID_ARG, "%s: a pointer is NULL", fn);
    HIP_TRY(launch_mask_overlap(bits_a, bits_b, n, out, stream));
    return FDGS_OK;
}

fdgs_status fdgs_build_active_mask_noalloc(const fdgs_model *model, const fdgs_mask_spec *spec,
                                           uint32_t *out_bits, uint32_t *out_idx, int64_t *out_count,
                                           hipStream_t stream) {
    const char *fn = "fdgs_build_active_mask_noalloc";
    float amin = 0.0f, dil = 0.0f;
    if (fdgs_status st = check_mask_args(model, spec, out_bits, out_idx, out_count, &amin, &dil, fn)) return st;
    if (spec->mode == FDGS_MASK_CONTRIBUTED)
        return fail(FDGS_ERR_UNSUPPORTED, "%s: mode FDGS_MASK_CONTRIBUTED renders views and needs allocations", fn);
    if (model->n > FDGS_NOALLOC_MAX_GAUSSIANS || compact_scratch_bytes(model->n) > kNoAllocBytes - kNoAllocCompact)
        return fail(FDGS_ERR_INVALID_ARG, "%s: n = %lld exceeds the maximum of %lld Gaussians", fn,
                    (long long)model->n, (long long)FDGS_NOALLOC_MAX_GAUSSIANS);
    unsigned char *base = nullptr;
    if (fdgs_status st = noalloc_scratch(reinterpret_cast<void **>(&base), fn)) return st;
    return enqueue_window_mask(model, spec, amin, dil, reinterpret_cast<double *>(base + kNoAllocFrames),
                               reinterpret_cast<KCam *>(base + kNoAllocViews), base + kNoAllocCompact, out_bits,
                               out_idx, out_count, stream);
}

}  // extern "C"

namespace {

RenderParams make_params(const fdgs_render_cfg *cfg, int32_t W, int32_t H) {
    RenderParams rp;
    rp.tile_w = cfg->tile_w;
    rp.tile_h = cfg->tile_h;
    rp.tiles_x = (W + cfg->tile_w - 1) / cfg->tile_w;
    rp.tiles_y = (H + cfg->tile_h - 1) / cfg->tile_h;
    for (int k = 0; k < 3; ++k) rp.bg[k] = cfg->bg[k];
    rp.alpha_min = cfg->alpha_min;
    rp.alpha_max = cfg->alpha_max;
    rp.t_min = cfg->t_min;
    rp.dilation = cfg->dilation;
    rp.temporal_cull = cfg->temporal_cull ? 1 : 0;
    rp.tile_cull = cfg->tile_cull ? 1 : 0;
    rp.vanilla_level = 2.0 * std::log(1.0 / (double)cfg->alpha_min) * (1.0 + 1e-4) + 1e-4;
    return rp;
}

// The forward pipeline for V views of one resolution.  V == 1: `one` by value,
// processed count optionally on the device (n_dev).  V > 1: `table` is a
// device copy of the views with host-known counts summing to n_total.
// With capture set nothing may synchronise or allocate: the caller guarantees
// buffers are already large enough and a fixed instance capacity is given.
fdgs_status run_forward(fdgs_ctx *ctx, fdgs_state *S, const ViewDesc *one, const ViewDesc *table, int32_t V,
                        const int64_t *n_dev, int64_t n_total, int32_t W, int32_t H, const fdgs_render_cfg *cfg,
                        float *out_rgb, float *out_T, bool need_state, hipStream_t stream, uint8_t *contrib,
                        float *weight) {
    const char *fn = "fdgs_render";
    const RenderParams rp = make_params(cfg, W, H);
    const int64_t tiles_per_view = (int64_t)rp.tiles_x * rp.tiles_y;
    const int64_t n_keys = tiles_per_view * V;
    if (n_keys >= (int64_t(1) << 31)) return fail(FDGS_ERR_INVALID_ARG, "%s: too many tiles x views", fn);
    const int32_t ppt = cfg->pixels_per_thread ? cfg->pixels_per_thread : kDefaultPpt;
    const int64_t n_max = n_total;
    const int64_t npx = (int64_t)W * H;

    HIP_TRY(ensure(S->rec, sizeof(Rec2D) * n_max));
    HIP_TRY(ensure(S->depth_key, sizeof(uint64_t) * n_max));
    HIP_TRY(ensure(S->rect, sizeof(int32_t) * 4 * n_max));
    HIP_TRY(ensure(S->tiles, sizeof(uint32_t) * n_max));
    HIP_TRY(ensure(S->visible, n_max));
    HIP_TRY(ensure(S->order_k, sizeof(uint32_t) * n_max));
    HIP_TRY(ensure(S->order_v, sizeof(uint32_t) * n_max));
    HIP_TRY(ensure(S->order_k2, sizeof(uint32_t) * n_max));
    HIP_TRY(ensure(S->order_v2, sizeof(uint32_t) * n_max));
    HIP_TRY(ensure(S->offsets, sizeof(uint64_t) * n_max));
    if (V > 1) HIP_TRY(ensure(S->view_of, sizeof(uint32_t) * n_max));
    // one view of at most kBucketMaxN processed Gaussians: depth order by buckets (three launches)
    const bool by_buckets = V == 1 && n_max <= kBucketMaxN;
    const int64_t n_buckets = int64_t(1) << bucket_log2_for(n_max);
    if (by_buckets) HIP_TRY(ensure(S->bucket, sizeof(uint32_t) * bucket_scratch_words(n_max)));
    uint32_t *bwork = by_buckets ? S->bucket.as<uint32_t>() : nullptr;
    HIP_TRY(ensure(S->counts, sizeof(int64_t) * 4));
    HIP_TRY(ensure(S->ranges, sizeof(uint32_t) * 2 * n_keys));
    if (cfg->schedule) HIP_TRY(ensure(S->sched, sizeof(uint32_t) * n_keys));
    if (need_state) {
        HIP_TRY(ensure(S->T_final, sizeof(float) * npx));
        HIP_TRY(ensure(S->n_contrib, sizeof(uint32_t) * npx));
    }
    const size_t scratch = std::max(scan_scratch_bytes(n_max), sort_scratch_bytes(n_max));
    HIP_TRY(ensure(S->scratch, scratch));
    int64_t *counts = S->counts.as<int64_t>();
    uint32_t *view_of = V > 1 ? S->view_of.as<uint32_t>() : nullptr;

    HIP_TRY(ensure(S->vis_count, sizeof(uint32_t) * (size_t)((n_total + kPreprocessBlock - 1) / kPreprocessBlock)));
    PreprocOut po{S->rec.as<Rec2D>(), S->depth_key.as<uint64_t>(), S->rect.as<int32_t>(),
                  S->tiles.as<uint32_t>(), S->visible.as<uint8_t>(), view_of, S->vis_count.as<uint32_t>()};
    {
        StageTimer tm(ctx, FDGS_STAGE_PREPROCESS, stream);
        HIP_TRY(launch_preprocess(one, table, V, n_dev, n_total, rp, po, stream));
    }
    {
        StageTimer tm(ctx, FDGS_STAGE_COMPACT, stream);
        if (need_state) HIP_TRY(ensure(S->vis_pos, sizeof(uint32_t) * n_max));
        HIP_TRY(compact_visible(S->visible.as<uint8_t>(), S->depth_key.as<uint64_t>(), n_dev, n_max, counts + 0,
                                S->order_k.as<uint32_t>(), S->order_v.as<uint32_t>(),
                                need_state ? S->vis_pos.as<uint32_t>() : nullptr, bwork, by_buckets ? 2 * n_buckets : 0,
                                by_buckets ? bwork + 3 * n_buckets + 1 : nullptr, S->scratch.p, stream,
                                S->vis_count.as<uint32_t>()));
    }
    uint32_t *ov = nullptr;
    {
        StageTimer tm(ctx, FDGS_STAGE_DEPTH_SORT, stream);
        if (by_buckets) {
            ov = S->order_v2.as<uint32_t>();
            HIP_TRY(depth_order_buckets(S->order_k.as<uint32_t>(), S->order_v.as<uint32_t>(), counts + 0, n_max,
                                        S->depth_key.as<uint64_t>(), bwork, S->order_v.as<uint32_t>(),
                                        S->order_k2.as<uint32_t>(), ov, stream));
        } else {
            int alt = 0;
            HIP_TRY(radix_sort_u32(S->order_k.as<uint32_t>(), S->order_v.as<uint32_t>(), S->order_k2.as<uint32_t>(),
                                   S->order_v2.as<uint32_t>(), counts + 0, n_max, 0, 32, S->scratch.p, &alt, stream));
            uint32_t *ok = alt ? S->order_k2.as<uint32_t>() : S->order_k.as<uint32_t>();
            ov = alt ? S->order_v2.as<uint32_t>() : S->order_v.as<uint32_t>();
            HIP_TRY(launch_fix_depth_ties(ok, ov, S->depth_key.as<uint64_t>(), counts + 0, n_max,
                                          ctx->overflow.as<int32_t>(), stream));
            if (V > 1) {
                // group by view, keeping the depth order inside each view (stable)
                uint32_t *kv = alt ? S->order_k.as<uint32_t>() : S->order_k2.as<uint32_t>();
                uint32_t *vv = alt ? S->order_v.as<uint32_t>() : S->order_v2.as<uint32_t>();
                HIP_TRY(launch_gather_u32(view_of, ov, ok, counts + 0, n_max, stream));
                int alt_v = 0;
                HIP_TRY(radix_sort_u32(ok, ov, kv, vv, counts + 0, n_max, 0, std::max(1, bits_for(V)), S->scratch.p,
                                       &alt_v, stream));
                if (alt_v) ov = vv;
            }
        }
    }
    S->vis_list = need_state ? S->vis_pos.as<uint32_t>() : nullptr;
    {
        StageTimer tm(ctx, FDGS_STAGE_OFFSETS, stream);
        HIP_TRY(scan_u32_to_u64(S->tiles.as<uint32_t>(), ov, S->offsets.as<uint64_t>(), counts + 0, n_max,
                                counts + 1, S->scratch.p, stream));
    }
    int64_t capacity = cfg->instance_capacity;
    if (capacity == 0) {
        HIP_TRY(hipMemcpyAsync(ctx->host_counts, counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        capacity = ctx->host_counts[1];
        if (capacity > 0xffffffffll)
            return fail(FDGS_ERR_CAPACITY, "%s: %lld tile instances exceed 2^32", fn, (long long)capacity);
    }
    HIP_TRY(ensure(S->tkeys, sizeof(uint32_t) * capacity));
    HIP_TRY(ensure(S->tids, sizeof(uint32_t) * capacity));
    HIP_TRY(ensure(S->tkeys2, sizeof(uint32_t) * capacity));
    HIP_TRY(ensure(S->tids2, sizeof(uint32_t) * capacity));
    // the duplicate writes the tile sort's first-digit histogram when its windows tile the sort's blocks
    const int tile_bits = std::max(1, bits_for(n_keys));
    const int sort_chunk = radix_chunk(capacity);
    const int64_t hist_cols = (capacity > 0 && sort_chunk % duplicate_window(capacity) == 0)
                                  ? (capacity + sort_chunk - 1) / sort_chunk * (sort_chunk / duplicate_window(capacity))
                                  : 0;
    HIP_TRY(ensure(S->scratch, std::max(scratch, sort_scratch_bytes(capacity, hist_cols))));
    {
        StageTimer tm(ctx, FDGS_STAGE_DUPLICATE, stream);
        HIP_TRY(launch_duplicate(ov, S->offsets.as<uint64_t>(), S->rect.as<int32_t>(), S->rec.as<Rec2D>(), view_of, counts + 0, n_max, rp,
                                 S->tkeys.as<uint32_t>(), S->tids.as<uint32_t>(), counts + 1, capacity,
                                 ctx->overflow.as<int32_t>(), hist_cols ? S->scratch.as<uint32_t>() : nullptr,
                                 radix_first_bits(0, tile_bits), hist_cols, stream));
    }
    {
        StageTimer tm(ctx, FDGS_STAGE_TILE_SORT, stream);
        int alt2 = 0;
        HIP_TRY(radix_sort_u32(S->tkeys.as<uint32_t>(), S->tids.as<uint32_t>(), S->tkeys2.as<uint32_t>(),
                               S->tids2.as<uint32_t>(), counts + 1, capacity, 0, tile_bits, S->scratch.p, &alt2, stream,
                               hist_cols));
        S->sorted_keys = alt2 ? S->tkeys2.as<uint32_t>() : S->tkeys.as<uint32_t>();
        S->sorted_ids = alt2 ? S->tids2.as<uint32_t>() : S->tids.as<uint32_t>();
    }
    {
        StageTimer tm(ctx, FDGS_STAGE_RANGES, stream);
        HIP_TRY(launch_tile_ranges(S->sorted_keys, counts + 1, capacity, (int32_t)n_keys, S->ranges.as<uint32_t>(),
                                   stream));
        // the longest-first schedule's item order, from the ranges
        if (cfg->schedule == 1)
            HIP_TRY(launch_tile_order(S->ranges.as<uint32_t>(), (int32_t)n_keys, S->sched.as<uint32_t>(), stream));
    }
    float *T_out = need_state ? S->T_final.as<float>() : out_T;
    uint64_t *acc = nullptr;
    if (ctx->prof && !ctx->capturing) {
        HIP_TRY(ensure(ctx->prof_acc, 5 * sizeof(uint64_t)));
        acc = ctx->prof_acc.as<uint64_t>();
        HIP_TRY(launch_accumulate_counts(n_dev, n_total, counts, capacity, acc, stream));
    }
    {
        StageTimer tm(ctx, FDGS_STAGE_COMPOSITE, stream);
        HIP_TRY(launch_composite(rp, W, H, V, cfg->batch, S->ranges.as<uint32_t>(), S->sorted_ids, S->rec.as<Rec2D>(),
                                 out_rgb, T_out, need_state ? S->n_contrib.as<uint32_t>() : nullptr,
                                 acc && ctx->prof == 2 ? acc + 3 : nullptr,
                                 ppt,
                                 cfg->schedule ? S->sched.as<uint32_t>() : nullptr, contrib, weight, stream));
    }
    if (need_state && out_T)
        HIP_TRY(hipMemcpyAsync(out_T, S->T_final.p, sizeof(float) * npx, hipMemcpyDeviceToDevice, stream));
    S->rp = rp;
    S->batch = cfg->batch;
    S->ppt = ppt;
    S->ordered = cfg->schedule == 1;   // its compositor ordered the tiles into sched
    S->capacity = capacity;
    S->W = W;
    S->H = H;
    return FDGS_OK;
}

}  // namespace

extern "C" {

fdgs_status fdgs_render_forward(fdgs_ctx *ctx, const fdgs_model *model, const uint32_t *idx,
                                const int64_t *n_idx_dev, const fdgs_camera *cam, double t,
                                const fdgs_render_cfg *cfg, float *out_rgb, float *out_T,
                                fdgs_state **keep_state, hipStream_t stream) {
    const char *fn = "fdgs_render_forward";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (fdgs_status st = check_model(model, fn)) return st;
    if (fdgs_status st = check_camera(cam, fn)) return st;
    if (fdgs_status st = check_cfg(cfg, fn)) return st;
    if (!std::isfinite(t)) return fail(FDGS_ERR_INVALID_ARG, "%s: t is not finite", fn);
    if (idx && !n_idx_dev) return fail(FDGS_ERR_INVALID_ARG, "%s: idx given without n_idx_dev", fn);
    if (!out_rgb) return fail(FDGS_ERR_INVALID_ARG, "%s: out_rgb is NULL", fn);
    fdgs_state *S = &ctx->scratch_state;
    if (keep_state) {
        if (*keep_state) {
            S = find_state(ctx, *keep_state);
            if (!S) return fail(FDGS_ERR_STATE, "%s: *keep_state does not belong to this context", fn);
        } else {
            S = new (std::nothrow) fdgs_state();
            if (!S) return fail(FDGS_ERR_HIP, "%s: out of host memory", fn);
            S->owner = ctx;
            ctx->states.push_back(S);
            *keep_state = S;
        }
    }
    HIP_TRY(hipSetDevice(ctx->device));
    S->has_forward = false;
    ViewDesc one;
    one.m = kmodel(model);
    one.cam = kcam(cam);
    one.t = t;
    one.idx = idx;
    one.p_off = 0;
    one.n_proc = model->n;
    const int64_t *n_dev = idx ? n_idx_dev : nullptr;
    if (fdgs_status st = run_forward(ctx, S, &one, nullptr, 1, n_dev, model->n, cam->width, cam->height, cfg,
                                     out_rgb, out_T, keep_state != nullptr, stream))
        return st;
    S->model = *model;
    S->idx = idx;
    S->n_idx_dev = n_idx_dev;
    S->cam = one.cam;
    S->t = t;
    S->n_max = model->n;
    S->has_forward = true;
    S->has_g2d = false;
    return FDGS_OK;
}

}  // extern "C"

namespace {

fdgs_status check_batch(const fdgs_model *scenes, int32_t n_scenes, const fdgs_view *views, int32_t n_views,
                        const char *fn) {
    if (n_scenes < 1 || !scenes) return fail(FDGS_ERR_INVALID_ARG, "%s: need at least one scene", fn);
    if (n_views < 1 || !views) return fail(FDGS_ERR_INVALID_ARG, "%s: need at least one view", fn);
    for (int k = 0; k < n_scenes; ++k)
        if (fdgs_status st = check_model(&scenes[k], fn)) return st;
    for (int v = 0; v < n_views; ++v) {
        const fdgs_view &w = views[v];
        if (w.scene < 0 || w.scene >= n_scenes)
            return fail(FDGS_ERR_INVALID_ARG, "%s: view %d names scene %d of %d", fn, v, w.scene, n_scenes);
        if (fdgs_status st = check_camera(&w.cam, fn)) return st;
        if (w.cam.width != views[0].cam.width || w.cam.height != views[0].cam.height)
            return fail(FDGS_ERR_INVALID_ARG, "%s: views differ in image size", fn);
        if (!std::isfinite(w.t)) return fail(FDGS_ERR_INVALID_ARG, "%s: view %d time not finite", fn, v);
        if (w.idx && (w.n_idx < 0 || w.n_idx > scenes[w.scene].n))
            return fail(FDGS_ERR_INVALID_ARG, "%s: view %d n_idx out of range", fn, v);
    }
    return FDGS_OK;
}

// Enqueue every launch of a batch (no graph handling).
fdgs_status enqueue_batch(fdgs_ctx *ctx, const fdgs_model *scenes, const fdgs_view *views, int32_t n_views,
                          const fdgs_render_cfg *cfg, int32_t per_launch, bool upload, float *out_rgb,
                          hipStream_t stream) {
    const int32_t W = views[0].cam.width, H = views[0].cam.height;
    const int64_t img = 3ll * W * H;
    const int32_t n_launch = (n_views + per_launch - 1) / per_launch;
    if (upload && (int32_t)ctx->batch_tables.size() < n_launch) ctx->batch_tables.resize(n_launch);
    // kernels of an earlier batch on this stream may still read the tables
    // about to be overwritten (the upload below is ordered on no stream)
    if (upload) HIP_TRY(hipStreamSynchronize(stream));
    for (int32_t c = 0; c < n_launch; ++c) {
        const int32_t v0 = c * per_launch, V = std::min(per_launch, n_views - v0);
        std::vector<ViewDesc> table(V);
        int64_t off = 0;
        for (int32_t k = 0; k < V; ++k) {
            const fdgs_view &w = views[v0 + k];
            ViewDesc &d = table[k];
            d.m = kmodel(&scenes[w.scene]);
            d.cam = kcam(&w.cam);
            d.t = w.t;
            d.idx = w.idx;
            d.n_proc = w.idx ? w.n_idx : scenes[w.scene].n;
            d.p_off = off;
            off += d.n_proc;
        }
        if (off >= (int64_t(1) << 32))
            return fail(FDGS_ERR_CAPACITY, "fdgs_render_batch: %lld Gaussians in one launch exceed 2^32",
                        (long long)off);
        Buf &tb = ctx->batch_tables[c];
        if (upload) {
            HIP_TRY(ensure(tb, sizeof(ViewDesc) * V));
            HIP_TRY(hipMemcpy(tb.p, table.data(), sizeof(ViewDesc) * V, hipMemcpyHostToDevice));
        }
        if (V == 1) {
            if (fdgs_status st = run_forward(ctx, &ctx->batch_state, &table[0], nullptr, 1, nullptr, off, W, H, cfg,
                                             out_rgb + v0 * img, nullptr, false, stream))
                return st;
        } else {
            if (fdgs_status st = run_forward(ctx, &ctx->batch_state, nullptr, tb.as<ViewDesc>(), V, nullptr, off, W,
                                             H, cfg, out_rgb + v0 * img, nullptr, false, stream))
                return st;
        }
    }
    return FDGS_OK;
}

// A captured graph holds the addresses of the batch buffers and view tables;
// any other use of them (which may re-upload or regrow them) retires it.
void drop_graph(fdgs_ctx *ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
}

template <typename T>
void append_bytes(std::vector<unsigned char> &k, const T *p, size_t n) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(p);
    k.insert(k.end(), b, b + sizeof(T) * n);
}

}  // namespace

extern "C" {

fdgs_status fdgs_render_batch(fdgs_ctx *ctx, const fdgs_model *scenes, int32_t n_scenes, const fdgs_view *views,
                              int32_t n_views, const fdgs_render_cfg *cfg, int32_t views_per_launch,
                              int32_t use_graph, float *out_rgb, hipStream_t stream) {
    const char *fn = "fdgs_render_batch";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (fdgs_status st = check_batch(scenes, n_scenes, views, n_views, fn)) return st;
    if (fdgs_status st = check_cfg(cfg, fn)) return st;
    if (!out_rgb) return fail(FDGS_ERR_INVALID_ARG, "%s: out_rgb is NULL", fn);
    if (views_per_launch < 0) return fail(FDGS_ERR_INVALID_ARG, "%s: views_per_launch < 0", fn);
    if (use_graph && cfg->instance_capacity <= 0)
        return fail(FDGS_ERR_INVALID_ARG, "%s: use_graph needs a fixed instance_capacity", fn);
    const int32_t per = views_per_launch ? std::min(views_per_launch, n_views) : n_views;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!use_graph) {
        drop_graph(ctx);
        return enqueue_batch(ctx, scenes, views, n_views, cfg, per, true, out_rgb, stream);
    }

    std::vector<unsigned char> key;
    append_bytes(key, scenes, n_scenes);
    append_bytes(key, views, n_views);
    append_bytes(key, cfg, 1);
    append_bytes(key, &per, 1);
    append_bytes(key, &out_rgb, 1);
    if (ctx->graph_exec && key == ctx->graph_key) {
        HIP_TRY(hipGraphLaunch(ctx->graph_exec, stream));
        return FDGS_OK;
    }
    drop_graph(ctx);
    // eager run: uploads the view tables and sizes every buffer
    if (fdgs_status st = enqueue_batch(ctx, scenes, views, n_views, cfg, per, true, out_rgb, stream)) return st;
    HIP_TRY(hipStreamSynchronize(stream));
    if (!ctx->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    fdgs_status st = enqueue_batch(ctx, scenes, views, n_views, cfg, per, false, out_rgb, cs);
    ctx->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != FDGS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(FDGS_ERR_HIP, "%s: capture failed: %s", fn, hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(FDGS_ERR_HIP, "%s: graph instantiation failed: %s", fn, hipGetErrorString(e));
    }
    ctx->graph = g;
    ctx->graph_exec = ex;
    ctx->graph_key = key;
    HIP_TRY(hipGraphLaunch(ctx->graph_exec, stream));
    return FDGS_OK;
}

fdgs_status fdgs_autotune(fdgs_ctx *ctx, const fdgs_model *scenes, int32_t n_scenes, const fdgs_view *views,
                          int32_t n_views, int32_t views_per_launch, int32_t repeats, fdgs_render_cfg *inout_cfg,
                          fdgs_tune_result *results, int32_t max_results, int32_t *n_results, hipStream_t stream) {
    const char *fn = "fdgs_autotune";
    if (!ctx || !inout_cfg) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx or cfg is NULL", fn);
    if (fdgs_status st = check_batch(scenes, n_scenes, views, n_views, fn)) return st;
    if (fdgs_status st = check_cfg(inout_cfg, fn)) return st;
    if (repeats < 1) repeats = 1;
    const int32_t per = views_per_launch > 0 ? std::min(views_per_launch, n_views) : n_views;
    HIP_TRY(hipSetDevice(ctx->device));
    drop_graph(ctx);
    const size_t img_bytes = sizeof(float) * 3ull * views[0].cam.width * views[0].cam.height * n_views;
    HIP_TRY(ensure(ctx->tune_ref, img_bytes));
    HIP_TRY(ensure(ctx->tune_img, img_bytes));
    HIP_TRY(ensure(ctx->tune_diff, sizeof(unsigned long long)));
    struct Cand { int tw, th, b, ppt, sched; };
    std::vector<Cand> cands;
    const int shapes[5][2] = {{16, 16}, {8, 8}, {32, 8}, {32, 16}, {32, 32}};
    for (int sched : {1, 0})
        for (auto &sh : shapes)
            for (int b : {64, 128, 256, 512, 1024})
                for (int ppt : {1, 2, 4})
                    if ((sh[0] * sh[1] > 64 || ppt == 1) && (b <= 256 || sh[0] * sh[1] == 1024))
                        cands.push_back({sh[0], sh[1], b, ppt, sched});
    hipEvent_t e0 = ctx->get_event(), e1 = ctx->get_event();
    if (!e0 || !e1) return fail(FDGS_ERR_HIP, "%s: event creation failed", fn);
    double best = 1e300;
    int best_i = -1;
    bool all_same = true;
    int32_t tried = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        fdgs_render_cfg c = *inout_cfg;
        c.tile_w = cands[i].tw;
        c.tile_h = cands[i].th;
        c.batch = cands[i].b;
        c.pixels_per_thread = cands[i].ppt;
        c.schedule = cands[i].sched;
        c.instance_capacity = 0;   // exact sizing: tile counts change with the tile shape
        float *dst = (i == 0 ? ctx->tune_ref : ctx->tune_img).as<float>();
        if (fdgs_status st = enqueue_batch(ctx, scenes, views, n_views, &c, per, true, dst, stream)) return st;
        double ms_best = 1e300;
        for (int r = 0; r < repeats; ++r) {
            HIP_TRY(hipEventRecord(e0, stream));
            if (fdgs_status st = enqueue_batch(ctx, scenes, views, n_views, &c, per, false, dst, stream)) return st;
            HIP_TRY(hipEventRecord(e1, stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            ms_best = std::min(ms_best, (double)ms);
        }
        bool same = true;
        if (i > 0) {
            unsigned long long diff = 0;
            HIP_TRY(launch_count_diff(ctx->tune_ref.as<uint32_t>(), ctx->tune_img.as<uint32_t>(),
                                      (int64_t)(img_bytes / 4), ctx->tune_diff.as<unsigned long long>(), stream));
            HIP_TRY(hipMemcpyAsync(&diff, ctx->tune_diff.p, sizeof diff, hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            same = diff == 0;
        }
        all_same = all_same && same;
        if (results && tried < max_results)
            results[tried] = fdgs_tune_result{c.tile_w, c.tile_h, c.batch, c.pixels_per_thread, c.schedule, ms_best,
                                              same ? 1 : 0};
        ++tried;
        if (same && ms_best < best) {
            best = ms_best;
            best_i = (int)i;
        }
    }
    ctx->free_events.push_back(e0);
    ctx->free_events.push_back(e1);
    if (n_results) *n_results = tried;
    if (best_i >= 0) {
        inout_cfg->tile_w = cands[best_i].tw;
        inout_cfg->tile_h = cands[best_i].th;
        inout_cfg->batch = cands[best_i].b;
        inout_cfg->pixels_per_thread = cands[best_i].ppt;
        inout_cfg->schedule = cands[best_i].sched;
    }
    if (!all_same) return fail(FDGS_ERR_STATE, "%s: a configuration rendered different images", fn);
    return FDGS_OK;
}

}  // extern "C"

namespace {

// The state a backward phase may use, or an error.
fdgs_status backward_state(fdgs_ctx *ctx, fdgs_state *state, const char *fn, fdgs_state **out) {
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    fdgs_state *S = state ? find_state(ctx, state) : nullptr;
    if (!S) return fail(FDGS_ERR_STATE, "%s: state is not a live state of this context", fn);
    if (!S->has_forward) return fail(FDGS_ERR_STATE, "%s: state holds no forward pass", fn);
    if (S->model.sh_index)
        return fail(FDGS_ERR_UNSUPPORTED, "%s: the forward used vector-quantised SH (no adjoint)", fn);
    *out = S;
    return FDGS_OK;
}

fdgs_status check_grads(const fdgs_state *S, const fdgs_grads *grads, const char *fn) {
    if (!grads) return fail(FDGS_ERR_INVALID_ARG, "%s: grads is NULL", fn);
    if (S->model.n > 0 && (!grads->mean || !grads->log_scale || !grads->q_left || !grads->q_right ||
                           !grads->opacity_logit || !grads->sh))
        return fail(FDGS_ERR_INVALID_ARG, "%s: a gradient pointer is NULL", fn);
    return FDGS_OK;
}

// Phase 1: adjoint compositor into the state's per-Gaussian 2D gradients.
fdgs_status enqueue_backward_2d(fdgs_ctx *ctx, fdgs_state *S, const float *dL_drgb, hipStream_t stream) {
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(ensure(S->g2d, sizeof(float) * 9 * std::max<int64_t>(S->n_max, 1)));
    StageTimer tm(ctx, FDGS_STAGE_BWD_COMPOSITE, stream);
    HIP_TRY(launch_fill_u32(S->g2d.as<uint32_t>(), 9 * std::max<int64_t>(S->n_max, 1), 0u, stream));
    // the adjoint takes the tiles longest list first: the forward's order when it
    // made one, else one made here
    const int32_t n_tiles = S->rp.tiles_x * S->rp.tiles_y;
    if (!S->ordered) {
        HIP_TRY(ensure(S->sched, sizeof(uint32_t) * std::max<int32_t>(n_tiles, 1)));
        HIP_TRY(launch_tile_order(S->ranges.as<uint32_t>(), n_tiles, S->sched.as<uint32_t>(), stream));
        S->ordered = true;
    }
    HIP_TRY(launch_composite_backward(S->rp, S->W, S->H, S->batch, S->ppt, S->ranges.as<uint32_t>(), S->sorted_ids,
                                      S->rec.as<Rec2D>(), S->T_final.as<float>(), S->n_contrib.as<uint32_t>(),
                                      dL_drgb, S->g2d.as<float>(), S->n_max, S->sched.as<uint32_t>(), stream));
    S->has_g2d = true;
    return FDGS_OK;
}

// Phase 2: the 2D gradients through projection, slicing and activations into grads.
fdgs_status enqueue_backward_params(fdgs_ctx *ctx, fdgs_state *S, const fdgs_grads *grads, hipStream_t stream) {
    HIP_TRY(hipSetDevice(ctx->device));
    StageTimer tm(ctx, FDGS_STAGE_BWD_PREPROCESS, stream);
    const int64_t *n_proc_dev = S->idx ? S->n_idx_dev : nullptr;
    HIP_TRY(launch_preprocess_backward(kmodel(&S->model), S->idx, n_proc_dev, S->n_max, S->cam, S->t, S->rp,
                                       S->vis_list, S->counts.as<int64_t>(), S->g2d.as<float>(), *grads, stream));
    return FDGS_OK;
}

}  // namespace

extern "C" {

fdgs_status fdgs_render_backward(fdgs_ctx *ctx, fdgs_state *state, const float *dL_drgb, const fdgs_grads *grads,
                                 hipStream_t stream) {
    const char *fn = "fdgs_render_backward";
    fdgs_state *S = nullptr;
    if (fdgs_status st = backward_state(ctx, state, fn, &S)) return st;
    if (!dL_drgb) return fail(FDGS_ERR_INVALID_ARG, "%s: dL_drgb is NULL", fn);
    if (fdgs_status st = check_grads(S, grads, fn)) return st;
    if (fdgs_status st = enqueue_backward_2d(ctx, S, dL_drgb, stream)) return st;
    return enqueue_backward_params(ctx, S, grads, stream);
}

fdgs_status fdgs_render_backward_2d(fdgs_ctx *ctx, fdgs_state *state, const float *dL_drgb, hipStream_t stream) {
    const char *fn = "fdgs_render_backward_2d";
    fdgs_state *S = nullptr;
    if (fdgs_status st = backward_state(ctx, state, fn, &S)) return st;
    if (!dL_drgb) return fail(FDGS_ERR_INVALID_ARG, "%s: dL_drgb is NULL", fn);
    return enqueue_backward_2d(ctx, S, dL_drgb, stream);
}

fdgs_status fdgs_render_backward_params(fdgs_ctx *ctx, fdgs_state *state, const fdgs_grads *grads,
                                        hipStream_t stream) {
    const char *fn = "fdgs_render_backward_params";
    fdgs_state *S = nullptr;
    if (fdgs_status st = backward_state(ctx, state, fn, &S)) return st;
    if (!S->has_g2d)
        return fail(FDGS_ERR_STATE, "%s: no fdgs_render_backward_2d since the state's last forward", fn);
    if (fdgs_status st = check_grads(S, grads, fn)) return st;
    return enqueue_backward_params(ctx, S, grads, stream);
}

fdgs_status fdgs_state_release(fdgs_ctx *ctx, fdgs_state *state) {
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "fdgs_state_release: ctx is NULL");
    if (!state) return FDGS_OK;
    auto it = std::find(ctx->states.begin(), ctx->states.end(), state);
    if (it == ctx->states.end()) return fail(FDGS_ERR_STATE, "fdgs_state_release: unknown state");
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    state->free_all();
    delete state;
    ctx->states.erase(it);
    return FDGS_OK;
}

fdgs_status fdgs_state_binning(fdgs_ctx *ctx, fdgs_state *state, fdgs_binning *out, hipStream_t stream) {
    const char *fn = "fdgs_state_binning";
    if (!ctx || !out) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx or out is NULL", fn);
    fdgs_state *S = state ? find_state(ctx, state) : nullptr;
    if (!S || !S->has_forward) return fail(FDGS_ERR_STATE, "%s: no forward pass in state", fn);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipMemcpyAsync(ctx->host_counts, S->counts.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    int64_t nproc = S->n_max;
    if (S->idx) HIP_TRY(hipMemcpyAsync(ctx->host_counts + 2, S->n_idx_dev, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (S->idx) nproc = std::min(ctx->host_counts[2], S->n_max);
    out->sorted_ids = S->sorted_ids;
    out->tile_ranges = S->ranges.as<uint32_t>();
    out->rects = S->rect.as<int32_t>();
    out->depth = reinterpret_cast<const double *>(S->depth_key.p);
    out->visible = S->visible.as<uint8_t>();
    out->n_vis = ctx->host_counts[0];
    out->n_inst = std::min(ctx->host_counts[1], S->capacity);
    out->n_proc = nproc;
    out->n_tiles = S->rp.tiles_x * S->rp.tiles_y;
    out->tiles_x = S->rp.tiles_x;
    out->tiles_y = S->rp.tiles_y;
    return FDGS_OK;
}

fdgs_status fdgs_profile_enable(fdgs_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "fdgs_profile_enable: ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    if (enable && !ctx->prof_acc.p) {
        HIP_TRY(ensure(ctx->prof_acc, 5 * sizeof(uint64_t)));
        HIP_TRY(hipMemset(ctx->prof_acc.p, 0, 5 * sizeof(uint64_t)));
    }
    ctx->prof = enable <= 0 ? 0 : (enable >= 2 ? 2 : 1);
    return FDGS_OK;
}

fdgs_status fdgs_profile_read(fdgs_ctx *ctx, fdgs_profile *out, int32_t reset) {
    if (!ctx || !out) return fail(FDGS_ERR_INVALID_ARG, "fdgs_profile_read: ctx or out is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipDeviceSynchronize());
    for (auto &p : ctx->pending) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.e0, p.e1));
        ctx->ms[p.stage] += ms;
        ctx->calls[p.stage] += 1;
        ctx->free_events.push_back(p.e0);
        ctx->free_events.push_back(p.e1);
    }
    ctx->pending.clear();
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < FDGS_NUM_STAGES; ++k) {
        out->ms[k] = ctx->ms[k];
        out->calls[k] = ctx->calls[k];
    }
    if (ctx->prof_acc.p) {
        uint64_t acc[5];
        HIP_TRY(hipMemcpy(acc, ctx->prof_acc.p, sizeof acc, hipMemcpyDeviceToHost));
        out->processed = (int64_t)acc[0];
        out->visible = (int64_t)acc[1];
        out->instances = (int64_t)acc[2];
        out->pairs = acc[3];
        out->blended = acc[4];
        if (reset) HIP_TRY(hipMemset(ctx->prof_acc.p, 0, sizeof acc));
    }
    if (reset) {
        for (int k = 0; k < FDGS_NUM_STAGES; ++k) {
            ctx->ms[k] = 0.0;
            ctx->calls[k] = 0;
        }
    }
    return FDGS_OK;
}

fdgs_status fdgs_spatial_score(fdgs_ctx *ctx, const fdgs_model *model, const fdgs_camera *cams, const double *times,
                               int32_t n_views, const fdgs_render_cfg *cfg, float *inout_score, hipStream_t stream) {
    const char *fn = "fdgs_spatial_score";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (fdgs_status st = check_model(model, fn)) return st;
    if (n_views < 0 || (n_views > 0 && (!cams || !times)))
        return fail(FDGS_ERR_INVALID_ARG, "%s: need n_views >= 0 cameras and times", fn);
    fdgs_render_cfg c;
    if (cfg) {
        if (fdgs_status st = check_cfg(cfg, fn)) return st;
        c = *cfg;
    } else {
        fdgs_render_cfg_default(&c);
        c.pixels_per_thread = 2;
    }
    c.instance_capacity = 0;
    if (c.tile_w * c.tile_h == 64) c.pixels_per_thread = 1;
    if (model->n > 0 && !inout_score) return fail(FDGS_ERR_INVALID_ARG, "%s: inout_score is NULL", fn);
    for (int v = 0; v < n_views; ++v) {
        if (fdgs_status st = check_camera(&cams[v], fn)) return st;
        if (!std::isfinite(times[v])) return fail(FDGS_ERR_INVALID_ARG, "%s: view %d time not finite", fn, v);
    }
    HIP_TRY(hipSetDevice(ctx->device));
    int64_t px_max = 1;
    for (int v = 0; v < n_views; ++v) px_max = std::max<int64_t>(px_max, (int64_t)cams[v].width * cams[v].height);
    HIP_TRY(ensure(ctx->mask_img, sizeof(float) * 3 * (size_t)px_max));
    for (int v = 0; v < n_views; ++v) {
        ViewDesc one;
        one.m = kmodel(model);
        one.cam = kcam(&cams[v]);
        one.t = times[v];
        one.idx = nullptr;
        one.p_off = 0;
        one.n_proc = model->n;
        if (fdgs_status st = run_forward(ctx, &ctx->scratch_state, &one, nullptr, 1, nullptr, model->n, cams[v].width,
                                         cams[v].height, &c, ctx->mask_img.as<float>(), nullptr, false, stream,
                                         nullptr, inout_score))
            return st;
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return FDGS_OK;
}

fdgs_status fdgs_variation_score(fdgs_ctx *ctx, const fdgs_model *model, const double *times, int32_t n_times,
                                 const float *spatial, float *out_score, hipStream_t stream) {
    const char *fn = "fdgs_variation_score";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (fdgs_status st = check_model(model, fn)) return st;
    if (n_times < 0 || (n_times > 0 && !times)) return fail(FDGS_ERR_INVALID_ARG, "%s: bad times", fn);
    for (int f = 0; f < n_times; ++f)
        if (!std::isfinite(times[f])) return fail(FDGS_ERR_INVALID_ARG, "%s: non-finite time", fn);
    const int64_t n = model->n;
    if (n > 0 && (!spatial || !out_score)) return fail(FDGS_ERR_INVALID_ARG, "%s: a score pointer is NULL", fn);
    if (n == 0) return FDGS_OK;
    if (n >= (int64_t(1) << 32)) return fail(FDGS_ERR_INVALID_ARG, "%s: n too large", fn);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(ensure(ctx->prune_times, sizeof(double) * std::max(1, n_times)));
    if (n_times > 0)
        HIP_TRY(hipMemcpyAsync(ctx->prune_times.p, times, sizeof(double) * n_times, hipMemcpyHostToDevice, stream));
    HIP_TRY(ensure(ctx->prune_a, sizeof(float) * n));      // S^TV
    HIP_TRY(ensure(ctx->prune_b, sizeof(uint32_t) * n));   // volume keys
    HIP_TRY(ensure(ctx->prune_c, sizeof(uint32_t) * n));   // values
    HIP_TRY(ensure(ctx->prune_d, sizeof(uint32_t) * 3 * n));   // sort ping-pong (keys, values) and a copy
    HIP_TRY(ensure(ctx->prune_e, sort_scratch_bytes(n)));
    uint32_t *vk = ctx->prune_b.as<uint32_t>(), *vv = ctx->prune_c.as<uint32_t>();
    uint32_t *k2 = ctx->prune_d.as<uint32_t>(), *v2 = k2 + n, *keep_keys = v2 + n;
    HIP_TRY(launch_temporal_volume(kmodel(model), ctx->prune_times.as<double>(), n_times, ctx->prune_a.as<float>(),
                                   vk, vv, stream));
    HIP_TRY(hipMemcpyAsync(keep_keys, vk, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, stream));
    int alt = 0;
    HIP_TRY(radix_sort_u32(vk, vv, k2, v2, nullptr, n, 0, 32, ctx->prune_e.p, &alt, stream));
    const uint32_t *sorted = alt ? k2 : vk;
    const int64_t q = (int64_t)std::floor(0.9 * (double)(n - 1));
    HIP_TRY(launch_variation_score(ctx->prune_a.as<float>(), keep_keys, sorted, n, q, spatial, out_score, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return FDGS_OK;
}

fdgs_status fdgs_prune(fdgs_ctx *ctx, const float *score, int64_t n, int64_t n_keep, uint32_t *out_bits,
                       uint32_t *out_idx, int64_t *out_count, hipStream_t stream) {
    const char *fn = "fdgs_prune";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (n < 0 || n >= (int64_t(1) << 32)) return fail(FDGS_ERR_INVALID_ARG, "%s: n out of range", fn);
    if (n_keep < 0 || n_keep > n) return fail(FDGS_ERR_INVALID_ARG, "%s: n_keep out of range", fn);
    if (!out_bits || !out_idx || !out_count || (n > 0 && !score))
        return fail(FDGS_ERR_INVALID_ARG, "%s: a pointer is NULL", fn);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(ensure(ctx->prune_b, sizeof(uint32_t) * std::max<int64_t>(n, 1)));
    HIP_TRY(ensure(ctx->prune_c, sizeof(uint32_t) * std::max<int64_t>(n, 1)));
    HIP_TRY(ensure(ctx->prune_d, sizeof(uint32_t) * 3 * std::max<int64_t>(n, 1)));
    HIP_TRY(ensure(ctx->prune_e, std::max(sort_scratch_bytes(n), compact_scratch_bytes(n))));
    HIP_TRY(ensure(ctx->mask_flags, (size_t)((n + 3) / 4) * 4 + 4));
    uint32_t *keys = ctx->prune_b.as<uint32_t>(), *vals = ctx->prune_c.as<uint32_t>();
    uint32_t *k2 = ctx->prune_d.as<uint32_t>(), *v2 = k2 + n;
    HIP_TRY(launch_fill_u32(ctx->mask_flags.as<uint32_t>(), (n + 3) / 4, 0u, stream));
    HIP_TRY(launch_prune_keys(score, n, keys, vals, stream));
    int alt = 0;
    HIP_TRY(radix_sort_u32(keys, vals, k2, v2, nullptr, n, 0, 32, ctx->prune_e.p, &alt, stream));
    HIP_TRY(launch_mark_first(alt ? v2 : vals, n_keep, ctx->mask_flags.as<uint8_t>(), stream));
    HIP_TRY(launch_flags_to_bits(ctx->mask_flags.as<uint8_t>(), n, out_bits, stream));
    HIP_TRY(compact_bits(out_bits, n, out_idx, out_count, ctx->prune_e.p, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return FDGS_OK;
}

fdgs_status fdgs_sh_kmeans(fdgs_ctx *ctx, const fdgs_model *model, const uint32_t *init_index, int64_t k,
                           int32_t iterations, float *codebook, uint32_t *assignment, hipStream_t stream) {
    const char *fn = "fdgs_sh_kmeans";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (fdgs_status st = check_model(model, fn)) return st;
    if (!model->sh) return fail(FDGS_ERR_INVALID_ARG, "%s: model->sh is NULL (nothing to quantise)", fn);
    if (k < 1 || k > (int64_t(1) << 24)) return fail(FDGS_ERR_INVALID_ARG, "%s: k=%lld not in [1, 2^24]", fn, (long long)k);
    if (iterations < 0 || iterations > 1000)
        return fail(FDGS_ERR_INVALID_ARG, "%s: iterations=%d not in [0, 1000]", fn, iterations);
    if (!init_index || !codebook || !assignment)
        return fail(FDGS_ERR_INVALID_ARG, "%s: init_index, codebook or assignment is NULL", fn);
    if (reinterpret_cast<uintptr_t>(codebook) % 16 != 0)
        return fail(FDGS_ERR_INVALID_ARG, "%s: codebook must be 16-byte aligned", fn);
    if (model->n == 0) return FDGS_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(ensure(ctx->vq_scratch, vq_scratch_bytes(model->n, k)));
    HIP_TRY(vq_kmeans(model->sh, model->n, init_index, k, iterations, codebook, assignment, ctx->vq_scratch.p,
                      stream));
    return FDGS_OK;
}

fdgs_status fdgs_adam_step(fdgs_ctx *ctx, float *param, const float *grad, float *m, float *v, int64_t n, float lr,
                           float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
    const char *fn = "fdgs_adam_step";
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "%s: ctx is NULL", fn);
    if (n < 0) return fail(FDGS_ERR_INVALID_ARG, "%s: n < 0", fn);
    if (n > 0 && (!param || !grad || !m || !v)) return fail(FDGS_ERR_INVALID_ARG, "%s: a pointer is NULL", fn);
    if (step < 1) return fail(FDGS_ERR_INVALID_ARG, "%s: step must be >= 1", fn);
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
        !std::isfinite(lr))
        return fail(FDGS_ERR_INVALID_ARG, "%s: need 0 <= beta < 1, eps > 0, finite lr", fn);
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step, stream));
    return FDGS_OK;
}

fdgs_status fdgs_check_overflow(fdgs_ctx *ctx, hipStream_t stream) {
    if (!ctx) return fail(FDGS_ERR_INVALID_ARG, "fdgs_check_overflow: ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    int32_t flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, ctx->overflow.p, sizeof flag, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (flag) {
        HIP_TRY(hipMemsetAsync(ctx->overflow.p, 0, sizeof flag, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (flag & 1)
            return fail(FDGS_ERR_CAPACITY, "fdgs_check_overflow: a forward pass exceeded its instance capacity");
        return fail(FDGS_ERR_UNSUPPORTED,
                    "fdgs_check_overflow: more than 4096 Gaussians shared one float32 depth; "
                    "their order fell back to processing order");
    }
    return FDGS_OK;
}

}  // extern "C"
