// Internal declarations shared by the host side of libfdgs (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fdgs.h"
#include "kernel_types.h"

namespace fdgs {

// Launch wrappers (each .hip file owns its kernels).  All are asynchronous.
hipError_t launch_slice(const KModel &m, double t, const uint32_t *idx, int64_t count,
                        float *mean3, float *cov3, float *p, hipStream_t s);

// One (scene, camera, time) view of a forward pass.  Its processed entries
// occupy [p_off, p_off + n_proc) of the concatenated per-Gaussian buffers.
struct ViewDesc {
    KModel m;
    KCam cam;
    double t;
    const uint32_t *idx;   // processed subset of the scene, or null for all
    int64_t p_off;
    int64_t n_proc;
};

struct PreprocOut {
    Rec2D *rec;          // [P]
    uint64_t *depth_key; // [P] float64 bits of z
    int32_t *rect;       // [P][4]
    uint32_t *tiles;     // [P] tiles touched (0 = not visible)
    uint8_t *visible;    // [P]
    uint32_t *view_of;   // [P] view of each entry (written when V > 1)
    uint32_t *vis_count; // [ceil(P / kPreprocessBlock)] visible entries per workgroup, or NULL
};
// Entries per preprocess workgroup (its visible counts feed the compaction's scan).
constexpr int kPreprocessBlock = 256;
// V == 1: `one` is passed by value and n_dev may hold the device count.
// V > 1: `table` is a device array of V views with host-known counts.
hipError_t launch_preprocess(const ViewDesc *one, const ViewDesc *table, int32_t V, const int64_t *n_dev,
                             int64_t n_total, const RenderParams &rp, const PreprocOut &out, hipStream_t s);

struct MaskArgs {
    const double *frames;   // device [n_frames]
    int32_t n_frames;
    const KCam *views;      // device [n_views]
    int32_t n_views;
    double key_lo, key_hi;
    int32_t mode;
    double level;           // 2 ln(1/alpha_min)
    double rect_level;      // footprint Mahalanobis level incl. margin
    double dilation;
};
hipError_t launch_mask_bits(const KModel &m, const MaskArgs &a, uint32_t *bits, hipStream_t s);

// Exclusive scans.  n is read from n_dev when non-null (bounded by n_max).
size_t scan_scratch_bytes(int64_t n_max);
hipError_t scan_flags_u8(const uint8_t *in, uint32_t *out, const int64_t *n_dev, int64_t n_max,
                         int64_t *total, void *scratch, hipStream_t s);
hipError_t scan_u32_to_u64(const uint32_t *in, const uint32_t *gather, uint64_t *out,
                           const int64_t *n_dev, int64_t n_max, int64_t *total,
                           void *scratch, hipStream_t s);
// Visible entries in order -> keys32 = float32 bits of their depth, vals = position (and, when asc is
// not NULL, asc = position too: a copy the depth sort does not overwrite); *total = count.  Before the
// entries are written, clear[0..n_clear) is zeroed and range (when not NULL) receives the [min, max]
// of the keys.  vis_count (may be NULL): the preprocess's visible count per workgroup of
// kPreprocessBlock entries (ceil(n_max / kPreprocessBlock) of them), which replaces the scan's
// first pass over the flags.
hipError_t compact_visible(const uint8_t *visible, const uint64_t *depth_key, const int64_t *n_dev, int64_t n_max,
                           int64_t *total, uint32_t *keys32, uint32_t *vals, uint32_t *asc, uint32_t *clear,
                           int64_t n_clear, uint32_t *range, void *scratch, hipStream_t s,
                           const uint32_t *vis_count = nullptr);

// Depth order of one view's visible entries by bucketing and per-bucket sorts: out[0..n_vis) = the
// positions (vals) ordered by (depth_key[pos], pos).  work holds bucket_scratch_words(n_max) words:
// counts and cursors (words [0, 2 nb), cleared by compact_visible), bucket starts, and the key range
// (words 3 nb + 1 and 3 nb + 2, filled by compact_visible).  bucketed and alt are scratch of n_max
// words; none of the arrays may alias.
int bucket_log2_for(int64_t n_max);
size_t bucket_scratch_words(int64_t n_max);
hipError_t depth_order_buckets(const uint32_t *keys32, const uint32_t *vals, const int64_t *n_vis_dev, int64_t n_max,
                               const uint64_t *depth_key, uint32_t *work, uint32_t *alt, uint32_t *bucketed,
                               uint32_t *out, hipStream_t s);
hipError_t compact_bits(const uint32_t *bits, int64_t n, uint32_t *idx, int64_t *count,
                        void *scratch, hipStream_t s);
size_t compact_scratch_bytes(int64_t n);

// Stable LSD radix sort of (key, uint32 value) pairs, digits of at most 8 bits (passes of near-equal
// width).  Keys [b chunk, (b + 1) chunk) form block b of every pass (chunk = radix_chunk(n_max)).  When
// first_hist_cols > 0 the first pass's digit histogram (digit-major, first_hist_cols columns, an equal
// number per block, digit width radix_first_bits) is already at the start of scratch.
size_t sort_scratch_bytes(int64_t n_max, int64_t hist_cols = 0);
int radix_chunk(int64_t n_max);
int radix_first_bits(int begin_bit, int end_bit);
hipError_t radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                          const int64_t *n_dev, int64_t n_max, int begin_bit, int end_bit,
                          void *scratch, int *result_in_alt, hipStream_t s, int64_t first_hist_cols = 0);

// Visible-set compaction, depth ordering and tile binning.
hipError_t launch_scatter_visible(const uint8_t *visible, const uint32_t *pos,
                                  const uint64_t *depth_key, const int64_t *n_dev, int64_t n_max,
                                  uint32_t *keys32, uint32_t *vals, hipStream_t s);
// flag |= 2 when a run of equal float32 depths is too long to reorder.
hipError_t launch_fix_depth_ties(uint32_t *keys32, uint32_t *vals, const uint64_t *depth_key,
                                 const int64_t *n_vis_dev, int64_t n_max, int32_t *flag, hipStream_t s);
// Tile key = view * tiles_per_view + ty * tiles_x + tx (view_of null: view 0).  Instances are written
// in windows of duplicate_window(capacity); with hist, window w also writes hist[d * hist_cols + w] = its count
// of keys whose low hist_bits bits equal d (d < 256), and the launch has exactly hist_cols windows.
int duplicate_window(int64_t capacity);
hipError_t launch_duplicate(const uint32_t *order, const uint64_t *offsets, const int32_t *rect,
                            const Rec2D *rec, const uint32_t *view_of, const int64_t *n_vis_dev, int64_t n_max,
                            const RenderParams &rp, uint32_t *tile_keys, uint32_t *ids,
                            const int64_t *n_inst_dev, int64_t capacity, int32_t *overflow, uint32_t *hist,
                            int hist_bits, int64_t hist_cols, hipStream_t s);
// dst[j] = src[idx[j]] for j < count.
hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, const int64_t *n_dev,
                             int64_t n_max, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t *tile_keys, const int64_t *n_inst_dev, int64_t n_max,
                              int32_t n_tiles, uint32_t *ranges, hipStream_t s);

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
// *out = number of 32-bit words where a and b differ.
hipError_t launch_count_diff(const uint32_t *a, const uint32_t *b, int64_t n, unsigned long long *out,
                             hipStream_t s);
// Profiling: acc[0..2] += processed, visible, instances (instances clamped to capacity).
hipError_t launch_accumulate_counts(const int64_t *n_proc_dev, int64_t n_proc, const int64_t *counts,
                                    int64_t capacity, uint64_t *acc, hipStream_t s);

// Compositing.  pair_counter (optional, two words) accumulates evaluated (pixel, Gaussian)
// pairs and, of those, the pairs that were blended.
// V views of W x H share one tile grid: item i renders tile i % n_tiles of
// view i / n_tiles; view v writes out_rgb + v*3*W*H (out_T, n_contrib: + v*W*H).
// sched == NULL: one workgroup per item in item order.  Otherwise sched holds
// the V * n_tiles items longest list first (launch_tile_order), and workgroup b
// renders the b-th of them.
// contrib (optional): contrib[id] = 1 for every processed entry some pixel
// blends; weight (optional): weight[id] += the entry's summed blend weights
// alpha T (state and counters are not recorded in either case).
hipError_t launch_composite(const RenderParams &rp, int32_t W, int32_t H, int32_t V, int32_t batch,
                            const uint32_t *ranges, const uint32_t *ids, const Rec2D *rec,
                            float *out_rgb, float *out_T, uint32_t *n_contrib,
                            uint64_t *pair_counter, int32_t pixels_per_thread, uint32_t *sched,
                            uint8_t *contrib, float *weight, hipStream_t s);
// bits[w] bit j = (flags[32 w + j] != 0), j < 32, for n flags.
hipError_t launch_flags_to_bits(const uint8_t *flags, int64_t n, uint32_t *bits, hipStream_t s);
// Rates measured on the current device (sink: device float[8 x CUs], never
// written in practice): out[0] LDS bytes/s read as broadcasts, out[1] LDS
// bytes/s read at lane-distinct addresses, out[2] float32 FMA lane-operations/s,
// out[3] compute units.  Synchronises s.
hipError_t measure_peaks(float *sink, double *out, hipStream_t s);
// out[0..2] = popcounts of a, b and a & b over the first n bits (device int64[3]).
hipError_t launch_mask_overlap(const uint32_t *a, const uint32_t *b, int64_t n, int64_t *out, hipStream_t s);

// Backward.
hipError_t launch_composite_backward(const RenderParams &rp, int32_t W, int32_t H, int32_t batch, int32_t ppt,
                                     const uint32_t *ranges, const uint32_t *ids, const Rec2D *rec,
                                     const float *T_final, const uint32_t *n_contrib,
                                     const float *dL_drgb, float *g2d, int64_t n_proc_max,
                                     const uint32_t *order, hipStream_t s);
// order[0 .. n_items): the items of ranges sorted by list length, longest first
// (the order of the compositors' longest-first schedule).
hipError_t launch_tile_order(const uint32_t *ranges, int32_t n_items, uint32_t *order, hipStream_t s);
hipError_t launch_preprocess_backward(const KModel &m, const uint32_t *idx, const int64_t *n_dev,
                                      int64_t n_max, const KCam &cam, double t,
                                      const RenderParams &rp, const uint32_t *vis_list,
                                      const int64_t *n_vis_dev, const float *g2d, const fdgs_grads &grads,
                                      hipStream_t s);

// Pruning score helpers (k_prune.hip).
hipError_t launch_temporal_volume(const KModel &m, const double *times, int32_t n_times, float *tv,
                                  uint32_t *vol_key, uint32_t *vals, hipStream_t s);
hipError_t launch_variation_score(const float *tv, const uint32_t *vol_key, const uint32_t *sorted_vol, int64_t n,
                                  int64_t q, const float *spatial, float *out, hipStream_t s);
hipError_t launch_prune_keys(const float *score, int64_t n, uint32_t *keys, uint32_t *vals, hipStream_t s);
hipError_t launch_mark_first(const uint32_t *sorted_vals, int64_t n_keep, uint8_t *flags, hipStream_t s);

// SH k-means (codebook [k][48], assignment [n]); scratch of vq_scratch_bytes(n, k).
size_t vq_scratch_bytes(int64_t n, int64_t k);
hipError_t vq_kmeans(const float *sh, int64_t n, const uint32_t *init, int64_t k, int32_t iterations, float *code,
                     uint32_t *assign, void *scratch, hipStream_t s);

// Adam (k_optim.hip).
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                       float eps, int32_t step, hipStream_t s);

}  // namespace fdgs
