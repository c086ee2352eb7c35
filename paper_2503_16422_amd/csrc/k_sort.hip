// Stable LSD radix sort of (uint32 key, uint32 value) pairs with 8-bit
// digits, plus the binning kernels around it: compaction of visible
// Gaussians, exact float64 depth order, tile-key duplication and tile ranges.
//
// Depth order (Eq. 2 blends "sorted by depth"): the visible Gaussians are
// sorted by the float32-rounded depth (4 digit passes over N_vis, stable, so
// equal keys stay in processing order), and runs of equal float32 keys, which
// are rare and short, are then re-ordered by the float64 depth and the
// processing position.  Rounding is monotone, so the result is the order by
// (float64 depth, position).
//
// Tile binning: instances are emitted in that depth order and then sorted
// stably by tile id alone (ceil(tile_bits / 8) passes over the instances),
// which yields each tile's list in depth order without sorting 64-bit
// (tile, depth) keys over every instance.
#include <hip/hip_runtime.h>

#include "dev_cull.h"
#include "dev_util.h"
#include "fdgs_internal.h"

namespace fdgs {
namespace {

constexpr int kNT = 256;
constexpr int kNW = kNT / 64;
constexpr int kRadix = 256;

__device__ __forceinline__ int64_t count_of(const int64_t *n_dev, int64_t n_max) {
    return n_dev ? min(*n_dev, n_max) : n_max;
}

// Lanes of the wave whose `bits`-bit digit equals this lane's, among the
// lanes where `valid` holds: one ballot per digit bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, bool valid) {
    uint64_t match = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        match &= bit ? bb : ~bb;
    }
    return match;
}

// Per-block digit histogram, stored digit-major: hist[d * nb + b].  Block b
// owns keys [b * KPT * kNT, (b + 1) * KPT * kNT).  All loads are issued
// before the first use (indices clamped to the last counted key, so no branch
// separates them).  Counting is by LDS atomics: a round of 64 keys whose
// digits are all equal (common for skewed digits: the exponent byte of
// depths, the high bits of tile ids) adds its count with one atomic, any other
// round one atomic per key (distinct digits proceed in parallel, equal ones
// serialise only among themselves).
template <int KPT>
__global__ void __launch_bounds__(kNT) upsweep_kernel(const uint32_t *keys, const int64_t *n_dev,
                                                      int64_t n_max, int shift, int bits, uint32_t *hist) {
    __shared__ uint32_t h[kRadix];
    const int64_t n = count_of(n_dev, n_max);
    const uint32_t mask = (1u << bits) - 1u;
    h[threadIdx.x] = 0;
    const int64_t c = xcd_item(blockIdx.x, gridDim.x);      // chunk of this block
    const int64_t base = c * (KPT * kNT) + (int64_t)wave_id() * (KPT * 64) + lane_id();
    uint32_t k[KPT];
    if (base < n) {
#pragma unroll
        for (int r = 0; r < KPT; ++r) k[r] = keys[min(base + (int64_t)r * 64, n - 1)];
    } else {
#pragma unroll
        for (int r = 0; r < KPT; ++r) k[r] = 0u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        // the valid lanes of a round are a prefix of the wave (lane 0 first)
        const bool valid = base + (int64_t)r * 64 < n;
        const uint32_t d = (k[r] >> shift) & mask;
        const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
        const uint64_t vm = __ballot(valid);
        const uint64_t same = __ballot(valid && d == d0);
        if (same == vm) {
            if (lane_id() == 0 && vm != 0ull) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * gridDim.x + c] = h[threadIdx.x];   // rows of used digits
}

// One block per digit: exclusive scan of that digit's per-block counts,
// total into digit_total[d].
__global__ void __launch_bounds__(1024) rowscan_kernel(uint32_t *hist, int64_t nb,
                                                       uint32_t *digit_total) {
    __shared__ uint32_t tmp[1024 / 64 + 1];
    uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    uint32_t carry = 0;
    for (int64_t start = 0; start < nb; start += 1024) {
        const int64_t j = start + threadIdx.x;
        const uint32_t v = j < nb ? row[j] : 0;
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum<1024>(v, tmp, &tot);
        if (j < nb) row[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// The same scan for long rows (more than kRowLongAbove blocks, such as the
// tile sort of an unfiltered frame).  A round covers up to kRowIpt counts per
// thread: the counts are loaded coalesced into LDS, each thread scans its
// kRowIpt consecutive ones (LDS rows padded by one word in 32, so that the
// strided reads hit distinct banks), and the results leave through LDS as
// coalesced stores; rows of up to 16384 blocks take one round (the scan above walks them
// in 1024-count rounds, one global latency each).  Short rows stay with the
// scan above: with frames pipelined over streams, this kernel's extra
// barriers cost more than its rounds save (measured 8589 against 7891
// headline frames/s on four streams).  The LDS is sized to the counts a round
// takes (row_scan_lds_bytes).
constexpr int kRowIpt = 16;
constexpr int64_t kRowLongAbove = 4096;
__device__ __forceinline__ int row_pad(int j) { return j + (j >> 5); }
inline int row_scan_per(int64_t nb) { return (int)std::min<int64_t>(kRowIpt, (nb + 1023) / 1024); }
inline size_t row_scan_lds_bytes(int64_t nb) {
    const int span = 1024 * std::max(row_scan_per(nb), 1);
    return sizeof(uint32_t) * (size_t)(span + span / 32);
}
__global__ void __launch_bounds__(1024) rowscan_long_kernel(uint32_t *hist, int64_t nb,
                                                       uint32_t *digit_total) {
    __shared__ uint32_t tmp[1024 / 64 + 1];
    extern __shared__ uint32_t s_v[];   // row_scan_lds_bytes(nb)
    uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    const int per = (int)min((int64_t)kRowIpt, (nb + 1023) / 1024);   // counts per thread and round (>= 1)
    const int t = (int)threadIdx.x;
    uint32_t carry = 0;
    for (int64_t start = 0; start < nb; start += 1024 * per) {
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int j = i * 1024 + t;
            if (i < per) s_v[row_pad(j)] = start + j < nb ? row[start + j] : 0u;
        }
        __syncthreads();
        uint32_t v[kRowIpt];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            v[i] = i < per ? s_v[row_pad(t * per + i)] : 0u;
            sum += v[i];
        }
        uint32_t tot;
        uint32_t ex = carry + block_exclusive_sum<1024>(sum, tmp, &tot);
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            if (i < per) s_v[row_pad(t * per + i)] = ex;
            ex += v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kRowIpt; ++i) {
            const int j = i * 1024 + t;
            if (i < per && start + j < nb) row[start + j] = s_v[row_pad(j)];
        }
        __syncthreads();
        carry += tot;
    }
    if (t == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter of one block's KPT * kNT keys.  Wave w owns the contiguous
// slice [w * KPT * 64, (w + 1) * KPT * 64) of the block's keys and ranks it
// alone: per round of 64 keys, lanes with equal digits are found with one
// ballot per digit bit, and a per-wave running count per digit in LDS gives
// each key its rank among the wave's keys with that digit.  One block barrier
// turns the per-wave counts into block-local digit offsets (earlier waves
// first); the keys are reordered by digit in LDS and then written out by
// consecutive threads, so each digit's run leaves the block as contiguous,
// coalesced stores.  Keys keep their order within a digit: the sort is stable.
template <int KPT>
__global__ void __launch_bounds__(kNT) downsweep_kernel(const uint32_t *keys, const uint32_t *vals,
                                                        uint32_t *keys_out, uint32_t *vals_out,
                                                        const int64_t *n_dev, int64_t n_max,
                                                        int shift, int bits, const uint32_t *hist,
                                                        int64_t hist_cols, int hist_ratio,
                                                        const uint32_t *digit_total) {
    constexpr int CH = KPT * kNT;
    __shared__ uint32_t s_cnt[kNW][kRadix];   // per-wave digit counts, then block-local offsets
    __shared__ uint32_t s_gap[kRadix];        // global start minus block-local start, per digit
    __shared__ uint32_t s_key[CH], s_val[CH];
    __shared__ uint32_t s_tmp[kNW + 1];
    const int64_t n = count_of(n_dev, n_max);
    const int lane = lane_id(), w = wave_id();
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kRadix / 64; ++k) s_cnt[w][k * 64 + lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int64_t c = xcd_item(blockIdx.x, gridDim.x);      // chunk of this block
    const int64_t bbase = c * CH;
    const int64_t wbase = bbase + (int64_t)w * (KPT * 64);
    uint32_t key[KPT], val[KPT], rank[KPT];
    // every load first (indices clamped to the last counted key), so that
    // the wave waits for memory once rather than once per round
    if (wbase + lane < n) {
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const int64_t j = min(wbase + (int64_t)r * 64 + lane, n - 1);
            key[r] = keys[j];
            val[r] = vals[j];
        }
    } else {
#pragma unroll
        for (int r = 0; r < KPT; ++r) key[r] = val[r] = 0u;
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const bool valid = wbase + (int64_t)r * 64 + lane < n;
        const uint32_t d = (key[r] >> shift) & mask;
        const uint64_t match = match_digit(d, bits, valid);
        const uint32_t before = __popcll(match & lt_mask);
        const uint32_t cnt = __popcll(match);
        const uint32_t run = valid ? s_cnt[w][d] : 0u;
        rank[r] = run + before;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (valid && before == cnt - 1) s_cnt[w][d] = run + cnt;   // last lane of its group
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    const int dd = threadIdx.x;                  // thread dd owns digit dd (rows past mask are not kept)
    const bool used = (uint32_t)dd <= mask;
    uint32_t tot;
    const uint32_t gbase = block_exclusive_sum<kNT>(used ? digit_total[dd] : 0u, s_tmp, &tot) +
                           (used ? hist[(int64_t)dd * hist_cols + c * hist_ratio] : 0u);
    uint32_t dcount = 0;
#pragma unroll
    for (int k = 0; k < kNW; ++k) dcount += s_cnt[k][dd];
    const uint32_t lbase = block_exclusive_sum<kNT>(dcount, s_tmp, &tot);
    s_gap[dd] = gbase - lbase;
    uint32_t run = lbase;
#pragma unroll
    for (int k = 0; k < kNW; ++k) {
        const uint32_t c = s_cnt[k][dd];
        s_cnt[k][dd] = run;
        run += c;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int64_t j = wbase + (int64_t)r * 64 + lane;
        if (j < n) {
            const uint32_t lpos = s_cnt[w][(key[r] >> shift) & mask] + rank[r];
            s_key[lpos] = key[r];
            s_val[lpos] = val[r];
        }
    }
    __syncthreads();
    const int valid_n = (int)min((int64_t)CH, n - bbase);
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int i = r * kNT + threadIdx.x;
        if (i < valid_n) {
            const uint32_t k = s_key[i];
            const uint32_t pos = s_gap[(k >> shift) & mask] + (uint32_t)i;
            keys_out[pos] = k;
            vals_out[pos] = s_val[i];
        }
    }
}

// Visible Gaussians -> (float32 depth bits, position) at their compacted slot.
__global__ void scatter_visible_kernel(const uint8_t *visible, const uint32_t *pos,
                                       const uint64_t *depth_key, const int64_t *n_dev,
                                       int64_t n_max, uint32_t *keys32, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count_of(n_dev, n_max) || !visible[i]) return;
    const double z = __longlong_as_double((long long)depth_key[i]);
    keys32[pos[i]] = __float_as_uint((float)z);   // z > 0: bit order = value order
    vals[pos[i]] = (uint32_t)i;
}

// Runs of equal float32 depth keys: insertion sort by (float64 depth, position).
// Runs longer than kMaxTieRun (many Gaussians at one depth to float32
// precision, which only constructed inputs produce) are left in processing
// order and reported through *flag, bounding the work of one thread.
constexpr int64_t kMaxTieRun = 4096;

__global__ void fix_ties_kernel(uint32_t *keys32, uint32_t *vals, const uint64_t *depth_key,
                                const int64_t *n_dev, int64_t n_max, int32_t *flag) {
    const int64_t n = count_of(n_dev, n_max);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j + 1 >= n) return;
    // the three keys are loaded together
    const uint32_t k = keys32[j], kn = keys32[j + 1], kp = keys32[j > 0 ? j - 1 : j];
    if (kn != k) return;
    if (j > 0 && kp == k) return;                 // not the start of the run
    int64_t e = j + 1;
    while (e < n && e - j <= kMaxTieRun && keys32[e] == k) ++e;
    if (e - j > kMaxTieRun) {
        atomicOr(flag, 2);
        return;
    }
    for (int64_t a = j + 1; a < e; ++a) {
        const uint32_t v = vals[a];
        const uint64_t dv = depth_key[v];
        int64_t b = a - 1;
        while (b >= j) {
            const uint32_t u = vals[b];
            const uint64_t du = depth_key[u];
            if (du < dv || (du == dv && u < v)) break;
            vals[b + 1] = u;
            --b;
        }
        vals[b + 1] = v;
    }
}

// Tile-key emission, balanced by instance.  Block b writes the instances
// [b E, (b + 1) E) (E = 1024 up to 2^21 instances, 2048 above: smaller
// windows give a masked frame's 0.8M instances twice the blocks, 26 -> 21 us,
// while the unfiltered frame's 65M run 1% faster with the larger ones),
// whatever Gaussians they belong to: in depth
// order the nearest, largest footprints come first, so a partition by
// Gaussian would give a few blocks most of the work.  The block finds the
// Gaussian holding its first instance with a 256-ary search of the offsets,
// then walks the Gaussians from there, 256 at a time, until one starts past
// its window.  Their tile rows (every row of each rectangle) are processed 256
// at a time: a thread finds its row's Gaussian by a binary search over the
// rows' prefix in LDS and evaluates the row's tile columns (the evaluation the
// per-Gaussian count used); a block scan of the row counts places the rows'
// instances, which are contiguous, and each thread writes the part of its row
// inside the window to an LDS image of the window.  The window then leaves
// the block as coalesced stores.  Counts and emission use the same float
// arithmetic, so each Gaussian fills exactly its slots; the LDS image is
// pre-filled with a valid (key, id) so that every slot holds one whatever the
// counts hold.
constexpr int kDupNT = 256;
constexpr int64_t kDupSmallUpTo = int64_t(1) << 21;

template <int kDupE>
__global__ void __launch_bounds__(kDupNT) duplicate_kernel(const uint32_t *order, const uint64_t *offsets,
                                                           const int32_t *rect, const Rec2D *rec,
                                                           const uint32_t *view_of, const int64_t *n_vis_dev,
                                                           int64_t n_max, RenderParams rp, uint32_t *tile_keys,
                                                           uint32_t *ids, const int64_t *n_inst_dev,
                                                           int64_t capacity, int32_t *overflow, uint32_t *hist,
                                                           int hist_bits) {
    __shared__ int4 s_rect[kDupNT];
    __shared__ CullEllipse s_ell[kDupNT];
    __shared__ uint32_t s_id[kDupNT], s_base[kDupNT];
    __shared__ uint32_t s_rbase[kDupNT + 1];     // first row of each Gaussian in the batch's row list
    __shared__ uint32_t s_key[kDupE], s_val[kDupE];
    __shared__ uint32_t s_tmp[kDupNT / 64 + 1];
    const int64_t n_vis = count_of(n_vis_dev, n_max);
    const int64_t n_inst_all = *n_inst_dev;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_inst_all > capacity) atomicOr(overflow, 1);
    const int64_t n_inst = min(n_inst_all, capacity);
    const int64_t wdx = xcd_item(blockIdx.x, gridDim.x);    // window of this block
    const int64_t e_lo = wdx * kDupE;
    if (e_lo >= n_inst || n_vis <= 0) {                // uniform
        if (hist && (int)threadIdx.x < (1 << hist_bits)) hist[(int64_t)threadIdx.x * gridDim.x + wdx] = 0u;
        return;                                        // an empty window
    }
    const int64_t e_hi = min(e_lo + (int64_t)kDupE, n_inst);
    const int t = threadIdx.x;

    // largest g < n_vis with offsets[g] <= e_lo: probes at lo + t * step, the
    // predicate holds on a prefix of them
    int64_t lo = 0, hi = n_vis;
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + kDupNT - 1) / kDupNT;
        const int64_t p = lo + (int64_t)t * step;
        const uint32_t pr = (p < hi && offsets[p] <= (uint64_t)e_lo) ? 1u : 0u;
        uint32_t c;
        block_exclusive_sum<kDupNT>(pr, s_tmp, &c);     // c >= 1: offsets[lo] <= e_lo
        const int64_t nlo = lo + (int64_t)(c > 1u ? c - 1u : 0u) * step;
        hi = min(nlo + step, hi);
        lo = nlo;
    }
    const uint32_t fill_id = order[lo];
    for (int i = t; i < kDupE; i += kDupNT) {
        s_key[i] = 0u;
        s_val[i] = fill_id;
    }
    uint64_t carry = offsets[lo];                      // first instance of the batch's first row
    bool done = false;
    for (int64_t g0 = lo; g0 < n_vis && !done; g0 += kDupNT) {
        const int64_t g = g0 + t;
        // rows in the low 20 bits, Gaussians starting before e_hi above them
        uint32_t packed = 0;
        if (g < n_vis && offsets[g] < (uint64_t)e_hi) {
            const uint32_t id = order[g];
            const int4 r = reinterpret_cast<const int4 *>(rect)[id];
            s_rect[t] = r;
            s_ell[t] = cull_ellipse(rec[id], rp);
            s_id[t] = id;
            // tile keys of view v start at v * tiles per view
            s_base[t] = view_of ? view_of[id] * (uint32_t)(rp.tiles_x * rp.tiles_y) : 0u;
            packed = (1u << 20) | (uint32_t)(r.w / rp.tile_h - r.y / rp.tile_h + 1);
        }
        uint32_t tot;
        s_rbase[t] = block_exclusive_sum<kDupNT>(packed, s_tmp, &tot) & 0xfffffu;
        const uint32_t n_rows_total = tot & 0xfffffu;
        const int cnt = (int)(tot >> 20);
        if (t == 0) s_rbase[kDupNT] = n_rows_total;
        __syncthreads();
        for (uint32_t row0 = 0; row0 < n_rows_total; row0 += kDupNT) {
            const uint32_t rho = row0 + (uint32_t)t;
            uint32_t n = 0, key0 = 0, rid = 0;
            if (rho < n_rows_total) {
                int a = 0, b = cnt - 1;                // largest Gaussian with s_rbase <= rho
                while (a < b) {
                    const int mid = (a + b + 1) >> 1;
                    if (s_rbase[mid] <= rho) a = mid; else b = mid - 1;
                }
                const int4 r = s_rect[a];
                const int ty = r.y / rp.tile_h + (int)(rho - s_rbase[a]);
                int c0, c1;
                if (tile_row_span(s_ell[a], r, ty, rp.tile_w, rp.tile_h, &c0, &c1)) {
                    n = (uint32_t)(c1 - c0 + 1);
                    key0 = s_base[a] + (uint32_t)(ty * rp.tiles_x + c0);
                }
                rid = s_id[a];
            }
            uint32_t chunk_total;
            const uint32_t pos = block_exclusive_sum<kDupNT>(n, s_tmp, &chunk_total);
            // this row holds the instances [carry + pos, carry + pos + n)
            const int64_t r0 = (int64_t)carry + pos;
            const int64_t ka = max(r0, e_lo), kb = min(r0 + (int64_t)n, e_hi);
            for (int64_t k = ka; k < kb; ++k) {
                s_key[k - e_lo] = key0 + (uint32_t)(k - r0);
                s_val[k - e_lo] = rid;
            }
            carry += chunk_total;
            if (carry >= (uint64_t)e_hi) {               // uniform: the window is full
                done = true;
                break;
            }
        }
        if (cnt < kDupNT) done = true;
        __syncthreads();                                 // the batch's LDS rows are reused
    }
    __syncthreads();
    const int len = (int)(e_hi - e_lo);
    for (int i = t; i < len; i += kDupNT) {
        tile_keys[e_lo + i] = s_key[i];
        ids[e_lo + i] = s_val[i];
    }
    if (hist) {
        // the window's counts of the tile sort's first digit, written where
        // that sort's upsweep would put them (column = window)
        uint32_t *s_h = s_rbase;                         // kDupNT + 1 >= 256 words, free again
        s_h[t] = 0u;
        __syncthreads();
        const uint32_t dmask = (1u << hist_bits) - 1u;
        for (int i = t; i < len; i += kDupNT) atomicAdd(&s_h[s_key[i] & dmask], 1u);
        __syncthreads();
        if (t < (1 << hist_bits)) hist[(int64_t)t * gridDim.x + wdx] = s_h[t];
    }
}

__global__ void gather_u32_kernel(const uint32_t *src, const uint32_t *idx, uint32_t *dst,
                                  const int64_t *n_dev, int64_t n_max) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count_of(n_dev, n_max)) dst[j] = src[idx[j]];
}

__global__ void count_diff_kernel(const uint32_t *a, const uint32_t *b, int64_t n, unsigned long long *out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool d = j < n && a[j] != b[j];
    const unsigned long long c = __popcll(__ballot(d));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = v;
}

// Tile ranges.  Tile t's list is [lower_bound(t), lower_bound(t + 1)) in the
// sorted keys.  Two equivalent kernels: with lists of a few hundred entries a
// thread per position i in [0, n] looks at the keys on either side of i (-1
// before the first, n_tiles after the last): every tile t with prev < t <=
// next has lower_bound(t) = i, and every tile with prev <= t < next has
// lower_bound(t + 1) = i, so each entry is written by exactly one thread from
// one streaming read of the keys.  With long lists (few tiles, many
// instances) a thread per tile binary-searches its two bounds instead.
__global__ void ranges_boundary_kernel(const uint32_t *keys, const int64_t *n_dev, int64_t n_max, int32_t n_tiles,
                                       uint32_t *ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = count_of(n_dev, n_max);
    if (i > n) return;
    const int64_t prev = i == 0 ? -1 : (int64_t)min(keys[i - 1], (uint32_t)n_tiles);
    const int64_t next = i == n ? (int64_t)n_tiles : (int64_t)min(keys[i], (uint32_t)n_tiles);
    if (prev == next) return;
    for (int64_t t = prev + 1; t <= next && t < n_tiles; ++t) ranges[2 * t] = (uint32_t)i;
    for (int64_t t = max(prev, (int64_t)0); t < next; ++t) ranges[2 * t + 1] = (uint32_t)i;
}

__global__ void ranges_search_kernel(const uint32_t *keys, const int64_t *n_dev, int64_t n_max, int32_t n_tiles,
                                     uint32_t *ranges) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t n = count_of(n_dev, n_max);
    auto lower = [&](uint32_t key) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < key) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    ranges[2 * t] = (uint32_t)lower((uint32_t)t);
    ranges[2 * t + 1] = (uint32_t)lower((uint32_t)t + 1u);
}

__global__ void accumulate_counts_kernel(const int64_t *n_proc_dev, int64_t n_proc, const int64_t *counts,
                                         int64_t capacity, unsigned long long *acc) {
    if (threadIdx.x != 0) return;
    const int64_t p = n_proc_dev ? min(*n_proc_dev, n_proc) : n_proc;
    atomicAdd(acc + 0, (unsigned long long)p);
    atomicAdd(acc + 1, (unsigned long long)counts[0]);
    atomicAdd(acc + 2, (unsigned long long)min(counts[1], capacity));
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

// instances per tile (capacity / tiles) above which ranges come from binary searches
constexpr int64_t kRangesSearchAbove = 2048;

}  // namespace

// Keys per thread: up to 2^21 keys short chunks (1024) so that more blocks run,
// above long ones (4096); either way the chunk is a multiple of the emission
// window, so a tile sort takes its first histogram from the emission.
inline int sort_kpt(int64_t n_max) { return n_max <= (int64_t(1) << 21) ? 4 : 16; }

size_t sort_scratch_bytes(int64_t n_max, int64_t hist_cols) {
    const int64_t chunk = (int64_t)sort_kpt(n_max) * kNT;
    const int64_t nb = std::max((n_max + chunk - 1) / chunk, hist_cols);
    return sizeof(uint32_t) * (size_t)(kRadix * (nb > 0 ? nb : 1) + kRadix);
}

// One digit pass.  hist_given: the digit histogram is already in hist with
// hist_cols columns, hist_cols / nb of them per block of this pass (written by
// the kernel that produced the keys), so the upsweep is skipped.
template <int KPT>
static void sort_pass(const uint32_t *src_k, const uint32_t *src_v, uint32_t *dst_k, uint32_t *dst_v,
                      const int64_t *n_dev, int64_t n_max, int shift, int bits, uint32_t *hist,
                      uint32_t *digit_total, int64_t nb, int64_t hist_cols, hipStream_t s) {
    if (hist_cols == 0) {
        hipLaunchKernelGGL((upsweep_kernel<KPT>), dim3((unsigned)nb), dim3(kNT), 0, s, src_k, n_dev, n_max, shift,
                           bits, hist);
        hist_cols = nb;
    }
    if (hist_cols > kRowLongAbove)
        hipLaunchKernelGGL(rowscan_long_kernel, dim3(1u << bits), dim3(1024), row_scan_lds_bytes(hist_cols), s, hist,
                           hist_cols, digit_total);
    else
        hipLaunchKernelGGL(rowscan_kernel, dim3(1u << bits), dim3(1024), 0, s, hist, hist_cols, digit_total);
    hipLaunchKernelGGL((downsweep_kernel<KPT>), dim3((unsigned)nb), dim3(kNT), 0, s, src_k, src_v, dst_k, dst_v,
                       n_dev, n_max, shift, bits, (const uint32_t *)hist, hist_cols, (int)(hist_cols / nb),
                       (const uint32_t *)digit_total);
}

int radix_chunk(int64_t n_max) { return sort_kpt(n_max) * kNT; }

int radix_first_bits(int begin_bit, int end_bit) {
    const int total_bits = end_bit - begin_bit;
    const int passes = (total_bits + 7) / 8;
    return total_bits / passes;
}

hipError_t radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                          const int64_t *n_dev, int64_t n_max, int begin_bit, int end_bit,
                          void *scratch, int *result_in_alt, hipStream_t s, int64_t first_hist_cols) {
    *result_in_alt = 0;
    const int kpt = sort_kpt(n_max);
    const int64_t chunk = (int64_t)kpt * kNT;
    const int64_t nb = (n_max + chunk - 1) / chunk;
    if (nb == 0 || end_bit <= begin_bit) return hipSuccess;
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    uint32_t *digit_total = hist + (size_t)kRadix * std::max(nb, first_hist_cols);
    uint32_t *src_k = keys, *src_v = vals, *dst_k = keys_alt, *dst_v = vals_alt;
    int alt = 0;
    // passes of near-equal width (13 tile bits: 7 + 6): narrower digits leave
    // longer runs per digit in each block's output, so the scatter writes
    // fuller cache lines
    const int total_bits = end_bit - begin_bit;
    const int passes = (total_bits + 7) / 8;
    for (int p = 0, shift = begin_bit; p < passes; ++p) {
        const int bits = (total_bits * (p + 1)) / passes - (total_bits * p) / passes;
        const int64_t given = p == 0 ? first_hist_cols : 0;
        if (kpt == 4)
            sort_pass<4>(src_k, src_v, dst_k, dst_v, n_dev, n_max, shift, bits, hist, digit_total, nb, given, s);
        else if (kpt == 8)
            sort_pass<8>(src_k, src_v, dst_k, dst_v, n_dev, n_max, shift, bits, hist, digit_total, nb, given, s);
        else
            sort_pass<16>(src_k, src_v, dst_k, dst_v, n_dev, n_max, shift, bits, hist, digit_total, nb, given, s);
        uint32_t *tk = src_k, *tv = src_v;
        src_k = dst_k; src_v = dst_v; dst_k = tk; dst_v = tv;
        alt ^= 1;
        shift += bits;
    }
    *result_in_alt = alt;
    return hipGetLastError();
}

hipError_t launch_scatter_visible(const uint8_t *visible, const uint32_t *pos,
                                  const uint64_t *depth_key, const int64_t *n_dev, int64_t n_max,
                                  uint32_t *keys32, uint32_t *vals, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_visible_kernel, dim3(blocks_for(n_max, 256)), dim3(256), 0, s, visible,
                       pos, depth_key, n_dev, n_max, keys32, vals);
    return hipGetLastError();
}

hipError_t launch_fix_depth_ties(uint32_t *keys32, uint32_t *vals, const uint64_t *depth_key,
                                 const int64_t *n_vis_dev, int64_t n_max, int32_t *flag, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    hipLaunchKernelGGL(fix_ties_kernel, dim3(blocks_for(n_max, 256)), dim3(256), 0, s, keys32, vals,
                       depth_key, n_vis_dev, n_max, flag);
    return hipGetLastError();
}

int duplicate_window(int64_t capacity) { return capacity <= kDupSmallUpTo ? 1024 : 2048; }

hipError_t launch_duplicate(const uint32_t *order, const uint64_t *offsets, const int32_t *rect,
                            const Rec2D *rec, const uint32_t *view_of, const int64_t *n_vis_dev, int64_t n_max,
                            const RenderParams &rp, uint32_t *tile_keys, uint32_t *ids,
                            const int64_t *n_inst_dev, int64_t capacity, int32_t *overflow, uint32_t *hist,
                            int hist_bits, int64_t hist_cols, hipStream_t s) {
    if (n_max == 0) return hipSuccess;
    // with a histogram, one window per column (hist_cols * window >= capacity)
    const int window = duplicate_window(capacity);
    const unsigned grid = hist ? (unsigned)hist_cols : std::max(1u, blocks_for(capacity, window));
    if (window == 1024)
        hipLaunchKernelGGL(duplicate_kernel<1024>, dim3(grid), dim3(kDupNT), 0, s, order, offsets, rect, rec, view_of,
                           n_vis_dev, n_max, rp, tile_keys, ids, n_inst_dev, capacity, overflow, hist, hist_bits);
    else
        hipLaunchKernelGGL(duplicate_kernel<2048>, dim3(grid), dim3(kDupNT), 0, s, order, offsets, rect, rec, view_of,
                           n_vis_dev, n_max, rp, tile_keys, ids, n_inst_dev, capacity, overflow, hist, hist_bits);
    return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, const int64_t *n_dev,
                             int64_t n_max, hipStream_t s) {
    if (n_max > 0)
        hipLaunchKernelGGL(gather_u32_kernel, dim3(blocks_for(n_max, 256)), dim3(256), 0, s, src, idx, dst, n_dev,
                           n_max);
    return hipGetLastError();
}

hipError_t launch_count_diff(const uint32_t *a, const uint32_t *b, int64_t n, unsigned long long *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t *>(out), (int64_t)2, 0u);
    if (n > 0) hipLaunchKernelGGL(count_diff_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_accumulate_counts(const int64_t *n_proc_dev, int64_t n_proc, const int64_t *counts,
                                    int64_t capacity, uint64_t *acc, hipStream_t s) {
    hipLaunchKernelGGL(accumulate_counts_kernel, dim3(1), dim3(64), 0, s, n_proc_dev, n_proc, counts, capacity,
                       reinterpret_cast<unsigned long long *>(acc));
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t *tile_keys, const int64_t *n_inst_dev, int64_t n_max,
                              int32_t n_tiles, uint32_t *ranges, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (n_max > (int64_t)kRangesSearchAbove * n_tiles)
        hipLaunchKernelGGL(ranges_search_kernel, dim3(blocks_for(n_tiles, 256)), dim3(256), 0, s, tile_keys,
                           n_inst_dev, n_max, n_tiles, ranges);
    else
        hipLaunchKernelGGL(ranges_boundary_kernel, dim3(blocks_for(n_max + 1, 256)), dim3(256), 0, s, tile_keys,
                           n_inst_dev, n_max, n_tiles, ranges);
    return hipGetLastError();
}

}  // namespace fdgs
