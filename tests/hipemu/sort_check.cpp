// Host run of the tile binning kernels (paper_2503_16422_amd/csrc/k_sort.hip)
// through the emulation header: tile-key emission by instance windows (with
// and without ellipse culling) and its first-digit histogram, the stable radix
// sort by tile using that histogram, and both tile-range kernels.  Expected
// values come from plain host loops over the same row spans.
#include "hip/hip_runtime.h"
#include "k_sort_host.inc"
#include <cstdio>
#include <random>
#include <string>
using namespace fdgs;

static int fail(const char *what) {
    std::printf("FAIL: %s\n", what);
    return 1;
}

int main(int argc, char **argv) {
    // argument "full": also the trial with an instance capacity above 2^20, where the emission writes
    // the sort's first-digit histogram (257 sort blocks: minutes in the emulation)
    const bool full = argc > 1 && std::string(argv[1]) == "full";
    std::mt19937_64 rng(9);
    auto U = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); };
    for (int trial = full ? 0 : 1; trial < 2; ++trial) {
        const int W = 200, H = 150, tw = 8, th = 8;
        RenderParams rp{};
        rp.tile_w = tw;
        rp.tile_h = th;
        rp.tiles_x = (W + tw - 1) / tw;
        rp.tiles_y = (H + th - 1) / th;
        rp.alpha_min = 1.0f / 255.0f;
        rp.alpha_max = 0.99f;
        rp.t_min = 1e-4f;
        rp.temporal_cull = 1;
        rp.tile_cull = trial == 0;
        rp.vanilla_level = 2.0 * std::log(255.0) * (1 + 1e-4) + 1e-4;
        const int64_t n_vis = trial == 0 ? 700 : 2000;
        std::vector<Rec2D> rec(n_vis);
        std::vector<int32_t> rect(4 * n_vis);
        std::vector<uint32_t> order(n_vis);
        std::vector<uint64_t> cnt(n_vis);
        for (int64_t g = 0; g < n_vis; ++g) {
            const double u = U(-10, W + 10), v = U(-10, H + 10), s = std::exp(U(0.0, 2.5));
            const double a = 1.0 / (s * s * U(0.3, 1.0)), c = 1.0 / (s * s * U(0.3, 1.0)), b = U(-0.8, 0.8) * std::sqrt(a * c);
            const float op = (float)U(0.02, 0.99);
            rec[g].a = float4{(float)u, (float)v, 0.f, 0.f};
            rec[g].b = float4{(float)a, (float)b, (float)c, op};
            rec[g].c = float4{0.5f, 0.5f, 0.5f, (float)U(1, 5)};
            const double q = 2.0 * std::log(op / rp.alpha_min) * (1 + 1e-4) + 1e-4;
            const double det = a * c - b * b, hx = std::sqrt(q * c / det), hy = std::sqrt(q * a / det);
            int x0 = (int)std::ceil(u - hx - 0.5), x1 = (int)std::floor(u + hx - 0.5);
            int y0 = (int)std::ceil(v - hy - 0.5), y1 = (int)std::floor(v + hy - 0.5);
            x0 = std::max(x0, 0); y0 = std::max(y0, 0); x1 = std::min(x1, W - 1); y1 = std::min(y1, H - 1);
            if (x0 > x1 || y0 > y1) { x0 = y0 = 0; x1 = y1 = 0; }      // keep every rect non-empty
            rect[4 * g] = x0; rect[4 * g + 1] = y0; rect[4 * g + 2] = x1; rect[4 * g + 3] = y1;
        }
        for (int64_t g = 0; g < n_vis; ++g) order[g] = (uint32_t)((g * 7919) % n_vis);   // a permutation
        // expected instances: per Gaussian in `order`, its culled tile rows in row-major order
        std::vector<uint32_t> ekey, eid;
        for (int64_t j = 0; j < n_vis; ++j) {
            const uint32_t id = order[j];
            const int4 r{rect[4 * id], rect[4 * id + 1], rect[4 * id + 2], rect[4 * id + 3]};
            const CullEllipse e = cull_ellipse(rec[id], rp);
            const uint64_t before = ekey.size();
            for (int ty = r.y / th; ty <= r.w / th; ++ty) {
                int c0, c1;
                if (!tile_row_span(e, r, ty, tw, th, &c0, &c1)) continue;
                for (int cx = c0; cx <= c1; ++cx) {
                    const uint32_t key = (uint32_t)(ty * rp.tiles_x + cx);
                    ekey.push_back(key);
                    eid.push_back(id);
                }
            }
            cnt[j] = ekey.size() - before;
            if (cnt[j] != count_tiles(e, r, tw, th)) return fail("row spans and tile count disagree");
        }
        std::vector<uint64_t> offsets(n_vis);
        uint64_t run = 0;
        for (int64_t j = 0; j < n_vis; ++j) { offsets[j] = run; run += cnt[j]; }
        const int64_t n_inst = (int64_t)run;
        // a capacity above 2^20 so that the emission writes the first-digit histogram
        const int64_t capacity = trial == 1 ? n_inst : (int64_t(1) << 20) + 4097;
        const int n_tiles = rp.tiles_x * rp.tiles_y;
        int bits = 1;
        while ((1 << bits) < n_tiles) ++bits;
        const int chunk = radix_chunk(capacity);
        const int64_t hist_cols = chunk % duplicate_window(capacity) == 0
                                      ? (capacity + chunk - 1) / chunk * (chunk / duplicate_window(capacity)) : 0;
        std::vector<uint8_t> scratch(sort_scratch_bytes(capacity, hist_cols));
        std::vector<uint32_t> keys(capacity, 0xdeadu), ids(capacity, 0xdeadu), keys2(capacity), ids2(capacity);
        int64_t n_vis_dev = n_vis, n_inst_dev = n_inst;
        int32_t overflow = 0;
        launch_duplicate(order.data(), offsets.data(), rect.data(), rec.data(), nullptr, &n_vis_dev, n_vis, rp,
                         keys.data(), ids.data(), &n_inst_dev, capacity, &overflow,
                         hist_cols ? reinterpret_cast<uint32_t *>(scratch.data()) : nullptr,
                         radix_first_bits(0, bits), hist_cols, nullptr);
        for (int64_t i = 0; i < n_inst; ++i)
            if (keys[i] != ekey[i] || ids[i] != eid[i]) return fail("emitted instances");
        if (overflow) return fail("overflow flag");
        if (hist_cols) {
            const uint32_t *h = reinterpret_cast<const uint32_t *>(scratch.data());
            const int fb = radix_first_bits(0, bits);
            const int E = duplicate_window(capacity);
            std::vector<uint32_t> c(256 * hist_cols, 0);
            for (int64_t i = 0; i < n_inst; ++i) ++c[(keys[i] & ((1u << fb) - 1u)) * hist_cols + i / E];
            for (int64_t x = 0; x < 256 * hist_cols; ++x)
                if (h[x] != c[x]) return fail("first-digit histogram");
        }
        int alt = 0;
        radix_sort_u32(keys.data(), ids.data(), keys2.data(), ids2.data(), &n_inst_dev, capacity, 0, bits,
                       scratch.data(), &alt, nullptr, hist_cols);
        const uint32_t *sk = alt ? keys2.data() : keys.data(), *si = alt ? ids2.data() : ids.data();
        // expected: stable sort of the emission by tile
        std::vector<int64_t> perm(n_inst);
        for (int64_t i = 0; i < n_inst; ++i) perm[i] = i;
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return ekey[a] < ekey[b]; });
        for (int64_t i = 0; i < n_inst; ++i)
            if (sk[i] != ekey[perm[i]] || si[i] != eid[perm[i]]) return fail("stable tile sort");
        std::vector<uint32_t> ranges(2 * n_tiles, 0xffffffffu);
        std::vector<uint32_t> tile_of(sk, sk + n_inst);
        // both range kernels: the boundary scan, and the binary searches (forced by a larger n_max)
        for (int search = 0; search < 2; ++search) {
            std::vector<uint32_t> ranges(2 * n_tiles, 0xffffffffu);
            if (search) {
                std::vector<uint32_t> big(sk, sk + n_inst);
                big.resize((size_t)n_tiles * 2049 + 1, 0xffffffffu);
                int64_t n_big = n_inst;
                launch_tile_ranges(big.data(), &n_big, (int64_t)big.size(), n_tiles, ranges.data(), nullptr);
            } else {
                launch_tile_ranges(sk, &n_inst_dev, capacity, n_tiles, ranges.data(), nullptr);
            }
            for (int t = 0; t < n_tiles; ++t) {
                const uint32_t lo = (uint32_t)(std::lower_bound(tile_of.begin(), tile_of.end(), (uint32_t)t) - tile_of.begin());
                const uint32_t hi =
                    (uint32_t)(std::lower_bound(tile_of.begin(), tile_of.end(), (uint32_t)t + 1) - tile_of.begin());
                if (ranges[2 * t] != lo || ranges[2 * t + 1] != hi) return fail(search ? "searched ranges" : "tile ranges");
            }
        }
        std::printf("trial %d: %lld instances, capacity %lld, histogram columns %lld: ok\n", trial, (long long)n_inst,
                    (long long)capacity, (long long)hist_cols);
    }
    // the digit-row scan on rows longer than one round (several counts per
    // thread and round, and a ragged last round): 3 rows of 40001 blocks
    {
        const int64_t nb = 40001;
        std::vector<uint32_t> hist(3 * nb), want(3 * nb), tot(3);
        for (auto &v : hist) v = (uint32_t)(rng() % 1000);
        for (int d = 0; d < 3; ++d) {
            uint32_t run = 0;
            for (int64_t j = 0; j < nb; ++j) {
                want[d * nb + j] = run;
                run += hist[d * nb + j];
            }
            want.push_back(run);
        }
        hipLaunchKernelGGL(rowscan_long_kernel, dim3(3), dim3(1024), row_scan_lds_bytes(nb), nullptr, hist.data(), nb,
                           tot.data());
        for (int d = 0; d < 3; ++d) {
            for (int64_t j = 0; j < nb; ++j)
                if (hist[d * nb + j] != want[d * nb + j]) return fail("row scan");
            if (tot[d] != want[3 * nb + d]) return fail("row scan total");
        }
        std::printf("row scan of 3 x %lld counts: ok\n", (long long)nb);
    }
    return 0;
}
