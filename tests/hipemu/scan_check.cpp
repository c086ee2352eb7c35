// Host run of the scans (paper_2503_16422_amd/csrc/k_scan.hip) through the
// emulation header: exclusive scan through a gather (the tile offsets), visible
// compaction with its key range and clearing, and the compaction of active-set
// bits into ascending indices, at sizes from one element to many chunks.
#include "hip/hip_runtime.h"
#include "k_scan_host.inc"
#include <cstdio>
#include <random>
using namespace fdgs;

static int fail(const char *what) {
    std::printf("FAIL: %s\n", what);
    return 1;
}

int main() {
    std::mt19937_64 rng(5);
    const int64_t sizes[] = {1, 2047, 2048, 5000, 70000};
    for (int64_t n_max : sizes) {
        const int64_t n = n_max > 100 ? n_max - 77 : n_max;      // device count below the bound
        std::vector<uint8_t> scratch(scan_scratch_bytes(n_max));
        // offsets: exclusive scan of counts read through a gather
        std::vector<uint32_t> cnt(n_max), gather(n_max);
        for (auto &x : cnt) x = (uint32_t)(rng() % 50);
        for (int64_t i = 0; i < n_max; ++i) gather[i] = (uint32_t)(n_max - 1 - i);
        std::vector<uint64_t> out(n_max, 77);
        int64_t nd = n, total = -1;
        scan_u32_to_u64(cnt.data(), gather.data(), out.data(), &nd, n_max, &total, scratch.data(), nullptr);
        uint64_t run = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (out[i] != run) return fail("exclusive scan");
            run += cnt[gather[i]];
        }
        for (int64_t i = n; i < n_max; ++i)
            if (out[i] != 77) return fail("scan wrote past the count");
        if (total != (int64_t)run) return fail("scan total");
        // visible compaction with the key range and the cleared words
        std::vector<uint8_t> vis(n_max);
        std::vector<uint64_t> dk(n_max);
        for (int64_t i = 0; i < n_max; ++i) {
            vis[i] = rng() % 3 != 0;
            const double z = 1.0 + (double)(rng() % 100000) / 1000.0;
            std::memcpy(&dk[i], &z, 8);
        }
        std::vector<uint32_t> keys(n_max, 9), vals(n_max, 9), asc(n_max, 9), clear(100, 5), range(2, 5);
        int64_t nvis = -1;
        compact_visible(vis.data(), dk.data(), &nd, n_max, &nvis, keys.data(), vals.data(), asc.data(),
                        clear.data(), 100, range.data(), scratch.data(), nullptr);
        int64_t j = 0;
        uint32_t kmin = ~0u, kmax = 0;
        for (int64_t i = 0; i < n; ++i)
            if (vis[i]) {
                double z;
                std::memcpy(&z, &dk[i], 8);
                const uint32_t k = __float_as_uint((float)z);
                if (keys[j] != k || vals[j] != (uint32_t)i || asc[j] != (uint32_t)i) return fail("compaction order");
                kmin = std::min(kmin, k);
                kmax = std::max(kmax, k);
                ++j;
            }
        if (nvis != j) return fail("compaction count");
        if (j > 0 && (range[0] != kmin || range[1] != kmax)) return fail("key range");
        for (uint32_t x : clear)
            if (x) return fail("clear");
        // the same compaction from per-workgroup visible counts (as the preprocess writes them)
        std::vector<uint32_t> vc((n_max + kPreprocessBlock - 1) / kPreprocessBlock, 0);
        for (int64_t i = 0; i < n; ++i) vc[i / kPreprocessBlock] += vis[i] ? 1u : 0u;
        std::vector<uint32_t> keys2(n_max, 9), vals2(n_max, 9), asc2(n_max, 9), clear2(100, 5), range2(2, 5);
        int64_t nvis2 = -1;
        compact_visible(vis.data(), dk.data(), &nd, n_max, &nvis2, keys2.data(), vals2.data(), asc2.data(),
                        clear2.data(), 100, range2.data(), scratch.data(), nullptr, vc.data());
        if (nvis2 != nvis || range2 != range || clear2 != clear) return fail("compaction from workgroup counts");
        for (int64_t i = 0; i < nvis; ++i)
            if (keys2[i] != keys[i] || vals2[i] != vals[i] || asc2[i] != asc[i])
                return fail("compaction order from workgroup counts");
        // active-set bits -> ascending indices
        std::vector<uint32_t> bits((n_max + 31) / 32);
        for (auto &w : bits) w = (uint32_t)rng();
        std::vector<uint32_t> idx(n_max, 0xffffffffu);
        int64_t count = -1;
        compact_bits(bits.data(), n_max, idx.data(), &count, scratch.data(), nullptr);
        int64_t c = 0;
        for (int64_t g = 0; g < n_max; ++g)
            if ((bits[g >> 5] >> (g & 31)) & 1u) {
                if (idx[c] != (uint32_t)g) return fail("bit compaction order");
                ++c;
            }
        if (count != c) return fail("bit compaction count");
        std::printf("n_max %lld: ok\n", (long long)n_max);
    }
    return 0;
}
