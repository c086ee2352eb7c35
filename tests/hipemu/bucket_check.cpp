// Host run of the depth-bucket kernels (paper_2503_16422_amd/csrc/k_bucket.hip)
// through the emulation header: random depths, ties (one bucket larger than an
// LDS sort, so the merge path runs) and a near outlier.  Checks that the output
// is exactly the visible positions ordered by (float64 depth, position).
#include "hip/hip_runtime.h"
#include "k_bucket_host.inc"
#include <cstdio>
#include <random>
using namespace fdgs;
int main() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 9; ++trial) {
        const int64_t n_max = trial < 3 ? 64 : (trial < 6 ? 3000 : 9000);
        std::vector<uint64_t> dk(n_max);
        std::vector<uint8_t> vis(n_max);
        for (int64_t i = 0; i < n_max; ++i) {
            double z = 2.0 + 4.0 * std::uniform_real_distribution<double>(0, 1)(rng);
            if (trial % 3 == 1 && i % 2) z = 3.25;                 // ties
            if (trial % 3 == 2 && i == 5) z = 0.011;                // near outlier
            std::memcpy(&dk[i], &z, 8);
            vis[i] = std::uniform_int_distribution<int>(0, 9)(rng) != 0;
        }
        const uint32_t nb = 1u << bucket_log2_for(n_max);
        std::vector<uint32_t> work(bucket_scratch_words(n_max), 0xdeadbeefu);
        std::vector<uint32_t> keys32, vals;
        uint32_t kmin = ~0u, kmax = 0;
        for (int64_t i = 0; i < n_max; ++i)
            if (vis[i]) {
                double z;
                std::memcpy(&z, &dk[i], 8);
                const uint32_t k = __float_as_uint((float)z);
                keys32.push_back(k);
                vals.push_back((uint32_t)i);
                kmin = std::min(kmin, k);
                kmax = std::max(kmax, k);
            }
        int64_t n_vis = (int64_t)keys32.size();
        keys32.resize(n_max, 0x7f7f7f7fu);
        vals.resize(n_max, 0x7f7f7f7fu);
        for (uint32_t i = 0; i < 2 * nb; ++i) work[i] = 0;        // what the compaction clears
        work[3 * nb + 1] = kmin;                                  // and the key range it finds
        work[3 * nb + 2] = kmax;
        std::vector<uint32_t> alt(n_max, 0x5a5a5a5au), bucketed(n_max, 0x5a5a5a5au), out(n_max, 0xa5a5a5a5u);
        depth_order_buckets(keys32.data(), vals.data(), &n_vis, n_max, dk.data(), work.data(), alt.data(),
                            bucketed.data(), out.data(), nullptr);
        std::vector<uint32_t> ref(vals.begin(), vals.begin() + n_vis);
        std::sort(ref.begin(), ref.end(),
                  [&](uint32_t a, uint32_t b) { return dk[a] < dk[b] || (dk[a] == dk[b] && a < b); });
        int64_t bad = 0;
        for (int64_t j = 0; j < n_vis; ++j) bad += out[j] != ref[j];
        std::printf("trial %d n_max %lld n_vis %lld buckets %u: %lld misplaced\n", trial, (long long)n_max,
                    (long long)n_vis, nb, (long long)bad);
        if (bad) return 1;
    }
    return 0;
}
