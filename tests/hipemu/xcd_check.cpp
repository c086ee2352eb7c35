// The XCD-aware block -> item map used by the radix passes and the tile-key
// emission: a bijection of [0, n) for every grid size, under which the blocks
// of each XCD (b = x mod 8) take one contiguous, increasing range of items.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "dev_util.h"

using namespace fdgs;

int main() {
    for (int64_t n = 1; n <= 5000; ++n) {
        std::vector<int> seen(n, 0);
        for (int64_t x = 0; x < 8; ++x) {
            int64_t prev = -1;
            for (int64_t b = x; b < n; b += 8) {
                const int64_t i = xcd_item(b, n);
                if (i < 0 || i >= n || seen[i]) {
                    std::printf("n %lld block %lld: item %lld out of range or repeated\n", (long long)n,
                                (long long)b, (long long)i);
                    return 1;
                }
                if (prev >= 0 && i != prev + 1) {
                    std::printf("n %lld: XCD %lld takes a non-contiguous range\n", (long long)n, (long long)x);
                    return 1;
                }
                seen[i] = 1;
                prev = i;
            }
        }
        for (int64_t i = 0; i < n; ++i)
            if (!seen[i]) {
                std::printf("n %lld: item %lld unassigned\n", (long long)n, (long long)i);
                return 1;
            }
    }
    std::printf("xcd_item: bijection with contiguous per-XCD ranges for n = 1..5000\n");
    return 0;
}
