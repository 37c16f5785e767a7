// CPU check of the lagged-Fibonacci tile geometry used by the dataflow LD kernel: for every tile
// of small runs, the tiles lf_tile_sources() names must be exactly the tiles holding the
// positions that the tile's numbers read (p - sl and p - ll), found here by brute force.
#include <cstdio>
#include <set>
#include <utility>

#include "../../paper_1003_1123_amd/csrc/lf_flow.hpp"

using namespace rngld;

static int check(uint64_t n, uint32_t block_log2, uint32_t ll, uint32_t sl, uint32_t steps) {
    const LfFlowGeom g = lf_flow_geom(n, block_log2, ll, sl);
    const uint64_t B = 1ull << block_log2, four_n = 4 * n;
    int bad = 0;
    for (uint32_t s = 0; s < steps; ++s)
        for (uint32_t c = 0; c < g.n_ctiles; ++c) {
            const uint32_t count = static_cast<uint32_t>((c + 1) * B <= n ? B : n - c * B);
            std::set<std::pair<int64_t, uint32_t>> brute, got;
            for (uint64_t off = 4 * c * B; off < 4 * c * B + 4ull * count; ++off) {
                const int64_t p = static_cast<int64_t>(s * four_n + off);
                for (int64_t lag : {static_cast<int64_t>(sl), static_cast<int64_t>(ll)}) {
                    const int64_t q = p - lag;
                    if (q < 0) continue;
                    brute.insert({q / static_cast<int64_t>(four_n),
                                  static_cast<uint32_t>((q % static_cast<int64_t>(four_n)) / (4 * B))});
                }
            }
            lf_tile_sources(g, s, c, count, [&](uint32_t s2, uint32_t c2) {
                got.insert({static_cast<int64_t>(s2), c2});
                return true;
            });
            if (brute != got) {
                if (bad < 5) std::printf("mismatch n=%llu B=%llu ll=%u sl=%u tile (%u,%u)\n", (unsigned long long)n,
                                         (unsigned long long)B, ll, sl, s, c);
                ++bad;
            }
        }
    return bad;
}

int main() {
    int bad = 0;
    const uint32_t lags[][2] = {{7, 3}, {17, 5}, {2281, 1252}, {4423, 3004}, {9689, 5502}};
    const uint64_t ns[] = {1, 2, 3, 5, 31, 64, 65, 100, 255, 256, 257, 1000, 3001};
    for (auto &lag : lags)
        for (uint64_t n : ns)
            for (uint32_t bl : {0u, 2u, 6u, 8u}) bad += check(n, bl, lag[0], lag[1], 8);
    // the configuration-2 shape: ll, sl of Table I's last row, n = 1e6, 256-oscillator tiles
    bad += check(1000000, 8, 3021377, 1010202, 3);
    std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
    return bad ? 1 : 0;
}
