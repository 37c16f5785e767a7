// lf_flow.hpp -- tile geometry of the shared lagged-Fibonacci sequence in a fused LD run.
//
// In a run of n oscillators, step s consumes the 4n consecutive positions (s, off), off in [0, 4n),
// oscillator o taking off = 4o .. 4o+3 (Alg. 3, RNS = 4).  A tile is the 4B positions of B
// consecutive oscillators of one step (the last tile of a step may be shorter).  Position (s, off)
// needs the positions sl and ll earlier (Eq. 3); these helpers name the tiles holding them.
// Plain C++ so that the host code and a CPU test can use it as well as the kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define RNGLD_HD __host__ __device__
#else
#define RNGLD_HD
#endif

namespace rngld {

struct LfFlowGeom {
    uint64_t four_n;      // positions per LD step
    uint32_t tile_shift;  // log2(4 B): positions per full tile
    uint32_t n_ctiles;    // tiles per step, ceil(n / B)
    uint64_t a_sl, b_sl;  // sl = a_sl * four_n + b_sl, 0 <= b_sl < four_n
    uint64_t a_ll, b_ll;  // ll likewise
};

struct LfTile {
    int64_t step;  // negative: before the run (already in the ring)
    uint32_t c;    // tile within the step
};

RNGLD_HD inline LfFlowGeom lf_flow_geom(uint64_t n, uint32_t block_log2, uint32_t ll, uint32_t sl) {
    LfFlowGeom g;
    g.four_n = 4 * n;
    g.tile_shift = block_log2 + 2;
    g.n_ctiles = static_cast<uint32_t>((n + (1ull << block_log2) - 1) >> block_log2);
    g.a_sl = sl / g.four_n;
    g.b_sl = sl % g.four_n;
    g.a_ll = ll / g.four_n;
    g.b_ll = ll % g.four_n;
    return g;
}

// tile holding position (s, off) - (a * four_n + b)
RNGLD_HD inline LfTile lf_tile_back(const LfFlowGeom &g, uint32_t s, uint64_t off, uint64_t a, uint64_t b) {
    LfTile t;
    if (off >= b) {
        t.step = static_cast<int64_t>(s) - static_cast<int64_t>(a);
        t.c = static_cast<uint32_t>((off - b) >> g.tile_shift);
    } else {
        t.step = static_cast<int64_t>(s) - static_cast<int64_t>(a) - 1;
        t.c = static_cast<uint32_t>((off + g.four_n - b) >> g.tile_shift);
    }
    return t;
}

RNGLD_HD inline LfTile lf_tile_next(const LfFlowGeom &g, LfTile t) {
    if (t.c + 1 < g.n_ctiles) {
        ++t.c;
    } else {
        t.c = 0;
        ++t.step;
    }
    return t;
}

// Call visit(step, c) for every tile (with step >= 0) holding a position that tile (s, c) of
// `count` oscillators reads, i.e. positions [off0 - lag, off1 - lag) for lag = sl and lag = ll.
// Each range spans at most three tiles (a short last tile can sit between two full ones); the
// loop is bounded accordingly.  Returns false if visit returned false.
template <class Visit>
RNGLD_HD inline bool lf_tile_sources(const LfFlowGeom &g, uint32_t s, uint32_t c, uint32_t count, Visit &&visit) {
    const uint64_t off0 = static_cast<uint64_t>(c) << g.tile_shift;
    const uint64_t off1 = off0 + 4ull * count;  // exclusive
    const uint64_t lags[2][2] = {{g.a_sl, g.b_sl}, {g.a_ll, g.b_ll}};
    for (int l = 0; l < 2; ++l) {
        LfTile t = lf_tile_back(g, s, off0, lags[l][0], lags[l][1]);
        const LfTile last = lf_tile_back(g, s, off1 - 1, lags[l][0], lags[l][1]);
        for (int guard = 0; guard < 4; ++guard) {
            if (t.step >= 0 && !visit(static_cast<uint32_t>(t.step), t.c)) return false;
            if (t.step == last.step && t.c == last.c) break;
            t = lf_tile_next(g, t);
        }
    }
    return true;
}

}  // namespace rngld
