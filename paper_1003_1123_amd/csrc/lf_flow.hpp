// lf_flow.hpp -- who waits for whom in the persistent lagged-Fibonacci LD run.
//
// The run consumes positions P = 0 .. Ptot-1 of the one sequence y_P = y_{P-ll} + y_{P-sl} mod 2^32
// (Eq. 3); LD step s takes positions s 4n .. s 4n + 4n - 1, oscillator o the four from s 4n + 4o
// (Alg. 3 with RNS = 4).  The run is cut into links of sl positions: link j = [j sl, (j+1) sl).
// Every position of link j depends only on links < j, since both lags are >= sl.
//
//  * Producer p owns the slice [p T, min((p+1) T, sl)) of the offsets within every link (T a power
//    of two).  Its short-lag source y_{P-sl} is its own number of the previous link, so only the
//    long-lag source y_{P-ll} is read from the ring.  After storing link j it publishes
//    prod[p] = j + 1 (links done).
//  * Consumer wave w owns the Kc consecutive tiles c = w Kc .. w Kc + Kc - 1 of 64 oscillators
//    (256 positions each) of every step; once all its numbers of step s are loaded it publishes
//    cons[w] = s + 1 (steps done).
//
// A producer handles one link per iteration and publishes after each.  (The CPU checker also
// simulates nb = 2 links per iteration, with the conditions below read with nb sl for sl.)
// A ring slot of R >= ll + sl words holds position P; the producer writing P overwrites P - R.
// The waits that make the run equal to the sequential recurrence, for a producer about to write
// positions P of link j:
//   (a) the producers of the sources P - ll (data dependency);
//   (b) the consumer of P - R (it must have read it);
//   (c) the producer of P - R + ll, which reads P - R as its long-lag source (it is this producer's
//       own earlier link when R = ll + sl);
//   (d) for P - R + sl in link 0: its producer, which reads P - R from the ring once at the start.
// A consumer wave's step waits for the producers of its (at most 256 Kc) positions.
//
// No deadlock, given R >= ll + sl and R >= sl + 256 Kc - 1: every wait of an iteration over link
// j0 is for producers' iterations that end by link j0 (a: sources lie at least sl back; c: the
// readers of P - R lie R - ll >= sl back; d: P - R + sl in link 0 puts P beyond link 0)
// or for a consumer step whose positions lie wholly before link j0 (b: a consumer's positions of a
// step end within 256 Kc - 1 positions of P - R).  A consumer waits only for the producers of its
// own positions and holds nothing while it waits.  So every wait points to earlier work, and with
// all waves resident the run always progresses.
//
// Plain C++, so that the host and a CPU test can use it as well as the kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define RNGLD_HD __host__ __device__
#else
#define RNGLD_HD
#endif

namespace rngld {

// lag = a * sl + b, 0 <= b < sl
struct LfLag {
    uint32_t a, b;
};

struct LfFlowGeom {
    uint64_t Ptot;        // positions of the run, 4 n T
    uint64_t four_n;      // positions per LD step
    uint64_t fourn_q;     // four_n = fourn_q * sl + fourn_r
    uint64_t sl_q;        // sl = sl_q * four_n + sl_r
    uint64_t sl_r;
    uint32_t fourn_r;
    uint32_t sl;          // link length (the short lag)
    uint32_t slice_log2;  // producer slice T = 2^slice_log2 offsets
    uint32_t n_slices;    // ceil(sl / T): producers with work
    uint32_t n_links;     // ceil(Ptot / sl)
    uint32_t n_ctiles;    // consumer tiles (64 oscillators) per step
    uint32_t Gc;          // consumer waves
    uint32_t Kc;          // consecutive tiles per consumer wave per step
    LfLag ll, R, R_ll, R_sl;  // ll, R, R - ll, R - sl
};

RNGLD_HD inline LfLag lf_lag(uint64_t lag, uint32_t sl) {
    LfLag L;
    L.a = static_cast<uint32_t>(lag / sl);
    L.b = static_cast<uint32_t>(lag % sl);
    return L;
}

inline LfFlowGeom lf_flow_geom(uint64_t n, uint32_t n_steps, uint32_t ll, uint32_t sl, uint32_t R,
                               uint32_t slice_log2, uint32_t Gc) {
    // Gc consumer waves, each with ceil(tiles / Gc) tiles per step
    LfFlowGeom g{};
    g.four_n = 4 * n;
    g.Ptot = g.four_n * n_steps;
    g.fourn_q = g.four_n / sl;
    g.fourn_r = static_cast<uint32_t>(g.four_n % sl);
    g.sl_q = g.four_n ? sl / g.four_n : 0;
    g.sl_r = g.four_n ? sl % g.four_n : 0;
    g.sl = sl;
    g.slice_log2 = slice_log2;
    g.n_slices = static_cast<uint32_t>((static_cast<uint64_t>(sl) + (1ull << slice_log2) - 1) >> slice_log2);
    g.n_links = static_cast<uint32_t>((g.Ptot + sl - 1) / sl);
    g.n_ctiles = static_cast<uint32_t>((n + 63) / 64);
    g.Gc = Gc;
    g.Kc = Gc ? (g.n_ctiles + Gc - 1) / Gc : 0;
    g.ll = lf_lag(ll, sl);
    g.R = lf_lag(R, sl);
    g.R_ll = lf_lag(static_cast<uint64_t>(R) - ll, sl);
    g.R_sl = lf_lag(static_cast<uint64_t>(R) - sl, sl);
    return g;
}

// ---- the run's own ring ------------------------------------------------------------------------------
// The persistent run keeps the sequence in a ring of nr links of its own: link L (positions
// [L sl, (L+1) sl) of the run; L < 0 before it) occupies the words [(L mod nr) slp,
// (L mod nr) slp + sl), slp = sl rounded up to 64 words.  Every link, and so every producer slice
// (its offsets start at multiples of 2^slice_log2 >= 256), then starts on a 256-byte boundary and a
// wave's 64 consecutive stores fill whole cache lines.  In position terms the ring holds R = nr sl
// positions: the R of the waits above, with P - R in the same slot as P.
struct LfPadRing {
    uint32_t nr;   // links held
    uint32_t slp;  // words per link
};

// nr = ceil(2 (ll + sl) / sl): twice the reach of the lags, so producers can run ahead
inline LfPadRing lf_pad_ring(uint32_t ll, uint32_t sl) {
    LfPadRing r;
    r.nr = static_cast<uint32_t>((2 * (static_cast<uint64_t>(ll) + sl) + sl - 1) / sl);
    r.slp = (sl + 63u) & ~63u;
    return r;
}

RNGLD_HD inline uint32_t lf_pad_base(const LfPadRing &r, int64_t link) {
    int64_t m = link % static_cast<int64_t>(r.nr);
    if (m < 0) m += r.nr;
    return static_cast<uint32_t>(m) * r.slp;
}

// word of run position P (P < 0: the window before the run)
RNGLD_HD inline uint32_t lf_pad_slot(const LfPadRing &r, uint32_t sl, int64_t P) {
    const int64_t link = P >= 0 ? P / sl : -((-P + sl - 1) / static_cast<int64_t>(sl));
    return lf_pad_base(r, link) + static_cast<uint32_t>(P - link * static_cast<int64_t>(sl));
}

// (link, off) of position (j, o) - lag; link < 0 means before the run
RNGLD_HD inline void lf_back(uint32_t j, uint32_t o, LfLag L, uint32_t sl, int64_t &link, uint32_t &off) {
    if (o >= L.b) {
        link = static_cast<int64_t>(j) - L.a;
        off = o - L.b;
    } else {
        link = static_cast<int64_t>(j) - L.a - 1;
        off = o + (sl - L.b);
    }
}

// visit(slice, link) for every producer slice holding a run position of [(link, off), + len),
// in order; positions before the run or at/after Ptot are skipped.  false if visit returned false.
template <class Visit>
RNGLD_HD inline bool lf_walk_producers(const LfFlowGeom &g, int64_t link, uint32_t off, uint32_t len, Visit &&visit) {
    while (len > 0) {
        const uint32_t slice = off >> g.slice_log2;
        uint32_t end = (slice + 1) << g.slice_log2;
        if (end > g.sl) end = g.sl;
        const uint32_t take = end - off < len ? end - off : len;
        if (link >= 0) {
            if (static_cast<uint64_t>(link) * g.sl + off >= g.Ptot) return true;
            if (!visit(slice, static_cast<uint32_t>(link))) return false;
        }
        len -= take;
        off += take;
        if (off == g.sl) {
            off = 0;
            ++link;
        }
    }
    return true;
}

// visit(wave, need) for every consumer wave holding a run position of [(step, off), + len), where
// off < four_n is the offset within the step and need = step + 1; step < 0 is skipped
template <class Visit>
RNGLD_HD inline bool lf_walk_consumers(const LfFlowGeom &g, int64_t step, uint64_t off, uint32_t len, Visit &&visit) {
    const uint64_t span = 256ull * g.Kc;  // positions of one wave per step
    while (len > 0) {
        const uint64_t wave = off / span;
        uint64_t end = (wave + 1) * span;
        if (end > g.four_n) end = g.four_n;
        const uint32_t take = end - off < len ? static_cast<uint32_t>(end - off) : len;
        if (step >= 0 && !visit(static_cast<uint32_t>(wave), static_cast<uint32_t>(step) + 1)) return false;
        len -= take;
        off += take;
        if (off == g.four_n) {
            off = 0;
            ++step;
        }
    }
    return true;
}

// (step, offset within the step) of position P - R for P = (0, o): a signed floor division, once
RNGLD_HD inline void lf_consumer_coord0(const LfFlowGeom &g, uint32_t o, uint64_t R, int64_t &step, uint64_t &off) {
    const int64_t q = static_cast<int64_t>(o) - static_cast<int64_t>(R);
    const int64_t fn = static_cast<int64_t>(g.four_n);
    int64_t s = q / fn;
    int64_t r = q - s * fn;
    if (r < 0) {
        r += fn;
        --s;
    }
    step = s;
    off = static_cast<uint64_t>(r);
}

// advance a (step, off) coordinate by one link (sl positions)
RNGLD_HD inline void lf_consumer_coord_next(const LfFlowGeom &g, int64_t &step, uint64_t &off) {
    step += static_cast<int64_t>(g.sl_q);
    off += g.sl_r;
    if (off >= g.four_n) {
        off -= g.four_n;
        ++step;
    }
}

// advance a (link, off) coordinate by one LD step (four_n positions)
RNGLD_HD inline void lf_link_coord_next_step(const LfFlowGeom &g, int64_t &link, uint32_t &off) {
    link += static_cast<int64_t>(g.fourn_q);
    const uint64_t o = static_cast<uint64_t>(off) + g.fourn_r;
    if (o >= g.sl) {
        off = static_cast<uint32_t>(o - g.sl);
        ++link;
    } else {
        off = static_cast<uint32_t>(o);
    }
}

// Every wait of producer p before it writes offsets [o_lo, o_lo + len) of link j (cases (a)-(d)
// above).  (step_R, off_R) is the consumer coordinate of (j, o_lo) - R.  prod_wait(slice, need) asks
// for prod[slice] >= need, cons_wait(wave, need) for cons[wave] >= need.
template <class ProdWait, class ConsWait>
RNGLD_HD inline bool lf_producer_waits(const LfFlowGeom &g, uint32_t p, uint32_t j, uint32_t o_lo, uint32_t len,
                                       int64_t step_R, uint64_t off_R, ProdWait &&prod_wait, ConsWait &&cons_wait) {
    int64_t link;
    uint32_t off;
    // (a) sources
    lf_back(j, o_lo, g.ll, g.sl, link, off);
    if (!lf_walk_producers(g, link, off, len, [&](uint32_t s, uint32_t l) { return prod_wait(s, l + 1); }))
        return false;
    // (b) the consumers of the overwritten positions
    if (!lf_walk_consumers(g, step_R, off_R, len, [&](uint32_t w, uint32_t need) { return cons_wait(w, need); }))
        return false;
    // (c) their long-lag readers
    lf_back(j, o_lo, g.R_ll, g.sl, link, off);
    if (!lf_walk_producers(g, link, off, len,
                           [&](uint32_t s, uint32_t l) { return s == p || prod_wait(s, l + 1); }))
        return false;
    // (d) their short-lag readers in link 0
    lf_back(j, o_lo, g.R_sl, g.sl, link, off);
    return lf_walk_producers(g, link, off, len,
                             [&](uint32_t s, uint32_t l) { return l != 0 || s == p || prod_wait(s, 1u); });
}

// From link lf_steady_link(g) on, waits (a) and (c) of a producer repeat from link to link with
// every need one higher, and (d) has none: they are need = j + d for a fixed list of (slice, d).
struct LfWaitTemplate {
    uint32_t n;
    uint32_t slice[6];
    int32_t d[6];
};

RNGLD_HD inline uint32_t lf_steady_link(const LfFlowGeom &g) { return g.R.a + 2; }  // > R / sl + 1

RNGLD_HD inline void lf_wait_template(const LfFlowGeom &g, uint32_t p, uint32_t o_lo, uint32_t len, LfWaitTemplate &t) {
    LfFlowGeom open = g;  // positions of the reference link need not lie inside the run
    open.Ptot = ~0ull;
    const uint32_t j = lf_steady_link(g);
    t.n = 0;
    int64_t link;
    uint32_t off;
    for (int i = 0; i < 6; ++i) {
        t.slice[i] = 0;
        t.d[i] = 0;
    }
    auto rec = [&](uint32_t s, uint32_t l) {
        const int32_t d = static_cast<int32_t>(static_cast<int64_t>(l) + 1 - static_cast<int64_t>(j));
        for (int i = 0; i < 6; ++i)  // constant indices (registers on the GPU)
            if (static_cast<uint32_t>(i) == t.n) {
                t.slice[i] = s;
                t.d[i] = d;
            }
        ++t.n;
        return true;
    };
    lf_back(j, o_lo, g.ll, g.sl, link, off);
    lf_walk_producers(open, link, off, len, rec);
    lf_back(j, o_lo, g.R_ll, g.sl, link, off);
    lf_walk_producers(open, link, off, len, [&](uint32_t s, uint32_t l) { return s == p || rec(s, l); });
}

}  // namespace rngld
