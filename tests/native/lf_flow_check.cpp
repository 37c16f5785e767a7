// CPU check of the waits of the persistent lagged-Fibonacci LD run (lf_flow.hpp).
//  1. For every producer link and consumer tile of small runs, the waits named by
//     lf_producer_waits / lf_walk_producers are exactly the ones found by brute force over the
//     positions involved.
//  2. The incremental coordinate updates the kernel uses agree with a fresh division.
//  3. A simulation of the whole protocol under random interleavings: producers read their sources
//     (after their waits) and write later, consumers read their numbers; every read must find the
//     position it expects in its ring slot, every value must equal the sequential recurrence, and
//     the run must always be able to progress (no deadlock).
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

#include "../../paper_1003_1123_amd/csrc/lf_flow.hpp"

using namespace rngld;

typedef std::set<std::tuple<int, uint32_t, uint32_t>> WaitSet;  // (0 prod / 1 cons, index, need)

struct Run {
    uint64_t n;
    uint32_t T, ll, sl, R, slice_log2, Gc;
    LfFlowGeom g;
    uint64_t Ptot;
    int64_t slice_of(int64_t P) const { return (P % sl) >> slice_log2; }
    int64_t link_of(int64_t P) const { return P / sl; }
    int64_t step_of(int64_t P) const { return P / static_cast<int64_t>(g.four_n); }
};

static Run make_run(uint64_t n, uint32_t T, uint32_t ll, uint32_t sl, uint32_t R, uint32_t slice_log2, uint32_t Gc) {
    Run r;
    r.n = n;
    r.T = T;
    r.ll = ll;
    r.sl = sl;
    r.R = R;
    r.slice_log2 = slice_log2;
    r.Gc = Gc;
    r.g = lf_flow_geom(n, T, ll, sl, R, slice_log2, Gc);
    r.Ptot = r.g.Ptot;
    return r;
}

// brute-force waits of producer p before writing offsets [o_lo, o_lo + len) of link j
static WaitSet brute_producer(const Run &r, uint32_t p, uint32_t j, uint32_t o_lo, uint32_t len) {
    WaitSet w;
    for (uint32_t o = o_lo; o < o_lo + len; ++o) {
        const int64_t P = static_cast<int64_t>(j) * r.sl + o;
        const int64_t src = P - r.ll;
        if (src >= 0) w.insert({0, static_cast<uint32_t>(r.slice_of(src)), static_cast<uint32_t>(r.link_of(src) + 1)});
        const int64_t Q = P - r.R;  // overwritten
        if (Q >= 0) {
            const uint32_t tile = static_cast<uint32_t>((Q % r.g.four_n) / 256);
            w.insert({1, tile / r.g.Kc, static_cast<uint32_t>(r.step_of(Q)) + 1});
        }
        const int64_t rl = Q + r.ll;  // its long-lag reader
        if (rl >= 0 && rl < static_cast<int64_t>(r.Ptot) && r.slice_of(rl) != p)
            w.insert({0, static_cast<uint32_t>(r.slice_of(rl)), static_cast<uint32_t>(r.link_of(rl) + 1)});
        const int64_t rs = Q + r.sl;  // its short-lag reader, which reads the ring only in link 0
        if (rs >= 0 && rs < static_cast<int64_t>(r.sl) && rs < static_cast<int64_t>(r.Ptot) && r.slice_of(rs) != p)
            w.insert({0, static_cast<uint32_t>(r.slice_of(rs)), 1u});
    }
    return w;
}

static uint32_t slice_len(const Run &r, uint32_t p, uint32_t j) {
    const uint64_t o_lo = static_cast<uint64_t>(p) << r.slice_log2;
    uint64_t o_hi = o_lo + (1ull << r.slice_log2);
    if (o_hi > r.sl) o_hi = r.sl;
    const uint64_t P_lo = static_cast<uint64_t>(j) * r.sl;
    if (P_lo + o_lo >= r.Ptot) return 0;
    if (P_lo + o_hi > r.Ptot) o_hi = r.Ptot - P_lo;
    return static_cast<uint32_t>(o_hi - o_lo);
}

static int check_waits(const Run &r) {
    int bad = 0;
    const LfFlowGeom &g = r.g;
    for (uint32_t p = 0; p < g.n_slices; ++p) {
        const uint32_t o_lo = p << r.slice_log2;
        int64_t sR;
        uint64_t oR;
        lf_consumer_coord0(g, o_lo, r.R, sR, oR);
        for (uint32_t j = 0; j < g.n_links; ++j) {
            // incremental coordinate vs a fresh division
            const int64_t Q = static_cast<int64_t>(j) * r.sl + o_lo - r.R;
            int64_t s_ref = Q / static_cast<int64_t>(g.four_n), o_ref = Q - s_ref * static_cast<int64_t>(g.four_n);
            if (o_ref < 0) {
                o_ref += g.four_n;
                --s_ref;
            }
            if (s_ref != sR || static_cast<uint64_t>(o_ref) != oR) {
                if (bad < 5) std::printf("coordinate mismatch link %u slice %u\n", j, p);
                ++bad;
            }
            const uint32_t len = slice_len(r, p, j);
            if (len) {
                WaitSet got;
                lf_producer_waits(
                    g, p, j, o_lo, len, sR, oR,
                    [&](uint32_t s, uint32_t need) { got.insert({0, s, need}); return true; },
                    [&](uint32_t w, uint32_t need) { got.insert({1, w, need}); return true; });
                if (got != brute_producer(r, p, j, o_lo, len)) {
                    if (bad < 5)
                        std::printf("producer waits differ: n=%llu ll=%u sl=%u R=%u T=%u p=%u link=%u\n",
                                    (unsigned long long)r.n, r.ll, r.sl, r.R, 1u << r.slice_log2, p, j);
                    ++bad;
                }
            }
            lf_consumer_coord_next(g, sR, oR);
        }
    }
    // steady-state templates of waits (a) and (c) plus the consumer walk (b) = all waits
    {
        for (uint32_t p = 0; p < g.n_slices; ++p) {
            const uint32_t o_lo = p << r.slice_log2;
            const uint32_t width = std::min<uint32_t>(1u << r.slice_log2, r.sl - o_lo);
            LfWaitTemplate t;
            lf_wait_template(g, p, o_lo, width, t);
            if (t.n > 6) {
                std::printf("template overflow\n");
                ++bad;
                continue;
            }
            int64_t sR;
            uint64_t oR;
            lf_consumer_coord0(g, o_lo, r.R, sR, oR);
            for (uint32_t j = 0; j < g.n_links; ++j) {
                const uint32_t len = slice_len(r, p, j);
                if (j >= lf_steady_link(g) && len == width) {
                    WaitSet got, ref;
                    for (uint32_t i = 0; i < t.n; ++i) got.insert({0, t.slice[i], static_cast<uint32_t>(static_cast<int64_t>(j) + t.d[i])});
                    lf_walk_consumers(g, sR, oR, len, [&](uint32_t w, uint32_t need) { got.insert({1, w, need}); return true; });
                    lf_producer_waits(
                        g, p, j, o_lo, len, sR, oR,
                        [&](uint32_t s, uint32_t need) { ref.insert({0, s, need}); return true; },
                        [&](uint32_t w, uint32_t need) { ref.insert({1, w, need}); return true; });
                    if (got != ref) {
                        if (bad < 5) std::printf("template waits differ: ll=%u sl=%u R=%u p=%u link=%u\n", r.ll, r.sl, r.R, p, j);
                        ++bad;
                    }
                }
                lf_consumer_coord_next(g, sR, oR);
            }
        }
    }
    // consumer tiles
    for (uint32_t c = 0; c < g.n_ctiles; ++c) {
        const uint64_t count = (c + 1) * 64ull <= r.n ? 64 : r.n - 64ull * c;
        int64_t link = static_cast<int64_t>((256ull * c) / r.sl);
        uint32_t off = static_cast<uint32_t>((256ull * c) % r.sl);
        for (uint32_t s = 0; s < r.T; ++s) {
            const uint64_t P0 = s * g.four_n + 256ull * c;
            if (link != static_cast<int64_t>(P0 / r.sl) || off != P0 % r.sl) {
                if (bad < 5) std::printf("tile coordinate mismatch\n");
                ++bad;
            }
            WaitSet got, brute;
            lf_walk_producers(g, link, off, static_cast<uint32_t>(4 * count), [&](uint32_t sl_, uint32_t l) {
                got.insert({0, sl_, l + 1});
                return true;
            });
            for (uint64_t P = P0; P < P0 + 4 * count; ++P)
                brute.insert({0, static_cast<uint32_t>(r.slice_of(P)), static_cast<uint32_t>(r.link_of(P) + 1)});
            if (got != brute) {
                if (bad < 5) std::printf("consumer waits differ: tile %u step %u\n", c, s);
                ++bad;
            }
            lf_link_coord_next_step(g, link, off);
        }
    }
    return bad;
}

// ---- protocol simulation ----------------------------------------------------------------------
static uint64_t rng_state = 88172645463325252ull;
static uint32_t rnd(uint32_t m) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return static_cast<uint32_t>(rng_state % m);
}

static int simulate(const Run &r, uint32_t nb, uint32_t slot0) {
    const LfFlowGeom &g = r.g;
    const uint32_t R = r.R;
    // the sequential sequence: positions -ll .. Ptot-1
    std::vector<uint32_t> seq(r.ll + r.Ptot);
    for (uint32_t i = 0; i < r.ll; ++i) seq[i] = 2654435761u * (i + 1) + 12345u;
    for (uint64_t P = 0; P < r.Ptot; ++P) seq[r.ll + P] = seq[r.ll + P - r.ll] + seq[r.ll + P - r.sl];
    auto expect = [&](int64_t P) { return seq[static_cast<size_t>(P + r.ll)]; };
    auto slot = [&](int64_t P) { return static_cast<uint32_t>(((static_cast<int64_t>(slot0) + P) % R + R) % R); };
    std::vector<int64_t> tag(R);
    std::vector<uint32_t> val(R);
    for (int64_t P = -static_cast<int64_t>(R); P < 0; ++P) {
        tag[slot(P)] = P;
        val[slot(P)] = P >= -static_cast<int64_t>(r.ll) ? expect(P) : 0u;
    }
    const uint32_t Gp = g.n_slices, Gc = r.Gc;
    std::vector<uint32_t> prod(Gp, 0), cons(Gc, 0);
    struct Producer {
        uint32_t j = 0;
        int phase = 0;  // 0: waits + loads, 1: stores + publish
        bool init = false;
        std::vector<uint32_t> chain, src;
        int64_t sR = 0;
        uint64_t oR = 0;
    };
    std::vector<Producer> P(Gp);
    for (uint32_t p = 0; p < Gp; ++p) {
        P[p].chain.assign(1u << r.slice_log2, 0);
        P[p].src.assign((1u << r.slice_log2) * nb, 0);
        lf_consumer_coord0(g, p << r.slice_log2, R, P[p].sR, P[p].oR);
    }
    // consumer w: C[w] steps published; H[w] the step whose numbers it has read and not yet
    // published (-1: none).  A consumer reads step C, then either publishes it, or (when the
    // producers of step C+1 have published) first reads step C+1 and then publishes step C.
    std::vector<uint32_t> C(Gc, 0);
    std::vector<int64_t> H(Gc, -1);
    auto wave_range = [&](uint32_t w, uint64_t step, uint64_t &P0, uint64_t &cnt) {  // positions of wave w
        const uint64_t c0 = static_cast<uint64_t>(w) * g.Kc;
        const uint64_t o0 = std::min<uint64_t>(64 * c0, r.n), o1 = std::min<uint64_t>(64 * (c0 + g.Kc), r.n);
        P0 = step * g.four_n + 4 * o0;
        cnt = 4 * (o1 - o0);
    };
    int bad = 0;
    auto read = [&](int64_t pos) {
        const uint32_t s = slot(pos);
        if (tag[s] != pos) {
            if (bad < 5) std::printf("stale read: wanted %lld found %lld\n", (long long)pos, (long long)tag[s]);
            ++bad;
        }
        return val[s];
    };
    for (;;) {
        std::vector<std::pair<int, uint32_t>> ready;
        bool all_done = true;
        for (uint32_t p = 0; p < Gp; ++p) {
            Producer &q = P[p];
            if (q.j >= g.n_links) continue;
            all_done = false;
            if (q.phase == 1) {
                ready.push_back({0, p});
                continue;
            }
            bool ok = true;
            int64_t sR = q.sR;
            uint64_t oR = q.oR;
            for (uint32_t jj = 0; jj < nb && q.j + jj < g.n_links && ok; ++jj) {
                const uint32_t len = slice_len(r, p, q.j + jj);
                if (len)
                    ok = lf_producer_waits(
                        g, p, q.j + jj, p << r.slice_log2, len, sR, oR,
                        [&](uint32_t s, uint32_t need) { return prod[s] >= need; },
                        [&](uint32_t w, uint32_t need) { return cons[w] >= need; });
                lf_consumer_coord_next(g, sR, oR);
            }
            if (ok) ready.push_back({0, p});
        }
        auto published = [&](uint32_t w, uint64_t step) {
            uint64_t P0, cnt;
            wave_range(w, step, P0, cnt);
            if (!cnt) return true;
            return lf_walk_producers(g, static_cast<int64_t>(P0 / r.sl), static_cast<uint32_t>(P0 % r.sl),
                                     static_cast<uint32_t>(cnt),
                                     [&](uint32_t s, uint32_t l) { return prod[s] >= l + 1; });
        };
        for (uint32_t w = 0; w < Gc; ++w) {
            if (C[w] >= r.T) continue;
            all_done = false;
            if (H[w] < 0) {
                if (published(w, C[w])) ready.push_back({1, w});  // read step C
            } else {
                ready.push_back({2, w});  // publish step C
                if (C[w] + 1 < r.T && published(w, C[w] + 1)) ready.push_back({3, w});  // read C+1, publish C
            }
        }
        if (all_done) break;
        if (ready.empty()) {
            std::printf("deadlock: n=%llu ll=%u sl=%u R=%u\n", (unsigned long long)r.n, r.ll, r.sl, R);
            return bad + 1;
        }
        const auto pick = ready[rnd(static_cast<uint32_t>(ready.size()))];
        if (pick.first == 0) {
            Producer &q = P[pick.second];
            const uint32_t p = pick.second, o_lo = p << r.slice_log2, Tsl = 1u << r.slice_log2;
            const uint32_t jn = q.j + nb <= g.n_links ? nb : g.n_links - q.j;
            if (q.phase == 0) {
                if (!q.init) {  // short-lag sources of link 0 come from the ring, once
                    for (uint32_t o = o_lo; o < o_lo + Tsl && o < r.sl; ++o)
                        q.chain[o - o_lo] = read(static_cast<int64_t>(o) - r.sl);
                    q.init = true;
                }
                for (uint32_t jj = 0; jj < jn; ++jj) {
                    const uint32_t len = slice_len(r, p, q.j + jj);
                    for (uint32_t o = o_lo; o < o_lo + len; ++o)
                        q.src[jj * Tsl + (o - o_lo)] = read(static_cast<int64_t>(q.j + jj) * r.sl + o - r.ll);
                }
                q.phase = 1;
            } else {
                for (uint32_t jj = 0; jj < jn; ++jj) {
                    const uint32_t len = slice_len(r, p, q.j + jj);
                    for (uint32_t o = o_lo; o < o_lo + len; ++o) {
                        const int64_t pos = static_cast<int64_t>(q.j + jj) * r.sl + o;
                        uint32_t &ch = q.chain[o - o_lo];
                        ch += q.src[jj * Tsl + (o - o_lo)];
                        if (ch != expect(pos)) {
                            if (bad < 5) std::printf("wrong value at %lld\n", (long long)pos);
                            ++bad;
                        }
                        tag[slot(pos)] = pos;
                        val[slot(pos)] = ch;
                    }
                    lf_consumer_coord_next(g, q.sR, q.oR);
                }
                q.j += jn;
                prod[p] = q.j;
                q.phase = 0;
            }
        } else {
            const uint32_t w = pick.second;
            // a consumer's loads are in flight from their issue until it publishes the step, so
            // each read is checked at both ends
            auto read_step = [&](uint64_t step) {
                uint64_t P0, cnt;
                wave_range(w, step, P0, cnt);
                for (uint64_t pos = P0; pos < P0 + cnt; ++pos)
                    if (read(static_cast<int64_t>(pos)) != expect(static_cast<int64_t>(pos))) {
                        if (bad < 5) std::printf("consumer read a wrong value at %llu\n", (unsigned long long)pos);
                        ++bad;
                    }
            };
            if (pick.first == 1) {
                read_step(C[w]);
                H[w] = C[w];
            } else {
                if (pick.first == 3) read_step(C[w] + 1);
                read_step(C[w]);
                cons[w] = ++C[w];
                H[w] = pick.first == 3 ? static_cast<int64_t>(C[w]) : -1;
            }
        }
    }
    return bad;
}

// The run's own ring (lf_pad_ring, lf_pad_slot): any R = nr sl consecutive positions occupy
// distinct words below nr slp, every link starts on a 64-word boundary, and the address rules of the
// kernels -- producer's own link base and long-lag bases advanced link by link, consumer's step
// window split over two links -- give lf_pad_slot of the position they mean.
static int check_pad_ring(uint32_t ll, uint32_t sl) {
    const LfPadRing pr = lf_pad_ring(ll, sl);
    const uint64_t R = static_cast<uint64_t>(pr.nr) * sl, words = static_cast<uint64_t>(pr.nr) * pr.slp;
    int bad = 0;
    if (R < static_cast<uint64_t>(ll) + sl || pr.slp % 64 || pr.slp < sl) ++bad;
    for (int64_t P0 : {-static_cast<int64_t>(ll), static_cast<int64_t>(0), 3 * static_cast<int64_t>(sl) + 5}) {
        std::vector<char> used(words, 0);
        for (int64_t P = P0; P < P0 + static_cast<int64_t>(R); ++P) {
            const uint32_t w = lf_pad_slot(pr, sl, P);
            if (w >= words || used[w]) {
                ++bad;
                break;
            }
            used[w] = 1;
            if (((P % sl) + sl) % sl == 0 && w % 64) ++bad;
        }
    }
    const uint32_t lla = ll / sl, llb = ll % sl, slp = pr.slp, rw = pr.nr * pr.slp;
    uint32_t base = 0, base_ll = lf_pad_base(pr, -static_cast<int64_t>(lla));
    for (int64_t j = 0; j < 3 * static_cast<int64_t>(pr.nr) + 2; ++j) {
        if (base != lf_pad_base(pr, j)) ++bad;
        const uint32_t bll1 = base_ll >= slp ? base_ll - slp : base_ll + rw - slp;
        for (uint32_t o : {0u, 1u, llb ? llb - 1 : 0u, llb, sl / 2, sl - 1, rnd(sl)}) {
            const uint32_t idx = o >= llb ? base_ll + (o - llb) : bll1 + (o + (sl - llb));
            if (idx != lf_pad_slot(pr, sl, j * static_cast<int64_t>(sl) + o - ll)) ++bad;
            if (base + o != lf_pad_slot(pr, sl, j * static_cast<int64_t>(sl) + o)) ++bad;
        }
        base = base + slp < rw ? base + slp : 0u;
        base_ll = base_ll + slp < rw ? base_ll + slp : 0u;
    }
    // consumer: a step of four_n positions from (link, off), the link base advanced with the link
    for (uint64_t four_n : {static_cast<uint64_t>(4), static_cast<uint64_t>(sl > 8 ? sl - 4 : 5),
                            static_cast<uint64_t>(sl) + 12, static_cast<uint64_t>(7) * sl + 1000}) {
        int64_t link = 0;
        uint32_t off = 0, lbase = lf_pad_base(pr, 0);
        for (int s = 0; s < 40; ++s) {
            const uint32_t nbase = lbase + slp < rw ? lbase + slp : 0u;
            const int64_t P0 = static_cast<int64_t>(s) * static_cast<int64_t>(four_n);
            // q < sl: the kernel takes a step window of at most sl positions (256 Kc <= sl)
            for (uint32_t q : {0u, 1u % sl, std::min(255u, sl - 1), sl - 1, rnd(sl)}) {
                const uint32_t o = off + q;
                const uint32_t idx = o < sl ? lbase + o : nbase + (o - sl);
                if (idx != lf_pad_slot(pr, sl, P0 + q)) ++bad;
            }
            const int64_t before = link;
            const uint64_t o2 = off + four_n;
            link += static_cast<int64_t>(o2 / sl);
            off = static_cast<uint32_t>(o2 % sl);
            lbase += (static_cast<uint32_t>(link - before) % pr.nr) * slp;
            if (lbase >= rw) lbase -= rw;
        }
    }
    if (bad) std::printf("pad ring (%u, %u): %d mismatches\n", ll, sl, bad);
    return bad;
}

int main() {
    int bad = 0;
    for (auto lag : {std::make_pair(7u, 3u), std::make_pair(2281u, 1252u), std::make_pair(9689u, 5502u),
                     std::make_pair(132049u, 54454u), std::make_pair(3021377u, 1010202u)})
        bad += check_pad_ring(lag.first, lag.second);
    const uint32_t lags[][2] = {{7, 3}, {17, 5}, {31, 13}, {100, 33}, {2281, 1252}, {4423, 3004}};
    const uint64_t ns[] = {1, 2, 5, 63, 64, 65, 100, 257, 1000};
    for (auto &lag : lags) {
        const uint32_t ll = lag[0], sl = lag[1];
        const uint32_t nbmax = ll / sl >= 2 ? 2 : 1;
        for (uint32_t nb = 1; nb <= nbmax; ++nb)
            for (uint64_t n : ns)
                for (uint32_t Gc : {1u, 3u, 7u}) {
                    // the smallest ring allowed for nb links per iteration and Kc tiles per consumer
                    // step, and larger ones
                    const uint32_t Kc = static_cast<uint32_t>(((n + 63) / 64 + Gc - 1) / Gc);
                    const uint32_t Rmin = std::max(ll + nb * sl, nb * sl + 256 * Kc - 1);
                    // the smallest rings, larger ones, and the ring of whole links the kernel uses
                    const uint32_t Rpad = lf_pad_ring(ll, sl).nr * sl;
                    for (uint32_t extra : {0u, 1u, 7u, ll + sl, Rpad > Rmin ? Rpad - Rmin : 0u}) {
                        const uint32_t R = Rmin + extra;
                        for (uint32_t sl2 : {0u, 2u, 6u, 8u, 10u}) {
                            if ((1u << sl2) > sl && sl2) continue;
                            const uint32_t T = n > 300 ? 3 : 9;
                            const Run r = make_run(n, T, ll, sl, R, sl2, Gc);
                            if (nb == 1) bad += check_waits(r);
                            if (r.Ptot <= 40000 && n <= 257)
                                for (uint32_t rep = 0; rep < 2; ++rep) bad += simulate(r, nb, rnd(R));
                        }
                    }
                }
    }
    // the configuration-2 shape: Table I's last row, n = 1e6, 1024-offset slices, 3072 consumer waves
    {
        const Run r = make_run(1000000, 2, 3021377, 1010202, lf_pad_ring(3021377, 1010202).nr * 1010202u, 10, 3072);
        bad += check_waits(r);
    }
    std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
    return bad ? 1 : 0;
}
