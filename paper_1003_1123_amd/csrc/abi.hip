// abi.hip -- host side of the C ABI declared in include/rngld.h: argument validation, buffer
// sizing, workspace layout, kernel launches, hipGraph plans, launch-shape tuning and autotuning.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"


using namespace rngld;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define RNGLD_TRY_HIP(expr)                                                                                   \
    do {                                                                                                      \
        const hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(RNGLD_EHIP, "%s: %s", #expr, hipGetErrorString(e_));                \
    } while (0)

#define RNGLD_TRY(expr)                                                                                       \
    do {                                                                                                      \
        const int rc_ = (expr);                                                                               \
        if (rc_ != RNGLD_OK) return rc_;                                                                      \
    } while (0)

constexpr uint64_t kMaxStreams = 1ull << 38;
constexpr uint32_t kPathDataflow = 1, kPathWaves = 2;  // workspace word 1 after an LF run
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// validated generator configuration
struct Gen {
    int kind = -1;
    uint64_t S = 0;
    uint32_t ll = 0, sl = 0, W = 0, R = 0;
    size_t state_bytes = 0;
    uint32_t rows = 0;  // per-thread state rows
    uint64_t leap = 0;  // LCG cycle division (0: independent seed words)
    size_t pring_off = 0;  // LAGFIB: byte offset of the bare-stream run's padded ring (0: none)
};

int check_cfg(const rngld_cfg *cfg, Gen *g) {
    if (!cfg) return fail(RNGLD_EINVAL, "cfg is NULL");
    g->kind = cfg->kind;
    switch (cfg->kind) {
        case RNGLD_HYBRID_TAUS:
        case RNGLD_RAN2:
        case RNGLD_LCG:
            if (cfg->n_streams > kMaxStreams) return fail(RNGLD_EINVAL, "n_streams %llu too large",
                                                          (unsigned long long)cfg->n_streams);
            g->S = cfg->n_streams;
            g->leap = cfg->kind == RNGLD_LCG ? cfg->lcg_leap : 0;
            g->rows = cfg->kind == RNGLD_HYBRID_TAUS ? 4 : (cfg->kind == RNGLD_RAN2 ? 35 : 1);
            g->state_bytes = static_cast<size_t>(g->S) * g->rows * 4;
            return RNGLD_OK;
        case RNGLD_NO_NOISE:  // no state: any number of oscillators
            g->S = kMaxStreams;
            g->rows = 0;
            g->state_bytes = 0;
            return RNGLD_OK;
        case RNGLD_LAGFIB: {
            const uint32_t ll = cfg->lf_ll, sl = cfg->lf_sl;
            if (sl == 0 || sl >= ll || ll >= (1u << 31))
                return fail(RNGLD_ELAG, "lagged Fibonacci needs 0 < sl < ll < 2^31 (ll=%u, sl=%u)", ll, sl);
            uint32_t W = cfg->lf_wave ? cfg->lf_wave : sl;
            W &= ~3u;
            if (W < 4 || W > sl) return fail(RNGLD_ELAG, "wave width %u must satisfy 4 <= W <= sl = %u", W, sl);
            // default ring 2 (ll + sl) (ll + sl when that reaches 2^30): enough for any wave width and
            // for the persistent LD run with slack between its producers and consumers
            const uint64_t twice = 2 * (static_cast<uint64_t>(ll) + sl);
            const uint64_t R = cfg->lf_ring ? cfg->lf_ring : (twice < (1ull << 30) ? twice : static_cast<uint64_t>(ll) + sl);
            if (R < static_cast<uint64_t>(ll) + W || R >= (1ull << 31))
                return fail(RNGLD_ELAG, "ring length %llu must satisfy ll + W <= R < 2^31", (unsigned long long)R);
            g->ll = ll;
            g->sl = sl;
            g->W = W;
            g->R = static_cast<uint32_t>(R);
            // header, ring, then (128-byte aligned) the bare-stream runs' progress words and, when
            // its addressing allows, (256-byte aligned) the producer/consumer stream's own ring
            const size_t flags = (sizeof(LfHeader) + static_cast<size_t>(R) * 4 + 127) & ~static_cast<size_t>(127);
            g->state_bytes = flags + kLfStreamFlagBytes;
            const LfPadRing pr = lf_pad_ring(ll, sl);
            const uint64_t pr_words = static_cast<uint64_t>(pr.nr) * pr.slp;
            if (sl >= 256 && pr_words < (1ull << 29) && static_cast<uint64_t>(pr.nr) * sl < (1ull << 31)) {
                g->pring_off = (g->state_bytes + 255) & ~static_cast<size_t>(255);
                g->state_bytes = g->pring_off + pr_words * 4;
            }
            return RNGLD_OK;
        }
        default:
            return fail(RNGLD_EINVAL, "unknown generator kind %d", cfg->kind);
    }
}

int check_state(const Gen &g, const void *d_state, size_t state_bytes) {
    if (state_bytes < g.state_bytes)
        return fail(RNGLD_ESIZE, "state buffer %zu bytes < %zu required", state_bytes, g.state_bytes);
    if (!d_state && g.state_bytes) return fail(RNGLD_EINVAL, "state pointer is NULL");
    return RNGLD_OK;
}

LfRing lf_ring(const Gen &g, void *d_state) {
    LfRing L;
    L.hdr = static_cast<const LfHeader *>(d_state);
    L.ring = reinterpret_cast<uint32_t *>(static_cast<LfHeader *>(d_state) + 1);
    L.R = g.R;
    L.ll = g.ll;
    L.sl = g.sl;
    return L;
}

int check_params(const ld_params &p, bool need_kT_positive = false) {
    const float vals[5] = {p.m, p.k, p.gamma, p.kT, p.dt};
    for (float v : vals)
        if (!std::isfinite(v)) return fail(RNGLD_EINVAL, "non-finite LD parameter");
    if (!(p.m > 0) || !(p.gamma > 0) || !(p.k >= 0) || !(p.kT >= 0) || !(p.dt > 0))
        return fail(RNGLD_EINVAL, "LD parameters need m > 0, gamma > 0, k >= 0, kT >= 0, dt > 0");
    if (need_kT_positive && !(p.kT > 0)) return fail(RNGLD_EINVAL, "gradients need kT > 0");
    if (p.scheme != 0 && p.scheme != 1) return fail(RNGLD_EINVAL, "unknown scheme %d", p.scheme);
    return RNGLD_OK;
}

LdCoef make_coef(const ld_params &p) {
    const double m = p.m, k = p.k, g = p.gamma, kT = p.kT, h = p.dt;
    LdCoef q{};
    q.c = static_cast<float>(1.0 - g * h);
    q.kap = static_cast<float>(k * h / m);
    q.sig = static_cast<float>(std::sqrt(2.0 * g * kT * h / m));
    q.h = static_cast<float>(h);
    const double xi = m * g;
    q.odc = static_cast<float>(k * h / xi);
    q.ods = static_cast<float>(std::sqrt(2.0 * kT * h / xi));
    q.scheme = p.scheme;
    return q;
}

// ensembles sorted by offset, inside [0, n_total), pairwise disjoint
int check_ensembles(const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total, bool need_kT_positive = false) {
    if (!h_ens || n_ens == 0) return fail(RNGLD_EINVAL, "need at least one ensemble");
    if (n_ens > 65535) return fail(RNGLD_EINVAL, "at most 65535 ensembles");
    std::vector<std::pair<uint64_t, uint64_t>> spans;
    spans.reserve(n_ens);
    for (uint32_t e = 0; e < n_ens; ++e) {
        const ld_ensemble &E = h_ens[e];
        if (E.offset > n_total || E.n > n_total - E.offset)
            return fail(RNGLD_EINVAL, "ensemble %u [%llu, +%llu) outside n_total %llu", e,
                        (unsigned long long)E.offset, (unsigned long long)E.n, (unsigned long long)n_total);
        RNGLD_TRY(check_params(E.p, need_kT_positive));
        if (E.n) spans.emplace_back(E.offset, E.offset + E.n);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return fail(RNGLD_EINVAL, "ensembles overlap");
    return RNGLD_OK;
}

// ---- tuning -----------------------------------------------------------------------------------------
std::mutex g_tune_mu;
ld_tuning g_tuning[5] = {{256, 1, 0, 0, 0}, {256, 1, 0, 0, 0}, {256, 1, 0, 0, 0}, {256, 1, 0, 0, 0}, {256, 1, 0, 0, 0}};

ld_tuning current_tuning(int kind) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuning[kind];
}

bool valid_tuning(const ld_tuning &t) {
    return (t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512) &&
           (t.osc_per_thread == 1 || t.osc_per_thread == 2) && t.blocks_per_cu <= 64 && t.lf_waves <= 1;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// ---- ld_run plan (host-side description of one call) ------------------------------------------------
// Workspace of ld_run: [status, path words | padding to 256] [EnsDev table] [partials]
// [x(t0), v(t0)].  The layout does not depend on the device.
struct RunLayout {
    std::vector<EnsDev> ens;
    uint32_t n_tiles = 0, P = 0;
    size_t off_ens = 0, off_partials = 0, off_t0 = 0, bytes = 0;
    // LF wave structure
    uint32_t Q = 0, bpp = 0;
    uint64_t Nq = 0;
    // LF persistent run: 64-oscillator tiles, progress words, its own ring (0 bytes: none)
    uint32_t flow_tiles = 0;
    size_t off_flags = 0, off_pring = 0, pring_bytes = 0;
};

int layout_run(const Gen &g, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total, uint32_t n_steps,
               const ld_obs *obs, const ld_tuning &t, RunLayout *L) {
    const uint32_t stride = obs ? obs->stride : 0;
    L->P = stride ? n_steps / stride + 1 : 0;
    L->ens.resize(n_ens);
    if (g.kind == RNGLD_LAGFIB) {
        if (n_ens != 1) return fail(RNGLD_ENOTSUP, "lagged Fibonacci runs one ensemble (one shared sequence)");
        const uint64_t n = h_ens[0].n;
        const uint64_t nmax = g.W / 4;
        L->Q = n ? static_cast<uint32_t>((n + nmax - 1) / nmax) : 0;
        L->Nq = L->Q ? (n + L->Q - 1) / L->Q : 0;
        L->bpp = static_cast<uint32_t>((L->Nq + kLfLdBlock - 1) / kLfLdBlock);
        L->flow_tiles = static_cast<uint32_t>((n + 63) / 64);
        L->n_tiles = std::max(L->Q * L->bpp, L->flow_tiles);  // partial slots for either mode
        EnsDev &E = L->ens[0];
        memset(&E, 0, sizeof(E));
        E.offset = h_ens[0].offset;
        E.n = n;
        E.tile_begin = 0;
        E.n_tiles = L->n_tiles;
        E.coef = make_coef(h_ens[0].p);
    } else {
        const uint64_t tile = static_cast<uint64_t>(t.block) * t.osc_per_thread;
        uint64_t acc = 0;
        for (uint32_t e = 0; e < n_ens; ++e) {
            EnsDev &E = L->ens[e];
            memset(&E, 0, sizeof(E));
            E.offset = h_ens[e].offset;
            E.n = h_ens[e].n;
            E.tile_begin = static_cast<uint32_t>(acc);
            E.n_tiles = static_cast<uint32_t>((E.n + tile - 1) / tile);
            E.coef = make_coef(h_ens[e].p);
            acc += E.n_tiles;
        }
        if (acc >= (1ull << 31)) return fail(RNGLD_EINVAL, "too many tiles");
        L->n_tiles = static_cast<uint32_t>(acc);
    }
    L->off_ens = kAlign;
    L->off_partials = align_up(L->off_ens + sizeof(EnsDev) * n_ens);
    L->off_t0 = align_up(L->off_partials + static_cast<size_t>(L->P) * L->n_tiles * RNGLD_NOBS * sizeof(double));
    L->bytes = L->off_t0 + (stride ? align_up(6 * static_cast<size_t>(n_total) * sizeof(float)) : 0);
    if (g.kind == RNGLD_LAGFIB) {  // producer and consumer progress words, the run's own ring
        L->off_flags = L->bytes;
        L->bytes += align_up(2 * static_cast<size_t>(kLfFlowMaxWaves) * kLfFlagStride * sizeof(uint32_t));
        const LfPadRing pr = lf_pad_ring(g.ll, g.sl);
        const uint64_t words = static_cast<uint64_t>(pr.nr) * pr.slp;
        if (words < (1ull << 30)) {
            L->off_pring = L->bytes;
            L->pring_bytes = align_up(words * sizeof(uint32_t));
            L->bytes += L->pring_bytes;
        }
    }
    return RNGLD_OK;
}

int check_run_args(const Gen &g, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total, uint32_t n_steps,
                   const ld_obs *obs) {
    RNGLD_TRY(check_ensembles(h_ens, n_ens, n_total));
    if (g.kind != RNGLD_LAGFIB && n_total > g.S)
        return fail(RNGLD_ESIZE, "n_total %llu exceeds the state's %llu streams", (unsigned long long)n_total,
                    (unsigned long long)g.S);
    if (obs && obs->stride && obs->t0 > n_steps) return fail(RNGLD_EINVAL, "t0 beyond the run");
    if (n_total > kMaxStreams) return fail(RNGLD_EINVAL, "n_total too large");
    return RNGLD_OK;
}

// enqueue one ld_run call; all arguments validated
bool debug_enabled() {
    static const bool on = [] {
        const char *e = getenv("RNGLD_DEBUG");
        return e && *e && *e != '0';
    }();
    return on;
}

// The persistent producer/consumer LF run, if this run fits it: returns 1 when launched, 0 when the
// wave path must run instead, an RNGLD error otherwise.
int try_lf_flow(const Gen &g, void *d_state, const RunLayout &L, uint32_t n_steps, float *d_x, float *d_v,
                uint64_t n_total, uint32_t stride, uint32_t t0, double *partials, float *t0buf, uint32_t *flags,
                uint32_t *pring, uint32_t *status, hipStream_t st) {
    const EnsDev &E = L.ens[0];
    const uint64_t n = E.n;
    // the run keeps the sequence in a ring of its own (nr links of slp words, each link on a
    // 256-byte boundary); in positions it holds R = nr sl >= 2 (ll + sl), which keeps the readers of
    // what a producer overwrites behind it
    if (n == 0 || g.sl < 256 || L.pring_bytes == 0) return 0;
    const LfPadRing pr = lf_pad_ring(g.ll, g.sl);
    const uint64_t R_run = static_cast<uint64_t>(pr.nr) * g.sl;
    // the kernel addresses the ring with 32-bit byte offsets below 2^31
    if (R_run >= (1ull << 31) || static_cast<uint64_t>(pr.nr) * pr.slp >= (1ull << 29)) return 0;
    const uint64_t Ptot = 4ull * n * n_steps;
    if ((Ptot + g.sl - 1) / g.sl >= (1ull << 31)) return 0;
    const int cus = device_cus();
    if (cus <= 0) return fail(RNGLD_EHIP, "cannot query the compute-unit count");
    const uint32_t wpb = kLfFlowBlock / 64;
    // producer waves per block: slices of at most kLfFlowSliceMax offsets cover a link
    uint32_t np = 1;
    while (np < wpb - 1 && static_cast<uint64_t>(np) * cus * kLfFlowSliceMax < g.sl) ++np;
    if (static_cast<uint64_t>(np) * cus * kLfFlowSliceMax < g.sl) return 0;
    const uint32_t Gp = np * static_cast<uint32_t>(cus), Gc = (wpb - np) * static_cast<uint32_t>(cus);
    if (Gp > kLfFlowMaxWaves || Gc > kLfFlowMaxWaves) return 0;
    uint32_t slice_log2 = 8;  // at least 256 offsets: a consumer tile then spans at most two slices
    while ((static_cast<uint64_t>(Gp) << slice_log2) < g.sl) ++slice_log2;
    const LfFlowGeom geom = lf_flow_geom(n, n_steps, g.ll, g.sl, static_cast<uint32_t>(R_run), slice_log2, Gc);
    uint32_t kc = 0;
    for (uint32_t k : {1u, 2u, 4u, 8u})
        if (geom.Kc <= k) {
            kc = k;
            break;
        }
    if (!kc) return 0;
    // the ring must also hold a consumer step's positions behind the producers (lf_flow.hpp), and a
    // consumer's positions of a step span at most two links
    if (R_run < static_cast<uint64_t>(g.sl) + 256ull * geom.Kc - 1 || 256ull * geom.Kc > g.sl) return 0;
    const size_t lds = static_cast<size_t>(wpb - np) * geom.Kc * 384u * sizeof(float);
    if (lds > 160 * 1024) return 0;
    if (debug_enabled())
        fprintf(stderr, "[rngld] LF persistent run: %d blocks, %u producer + %u consumer waves each, slice %u, "
                        "%u tiles per consumer (kc %u), LDS %zu\n",
                cus, np, wpb - np, 1u << slice_log2, geom.Kc, kc, lds);
    LfFlowArgs a{};
    a.L = lf_ring(g, d_state);
    a.geom = geom;
    a.pring = pring;
    a.pr = pr;
    a.x = d_x + E.offset;
    a.v = d_v + E.offset;
    a.t0buf = t0buf;
    a.partials = partials;
    a.prod = flags;
    a.cons = flags + static_cast<size_t>(kLfFlowMaxWaves) * kLfFlagStride;
    a.status = status;
    a.N = n_total;
    a.n = n;
    a.coef = E.coef;
    a.n_steps = n_steps;
    a.stride = stride;
    a.t0 = t0;
    a.pstride = L.n_tiles;
    a.spin_limit = 1u << 20;
    a.np = np;
    RNGLD_TRY_HIP(launch_lf_pad_in(a.L, pring, pr, st));
    RNGLD_TRY_HIP(launch_fill_u32(a.prod, static_cast<uint64_t>(Gp) * kLfFlagStride, 0u, st));
    RNGLD_TRY_HIP(launch_fill_u32(a.cons, static_cast<uint64_t>(Gc) * kLfFlagStride, 0u, st));
    const hipError_t e = launch_lf_flow(a, static_cast<uint32_t>(cus), kc, static_cast<uint32_t>(lds), st);
    if (debug_enabled()) fprintf(stderr, "[rngld] LF persistent launch: %s\n", hipGetErrorString(e));
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return 0;
    }
    if (e != hipSuccess) return fail(RNGLD_EHIP, "persistent LF launch: %s", hipGetErrorString(e));
    RNGLD_TRY_HIP(launch_lf_pad_out(a.L, pring, pr, Ptot, st));
    return 1;
}

// status_words: where the status and path words go (NULL: the workspace's first eight bytes)
int enqueue_run(const Gen &g, void *d_state, const RunLayout &L, const ld_tuning &t, uint64_t n_total,
                uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs, double *d_obs, void *d_ws,
                hipStream_t st, bool upload, bool allow_flow = true, uint32_t *status_words = nullptr) {
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    EnsDev *d_ens = reinterpret_cast<EnsDev *>(ws + L.off_ens);
    double *partials = reinterpret_cast<double *>(ws + L.off_partials);
    float *t0buf = reinterpret_cast<float *>(ws + L.off_t0);
    uint32_t *status = status_words ? status_words : reinterpret_cast<uint32_t *>(ws);
    const uint32_t stride = obs ? obs->stride : 0, t0 = obs ? obs->t0 : 0;
    RNGLD_TRY_HIP(launch_fill_u32(status, 2, 0u, st));  // status, path

    if (g.kind == RNGLD_LAGFIB && allow_flow && !t.lf_waves) {
        // one persistent launch for the whole run; observables are tiled by 64-oscillator tile
        std::vector<EnsDev> ens = L.ens;
        ens[0].n_tiles = L.flow_tiles;
        RNGLD_TRY_HIP(launch_upload(d_ens, ens.data(), sizeof(EnsDev), st));
        uint32_t *flags = reinterpret_cast<uint32_t *>(ws + L.off_flags);
        const int r = try_lf_flow(g, d_state, L, n_steps, d_x, d_v, n_total, stride, t0, partials,
                                  t0buf + L.ens[0].offset, flags,
                                  reinterpret_cast<uint32_t *>(ws + L.off_pring), status, st);
        if (r < 0) return r;
        if (r == 1) {
            RNGLD_TRY_HIP(launch_fill_u32(status + 1, 1, kPathDataflow, st));
            const uint64_t count = 4ull * ens[0].n * n_steps;
            RNGLD_TRY_HIP(launch_lf_advance(static_cast<LfHeader *>(d_state), count,
                                            static_cast<uint32_t>(count % g.R), st));
            if (L.P)
                RNGLD_TRY_HIP(launch_obs_finalize(partials, L.n_tiles, L.P, d_ens, 1, d_obs, st));
            return RNGLD_OK;
        }
    }
    if (g.kind == RNGLD_LAGFIB) {
        std::vector<EnsDev> ens = L.ens;
        ens[0].n_tiles = L.Q * L.bpp;
        RNGLD_TRY_HIP(launch_upload(d_ens, ens.data(), sizeof(EnsDev), st));
        RNGLD_TRY_HIP(launch_fill_u32(status + 1, 1, kPathWaves, st));
    } else if (upload) {
        RNGLD_TRY_HIP(launch_upload(d_ens, L.ens.data(), sizeof(EnsDev) * L.ens.size(), st));
    }

    if (g.kind == RNGLD_LAGFIB) {
        const EnsDev &E = L.ens[0];
        const uint64_t n = E.n;
        LfLdPhase ph{};
        ph.L = lf_ring(g, d_state);
        ph.N = n_total;
        ph.n_osc = n;
        ph.x = d_x + E.offset;
        ph.v = d_v + E.offset;
        ph.coef = E.coef;
        ph.stride = stride;
        ph.t0 = t0;
        ph.n_tiles = L.n_tiles;
        ph.partials = partials;
        ph.t0buf = t0buf + E.offset;
        for (uint32_t s = 0; s < n_steps; ++s) {
            for (uint32_t q = 0; q < L.Q; ++q) {
                const uint64_t begin = static_cast<uint64_t>(q) * L.Nq;
                ph.osc_begin = begin;
                ph.osc_count = static_cast<uint32_t>(std::min<uint64_t>(L.Nq, n - begin));
                ph.pos_rel = 4ull * n * s + 4ull * begin;
                ph.off_mod = static_cast<uint32_t>(ph.pos_rel % g.R);
                ph.step = s;
                ph.tile_base = q * L.bpp;
                RNGLD_TRY_HIP(launch_lf_ld_phase(ph, st));
            }
        }
        if (stride && n_steps % stride == 0 && L.Q)
            RNGLD_TRY_HIP(launch_lf_observe(ph, L.Q, L.Nq, n_steps / stride, t0 == n_steps, st));
        const uint64_t count = 4ull * n * n_steps;
        RNGLD_TRY_HIP(launch_lf_advance(const_cast<LfHeader *>(ph.L.hdr), count, static_cast<uint32_t>(count % g.R), st));
    } else {
        LdArgs a{};
        a.state = d_state;
        a.S = g.S;
        a.x = d_x;
        a.v = d_v;
        a.NT = n_total;
        a.ens = d_ens;
        a.n_ens = static_cast<uint32_t>(L.ens.size());
        a.n_tiles = L.n_tiles;
        a.n_steps = n_steps;
        a.stride = stride;
        a.t0 = t0;
        a.P = L.P;
        a.partials = partials;
        a.t0buf = t0buf;
        uint32_t grid = L.n_tiles;
        if (t.blocks_per_cu) {
            const int cus = device_cus();
            if (cus <= 0) return fail(RNGLD_EHIP, "cannot query the compute-unit count");
            grid = std::min<uint32_t>(grid, t.blocks_per_cu * static_cast<uint32_t>(cus));
        }
        const uint32_t spl = t.steps_per_launch ? t.steps_per_launch : std::max<uint32_t>(n_steps, 1);
        if (grid > 0) {
            uint32_t b = 0;
            do {
                a.step_begin = b;
                a.step_end = std::min<uint64_t>(static_cast<uint64_t>(b) + spl, n_steps);
                RNGLD_TRY_HIP(launch_ld_run(g.kind, a, t, grid, st));
                b = a.step_end;
            } while (b < n_steps);
        }
    }
    if (L.P) {
        RNGLD_TRY_HIP(launch_obs_finalize(partials, L.n_tiles, L.P, d_ens, static_cast<uint32_t>(L.ens.size()),
                                          d_obs, st));
    }
    return RNGLD_OK;
}

}  // namespace

// =====================================================================================================
// the status word and progress words that a LAGFIB state keeps after its ring (128-byte aligned)
uint32_t *lf_stream_flags(const Gen &g, void *d_state) {
    const uintptr_t p = reinterpret_cast<uintptr_t>(d_state) + sizeof(LfHeader) + static_cast<uintptr_t>(g.R) * 4;
    return reinterpret_cast<uint32_t *>((p + 127) & ~static_cast<uintptr_t>(127));
}

// The persistent producer/consumer run as a bare Gaussian stream: producers
// extend the sequence in the state's padded ring exactly as in the fused LD run, and the consumers,
// kc tiles of 64 virtual oscillators with four positions per step each, write their positions'
// Box-Muller pairs to out.  It covers the first 4 n T positions of the call, n = 64 kc
// times the consumer waves, T = count / (4 n) steps; returns the number of positions launched (0:
// the run does not fit and nothing was enqueued), an RNGLD error below 0.
int64_t try_lf_pc_gauss(const Gen &g, void *d_state, uint32_t *d_out, uint64_t count, hipStream_t st) {
    if (!g.pring_off || (reinterpret_cast<uintptr_t>(d_out) & 15u)) return 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (cs != hipStreamCaptureStatusNone) return 0;
    const LfPadRing pr = lf_pad_ring(g.ll, g.sl);
    const uint64_t R_run = static_cast<uint64_t>(pr.nr) * g.sl;
    const int cus = device_cus();
    if (cus <= 0) return fail(RNGLD_EHIP, "cannot query the compute-unit count");
    const uint32_t wpb = kLfFlowBlock / 64;
    uint32_t np = 1;
    while (np < wpb - 1 && static_cast<uint64_t>(np) * cus * kLfFlowSliceMax < g.sl) ++np;
    if (static_cast<uint64_t>(np) * cus * kLfFlowSliceMax < g.sl) return 0;
    const uint32_t Gp = np * static_cast<uint32_t>(cus), Gc = (wpb - np) * static_cast<uint32_t>(cus);
    if (Gp > kLfFlowMaxWaves || Gc > kLfFlowMaxWaves) return 0;
    // kc tiles of 64 virtual oscillators per consumer wave, as many as leave at least 4 steps: a
    // step then moves 1 KiB per tile and wave, and the per-step waits and publications are
    // amortised over kc tiles
    uint32_t kc = 4;
    while (kc > 1 && count / (4ull * 64 * Gc * kc) < 4) kc /= 2;
    const uint64_t n = 64ull * Gc * kc;
    const uint64_t T = count / (4 * n);
    if (T < 4 || T >= (1ull << 32)) return 0;
    const uint64_t Ptot = 4 * n * T;
    if ((Ptot + g.sl - 1) / g.sl >= (1ull << 31)) return 0;
    uint32_t slice_log2 = 8;
    while ((static_cast<uint64_t>(Gp) << slice_log2) < g.sl) ++slice_log2;
    const LfFlowGeom geom =
        lf_flow_geom(n, static_cast<uint32_t>(T), g.ll, g.sl, static_cast<uint32_t>(R_run), slice_log2, Gc);
    if (geom.Kc != kc || R_run < static_cast<uint64_t>(g.sl) + 256ull * kc - 1 || 256ull * kc > g.sl) return 0;
    LfFlowArgs a{};
    a.L = lf_ring(g, d_state);
    a.geom = geom;
    a.pring = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(d_state) + g.pring_off);
    a.pr = pr;
    uint32_t *flags = lf_stream_flags(g, d_state);
    a.status = flags;
    a.prod = flags + kLfFlagStride;
    a.cons = a.prod + static_cast<size_t>(kLfFlowMaxWaves) * kLfFlagStride;
    a.N = n;
    a.n = n;
    a.n_steps = static_cast<uint32_t>(T);
    a.spin_limit = 1u << 20;
    a.np = np;
    a.out = d_out;
    RNGLD_TRY_HIP(launch_lf_pad_in(a.L, a.pring, pr, st));
    RNGLD_TRY_HIP(launch_fill_u32(flags, 1, 0u, st));
    RNGLD_TRY_HIP(launch_fill_u32(a.prod, static_cast<uint64_t>(Gp) * kLfFlagStride, 0u, st));
    RNGLD_TRY_HIP(launch_fill_u32(a.cons, static_cast<uint64_t>(Gc) * kLfFlagStride, 0u, st));
    const hipError_t e = launch_lf_flow(a, static_cast<uint32_t>(cus), kc, 0, st, kFlowGauss);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return 0;
    }
    if (e != hipSuccess) return fail(RNGLD_EHIP, "persistent LF stream launch: %s", hipGetErrorString(e));
    RNGLD_TRY_HIP(launch_lf_pad_out(a.L, a.pring, pr, Ptot, st));
    RNGLD_TRY_HIP(launch_lf_advance(const_cast<LfHeader *>(a.L.hdr), Ptot, static_cast<uint32_t>(Ptot % g.R), st));
    return static_cast<int64_t>(Ptot);
}

// The persistent bare-stream run for count values, if it fits: 1 when launched, 0 when the wave
// path must run, an RNGLD error otherwise.  Needs links long enough to keep the chip busy.
int try_lf_stream(const Gen &g, void *d_state, uint32_t *d_out, uint64_t count, hipStream_t st) {
    if (g.sl < 4096 || count < 4ull * g.sl) return 0;
    if ((count + g.sl - 1) / g.sl >= (1ull << 31)) return 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (cs != hipStreamCaptureStatusNone) return 0;
    const int cus = device_cus();
    if (cus <= 0) return fail(RNGLD_EHIP, "cannot query the compute-unit count");
    const uint64_t waves = static_cast<uint64_t>(cus) * (kLfFlowBlock / 64);
    uint32_t m = 0, slice_log2 = 0;
    if (waves * 256 >= g.sl) {
        m = 4;
        slice_log2 = 8;
    } else if (waves * 1024 >= g.sl) {
        m = 16;
        slice_log2 = 10;
    } else {
        return 0;
    }
    LfStreamArgs a{};
    a.L = lf_ring(g, d_state);
    a.geom.sl = g.sl;
    a.geom.slice_log2 = slice_log2;
    a.geom.Ptot = count;
    a.out = d_out;
    uint32_t *flags = lf_stream_flags(g, d_state);
    a.status = flags;
    a.prod = flags + kLfFlagStride;
    a.lla = g.ll / g.sl;
    a.llb = g.ll % g.sl;
    a.n_slices = static_cast<uint32_t>((static_cast<uint64_t>(g.sl) + (1u << slice_log2) - 1) >> slice_log2);
    a.n_links = static_cast<uint32_t>((count + g.sl - 1) / g.sl);
    a.spin_limit = 1u << 20;
    if (a.n_slices + 1 > kLfFlowMaxWaves) return 0;
    RNGLD_TRY_HIP(launch_fill_u32(flags, static_cast<uint64_t>(a.n_slices + 1) * kLfFlagStride, 0u, st));
    const hipError_t e = launch_lf_stream(a, static_cast<uint32_t>(cus), m, st);
    if (e == hipErrorCooperativeLaunchTooLarge) {
        (void)hipGetLastError();
        return 0;
    }
    if (e != hipSuccess) return fail(RNGLD_EHIP, "persistent LF stream launch: %s", hipGetErrorString(e));
    return 1;
}

extern "C" {

const char *rngld_last_error(void) { return g_last_error.c_str(); }
int rngld_version(void) { return 1; }

int rngld_state_bytes(const rngld_cfg *cfg, size_t *bytes) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (!bytes) return fail(RNGLD_EINVAL, "bytes is NULL");
    *bytes = g.state_bytes;
    return RNGLD_OK;
}

int rng_init(const rngld_cfg *cfg, void *d_state, size_t state_bytes, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g.kind == RNGLD_NO_NOISE) return RNGLD_OK;
    if (g.kind == RNGLD_LAGFIB) {
        if (cfg->lf_discard > (1ull << 40)) return fail(RNGLD_EINVAL, "lf_discard above 2^40");
        RNGLD_TRY_HIP(launch_lf_seed(d_state, g.ll, g.sl, g.R, g.W, cfg->seed, st));
        const uint64_t D = cfg->lf_discard;
        if (D) {
            // waves of W positions (each wave's sources lie in earlier waves or the window), then the
            // window's newest slot moves D positions on while pos stays 0
            const LfRing L = lf_ring(g, d_state);
            for (uint64_t first = 0; first < D; first += g.W)
                RNGLD_TRY_HIP(launch_lf_discard_phase(L, static_cast<uint32_t>(first % g.R),
                                                      static_cast<uint32_t>(std::min<uint64_t>(g.W, D - first)), st));
            RNGLD_TRY_HIP(launch_lf_advance(static_cast<LfHeader *>(d_state), 0, static_cast<uint32_t>(D % g.R), st));
        }
    } else {
        if (cfg->stream_base > kMaxStreams) return fail(RNGLD_EINVAL, "stream_base too large");
        RNGLD_TRY_HIP(launch_seed(g.kind, d_state, g.S, cfg->seed, cfg->stream_base, 0, g.S, g.leap, st));
    }
    return RNGLD_OK;
}

int rng_init_ensembles(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                       uint32_t n_ens, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (g.kind == RNGLD_LAGFIB) return fail(RNGLD_ENOTSUP, "ensembles need a per-thread generator");
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    if (!h_ens && n_ens) return fail(RNGLD_EINVAL, "ensembles pointer is NULL");
    for (uint32_t e = 0; e < n_ens; ++e)
        if (h_ens[e].offset > g.S || h_ens[e].n > g.S - h_ens[e].offset)
            return fail(RNGLD_ESIZE, "ensemble %u exceeds the state's streams", e);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g.kind == RNGLD_NO_NOISE) return RNGLD_OK;
    for (uint32_t e = 0; e < n_ens; ++e)
        RNGLD_TRY_HIP(launch_seed(g.kind, d_state, g.S, h_ens[e].seed, 0, h_ens[e].offset, h_ens[e].n, g.leap, st));
    return RNGLD_OK;
}

int rng_uniform(const rngld_cfg *cfg, void *d_state, size_t state_bytes, uint64_t per_stream, uint32_t *d_out,
                uint64_t out_len, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (g.kind == RNGLD_NO_NOISE) return fail(RNGLD_ENOTSUP, "the no-noise kind generates no numbers");
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g.kind == RNGLD_LAGFIB) {
        const uint64_t count = per_stream;
        if (count > (1ull << 40)) return fail(RNGLD_EINVAL, "count too large");
        if (out_len < count) return fail(RNGLD_ESIZE, "output holds %llu < %llu values",
                                         (unsigned long long)out_len, (unsigned long long)count);
        if (count == 0) return RNGLD_OK;
        if (!d_out) return fail(RNGLD_EINVAL, "output pointer is NULL");
        const LfRing L = lf_ring(g, d_state);
        const int r = try_lf_stream(g, d_state, d_out, count, st);
        if (r < 0) return r;
        if (r == 0)
            for (uint64_t first = 0; first < count; first += g.W)
                RNGLD_TRY_HIP(launch_lf_uniform_phase(L, d_out, first,
                                                      static_cast<uint32_t>(std::min<uint64_t>(g.W, count - first)), st));
        const uint64_t m = std::min<uint64_t>(count, g.ll);
        RNGLD_TRY_HIP(launch_lf_ring_store(L, d_out, count, static_cast<uint32_t>((count - m) % g.R), st));
        RNGLD_TRY_HIP(launch_lf_advance(const_cast<LfHeader *>(L.hdr), count, static_cast<uint32_t>(count % g.R), st));
        return RNGLD_OK;
    }
    if (per_stream && g.S && per_stream > ~0ull / g.S) return fail(RNGLD_EINVAL, "size overflow");
    const uint64_t need = per_stream * g.S;
    if (out_len < need) return fail(RNGLD_ESIZE, "output holds %llu < %llu values", (unsigned long long)out_len,
                                    (unsigned long long)need);
    if (need == 0) return RNGLD_OK;
    if (!d_out) return fail(RNGLD_EINVAL, "output pointer is NULL");
    RNGLD_TRY_HIP(launch_bulk_uniform(g.kind, d_state, g.S, per_stream, d_out, st));
    return RNGLD_OK;
}

int rng_gaussian(const rngld_cfg *cfg, void *d_state, size_t state_bytes, uint64_t per_stream, float *d_out,
                 uint64_t out_len, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (g.kind == RNGLD_NO_NOISE) return fail(RNGLD_ENOTSUP, "the no-noise kind generates no numbers");
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    if (per_stream % 2) return fail(RNGLD_EINVAL, "Gaussians come in Box-Muller pairs: per_stream must be even");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (g.kind == RNGLD_LAGFIB) {
        const uint64_t count = per_stream;
        if (count > (1ull << 40)) return fail(RNGLD_EINVAL, "count too large");
        if (out_len < count) return fail(RNGLD_ESIZE, "output holds %llu < %llu values",
                                         (unsigned long long)out_len, (unsigned long long)count);
        if (count == 0) return RNGLD_OK;
        if (!d_out) return fail(RNGLD_EINVAL, "output pointer is NULL");
        const LfRing L = lf_ring(g, d_state);
        // long calls: the producer/consumer run (integers in the state's own ring, each Box-Muller
        // pair written once by the consumers) takes the first 4 n T values; the rest continue from
        // there
        uint32_t *words = reinterpret_cast<uint32_t *>(d_out);
        const int64_t done = try_lf_pc_gauss(g, d_state, words, count, st);
        if (done < 0) return static_cast<int>(done);
        if (static_cast<uint64_t>(done) == count) return RNGLD_OK;
        if (done > 0) return rng_gaussian(cfg, d_state, state_bytes, count - done, d_out + done, out_len - done, stream);
        // the persistent stream of integers into the output (the lag table); the ring takes the last
        // ll of them, then every pair is transformed in place
        const int r = try_lf_stream(g, d_state, words, count, st);
        if (r < 0) return r;
        if (r == 1) {
            const uint64_t m = std::min<uint64_t>(count, g.ll);
            RNGLD_TRY_HIP(launch_lf_ring_store(L, words, count, static_cast<uint32_t>((count - m) % g.R), st));
            RNGLD_TRY_HIP(launch_box_muller_inplace(words, count / 2, st));
        } else {
            for (uint64_t first = 0; first < count; first += g.W)
                RNGLD_TRY_HIP(launch_lf_gauss_phase(L, d_out, first, static_cast<uint32_t>(first % g.R),
                                                    static_cast<uint32_t>(std::min<uint64_t>(g.W, count - first)), st));
        }
        RNGLD_TRY_HIP(launch_lf_advance(const_cast<LfHeader *>(L.hdr), count, static_cast<uint32_t>(count % g.R), st));
        return RNGLD_OK;
    }
    if (per_stream && g.S && per_stream > ~0ull / g.S) return fail(RNGLD_EINVAL, "size overflow");
    const uint64_t need = per_stream * g.S;
    if (out_len < need) return fail(RNGLD_ESIZE, "output holds %llu < %llu values", (unsigned long long)out_len,
                                    (unsigned long long)need);
    if (need == 0) return RNGLD_OK;
    if (!d_out) return fail(RNGLD_EINVAL, "output pointer is NULL");
    RNGLD_TRY_HIP(launch_bulk_gaussian(g.kind, d_state, g.S, per_stream, d_out, st));
    return RNGLD_OK;
}

int rng_box_muller(const uint32_t *d_words, uint64_t n_pairs, float *d_out, void *stream) {
    if (n_pairs == 0) return RNGLD_OK;
    if (!d_words || !d_out) return fail(RNGLD_EINVAL, "words or output is NULL");
    if (n_pairs > (1ull << 40)) return fail(RNGLD_EINVAL, "too many pairs");
    RNGLD_TRY_HIP(launch_box_muller(d_words, n_pairs, d_out, static_cast<hipStream_t>(stream)));
    return RNGLD_OK;
}

int ld_step(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_params *p, uint64_t n, float *d_x,
            float *d_v, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    if (!p) return fail(RNGLD_EINVAL, "params is NULL");
    RNGLD_TRY(check_params(*p));
    if (n == 0) return RNGLD_OK;
    if (!d_x || !d_v) return fail(RNGLD_EINVAL, "x or v is NULL");
    if (n > kMaxStreams) return fail(RNGLD_EINVAL, "n too large");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const LdCoef coef = make_coef(*p);
    if (g.kind == RNGLD_LAGFIB) {
        const uint64_t nmax = g.W / 4;
        const uint64_t Q = (n + nmax - 1) / nmax, Nq = (n + Q - 1) / Q;
        LfLdPhase ph{};
        ph.L = lf_ring(g, d_state);
        ph.N = n;
        ph.n_osc = n;
        ph.x = d_x;
        ph.v = d_v;
        ph.coef = coef;
        for (uint64_t q = 0; q < Q; ++q) {
            ph.osc_begin = q * Nq;
            ph.osc_count = static_cast<uint32_t>(std::min<uint64_t>(Nq, n - q * Nq));
            ph.pos_rel = 4ull * q * Nq;
            ph.off_mod = static_cast<uint32_t>(ph.pos_rel % g.R);
            RNGLD_TRY_HIP(launch_lf_ld_phase(ph, st));
        }
        RNGLD_TRY_HIP(launch_lf_advance(const_cast<LfHeader *>(ph.L.hdr), 4ull * n,
                                        static_cast<uint32_t>((4ull * n) % g.R), st));
        return RNGLD_OK;
    }
    if (n > g.S) return fail(RNGLD_ESIZE, "n %llu exceeds the state's %llu streams", (unsigned long long)n,
                             (unsigned long long)g.S);
    if (g.kind == RNGLD_RAN2 && g.S >= (1ull << 32)) return fail(RNGLD_ENOTSUP, "Ran2 step needs S < 2^32");
    RNGLD_TRY_HIP(launch_ld_step(g.kind, d_state, g.S, coef, n, d_x, d_v, st));
    return RNGLD_OK;
}

int ld_workspace_bytes(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                       uint32_t n_steps, const ld_obs *obs, size_t *bytes) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (!bytes) return fail(RNGLD_EINVAL, "bytes is NULL");
    RNGLD_TRY(check_run_args(g, h_ens, n_ens, n_total, n_steps, obs));
    RunLayout L;
    RNGLD_TRY(layout_run(g, h_ens, n_ens, n_total, n_steps, obs, current_tuning(g.kind), &L));
    *bytes = L.bytes;
    return RNGLD_OK;
}

int ld_run(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens, uint32_t n_ens,
           uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs, double *d_obs, void *d_ws,
           size_t ws_bytes, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    RNGLD_TRY(check_run_args(g, h_ens, n_ens, n_total, n_steps, obs));
    const ld_tuning t = current_tuning(g.kind);
    RunLayout L;
    RNGLD_TRY(layout_run(g, h_ens, n_ens, n_total, n_steps, obs, t, &L));
    if (ws_bytes < L.bytes) return fail(RNGLD_ESIZE, "workspace %zu bytes < %zu required", ws_bytes, L.bytes);
    if (!d_ws) return fail(RNGLD_EINVAL, "workspace is NULL");
    if (n_total && (!d_x || !d_v)) return fail(RNGLD_EINVAL, "x or v is NULL");
    if (L.P && !d_obs) return fail(RNGLD_EINVAL, "observables requested but d_obs is NULL");
    return enqueue_run(g, d_state, L, t, n_total, n_steps, d_x, d_v, obs, d_obs, d_ws,
                       static_cast<hipStream_t>(stream), true);
}

}  // extern "C"

// ---- allocation-free ld_run ---------------------------------------------------------------------
// The workspace of ld_run_noalloc: a library-owned device array, one copy on every GPU the library
// runs on, kept until the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: host code uses only the device address that hipGetSymbolAddress returns for the
// current device (scratch_address below), never the array's name.
static __device__ __align__(256) uint8_t scratch[RNGLD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of the current GPU's copy of `scratch`, looked up on the first call on that GPU
int scratch_address(void **out) {
    int dev = -1;
    RNGLD_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RNGLD_ENOTSUP, "device %d: the allocation-free entry point serves devices 0..%d", dev,
                    kMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RNGLD_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RNGLD_OK;
}

}  // namespace

extern "C" {

int ld_run_noalloc(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens, uint32_t n_ens,
                   uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v, const ld_obs *obs, double *d_obs,
                   uint32_t *d_status, void *stream) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    RNGLD_TRY(check_run_args(g, h_ens, n_ens, n_total, n_steps, obs));
    const ld_tuning t = current_tuning(g.kind);
    RunLayout L;
    RNGLD_TRY(layout_run(g, h_ens, n_ens, n_total, n_steps, obs, t, &L));
    if (L.bytes > RNGLD_NOALLOC_SCRATCH_BYTES)
        return fail(RNGLD_ESIZE, "this run needs %zu bytes of workspace, more than the %zu the allocation-free "
                                 "entry point holds; call ld_run with a workspace of ld_workspace_bytes()",
                    L.bytes, static_cast<size_t>(RNGLD_NOALLOC_SCRATCH_BYTES));
    if (n_total && (!d_x || !d_v)) return fail(RNGLD_EINVAL, "x or v is NULL");
    if (L.P && !d_obs) return fail(RNGLD_EINVAL, "observables requested but d_obs is NULL");
    void *ws = nullptr;
    RNGLD_TRY(scratch_address(&ws));
    return enqueue_run(g, d_state, L, t, n_total, n_steps, d_x, d_v, obs, d_obs, ws, static_cast<hipStream_t>(stream),
                       true, true, d_status);
}

int ld_get_tuning(int32_t kind, ld_tuning *out) {
    if (kind < 0 || kind > RNGLD_NO_NOISE) return fail(RNGLD_EINVAL, "unknown generator kind %d", kind);
    if (!out) return fail(RNGLD_EINVAL, "out is NULL");
    *out = current_tuning(kind);
    return RNGLD_OK;
}

int ld_set_tuning(int32_t kind, const ld_tuning *t) {
    if (kind < 0 || kind > RNGLD_NO_NOISE) return fail(RNGLD_EINVAL, "unknown generator kind %d", kind);
    if (!t || !valid_tuning(*t))
        return fail(RNGLD_EINVAL, "tuning needs block in {64,128,256,512}, osc_per_thread in {1,2}, "
                                  "blocks_per_cu <= 64");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuning[kind] = *t;
    return RNGLD_OK;
}

}  // extern "C"

// ---- hipGraph plans ---------------------------------------------------------------------------------
struct rngld_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int ld_plan_create(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                              uint32_t n_ens, uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v,
                              const ld_obs *obs, double *d_obs, void *d_ws, size_t ws_bytes, void *stream,
                              rngld_plan **out) {
    if (!out) return fail(RNGLD_EINVAL, "out is NULL");
    *out = nullptr;
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    RNGLD_TRY(check_run_args(g, h_ens, n_ens, n_total, n_steps, obs));
    const ld_tuning t = current_tuning(g.kind);
    RunLayout L;
    RNGLD_TRY(layout_run(g, h_ens, n_ens, n_total, n_steps, obs, t, &L));
    if (ws_bytes < L.bytes) return fail(RNGLD_ESIZE, "workspace %zu bytes < %zu required", ws_bytes, L.bytes);
    if (!d_ws) return fail(RNGLD_EINVAL, "workspace is NULL");
    if (n_total && (!d_x || !d_v)) return fail(RNGLD_EINVAL, "x or v is NULL");
    if (L.P && !d_obs) return fail(RNGLD_EINVAL, "observables requested but d_obs is NULL");
    hipStream_t user = static_cast<hipStream_t>(stream);
    // the ensemble table is written once, outside the graph, on the caller's stream
    RNGLD_TRY_HIP(launch_upload(static_cast<uint8_t *>(d_ws) + L.off_ens, L.ens.data(), sizeof(EnsDev) * L.ens.size(),
                                user));
    RNGLD_TRY_HIP(hipStreamSynchronize(user));
    hipStream_t cap = nullptr;
    RNGLD_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    rngld_plan *plan = new rngld_plan();
    int rc = RNGLD_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue_run(g, d_state, L, t, n_total, n_steps, d_x, d_v, obs, d_obs, d_ws, cap, false, false);
        const hipError_t e2 = hipStreamEndCapture(cap, &plan->graph);
        if (rc == RNGLD_OK && e2 != hipSuccess) rc = fail(RNGLD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    } else {
        rc = fail(RNGLD_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    if (rc == RNGLD_OK) {
        e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(RNGLD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cap);
    if (rc != RNGLD_OK) {
        if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
        if (plan->graph) (void)hipGraphDestroy(plan->graph);
        delete plan;
        return rc;
    }
    *out = plan;
    return RNGLD_OK;
}

extern "C" int ld_plan_launch(rngld_plan *plan, void *stream) {
    if (!plan || !plan->exec) return fail(RNGLD_EINVAL, "plan is NULL");
    RNGLD_TRY_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return RNGLD_OK;
}

extern "C" int ld_plan_destroy(rngld_plan *plan) {
    if (!plan) return RNGLD_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return RNGLD_OK;
}

// ---- autotuner --------------------------------------------------------------------------------------
namespace {

std::string device_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string s = prop.gcnArchName;
    for (char &c : s)
        if (c == ' ' || c == ':') c = '_';
    return s + "_cu" + std::to_string(prop.multiProcessorCount);
}

// FNV-1a over the workload shape: every ensemble's size and integrator scheme (the launch shape's
// speed depends on the tiles, not on the physical parameters)
uint64_t shape_hash(const ld_ensemble *h_ens, uint32_t n_ens) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xFF;
            h *= 1099511628211ull;
        }
    };
    for (uint32_t e = 0; e < n_ens; ++e) {
        mix(h_ens[e].n);
        mix(static_cast<uint64_t>(h_ens[e].p.scheme));
    }
    return h;
}

// one cache line: "<device> <kind> <n_total> <n_ens> <n_steps> <shape hash> block opt spl bpc"
std::string cache_key(int kind, uint64_t n_total, uint32_t n_ens, uint32_t n_steps, uint64_t hash) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s kind%d n%llu e%u s%u h%016llx", device_name().c_str(), kind,
             static_cast<unsigned long long>(n_total), n_ens, n_steps, static_cast<unsigned long long>(hash));
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, ld_tuning *t) {
    if (!path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        char k[6][128];
        unsigned b, o, s, c;
        if (sscanf(line, "%127s %127s %127s %127s %127s %127s %u %u %u %u", k[0], k[1], k[2], k[3], k[4], k[5], &b, &o,
                   &s, &c) == 10) {
            const std::string lk = std::string(k[0]) + " " + k[1] + " " + k[2] + " " + k[3] + " " + k[4] + " " + k[5];
            ld_tuning cand{b, o, s, c, 0};
            if (lk == key && valid_tuning(cand)) {
                *t = cand;
                found = true;
            }
        }
    }
    fclose(f);
    return found;
}

// rewrite the cache with this key's line replaced (or added); other lines are kept as they are
void cache_store(const char *path, const std::string &key, const ld_tuning &t) {
    if (!path) return;
    std::vector<std::string> keep;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof(line), f)) {
            std::string l(line);
            if (l.compare(0, key.size() + 1, key + " ") != 0) keep.push_back(l);
        }
        fclose(f);
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    for (const std::string &l : keep) fputs(l.c_str(), f);
    fprintf(f, "%s %u %u %u %u\n", key.c_str(), t.block, t.osc_per_thread, t.steps_per_launch, t.blocks_per_cu);
    const bool ok = fclose(f) == 0;
    if (ok) rename(tmp.c_str(), path);
}

struct DeviceScratch {
    std::vector<void *> ptrs;
    void *get(size_t bytes) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
    ~DeviceScratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

// timing resources of one autotune call: a private stream (never the legacy default stream) and two
// events recorded on it
struct TuneTimer {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneTimer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    }
    int init() {
        RNGLD_TRY_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        RNGLD_TRY_HIP(hipEventCreate(&e0));
        RNGLD_TRY_HIP(hipEventCreate(&e1));
        return RNGLD_OK;
    }
    // milliseconds of the work `fn` enqueues on st
    template <class F>
    int time(F &&fn, float *ms) {
        RNGLD_TRY_HIP(hipEventRecord(e0, st));
        RNGLD_TRY(fn());
        RNGLD_TRY_HIP(hipEventRecord(e1, st));
        RNGLD_TRY_HIP(hipEventSynchronize(e1));
        RNGLD_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
        return RNGLD_OK;
    }
};

// capture one run (the shape and chunking of t) into an executable graph on the timer's stream
int capture_run(const Gen &g, void *state, const RunLayout &L, const ld_tuning &t, uint64_t n_total, uint32_t steps,
                float *x, float *v, void *ws, hipGraph_t *graph, hipGraphExec_t *exec) {
    hipStream_t cap = nullptr;
    RNGLD_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    int rc = RNGLD_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue_run(g, state, L, t, n_total, steps, x, v, nullptr, nullptr, ws, cap, false, false);
        const hipError_t e2 = hipStreamEndCapture(cap, graph);
        if (rc == RNGLD_OK && e2 != hipSuccess) rc = fail(RNGLD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
    } else {
        rc = fail(RNGLD_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    if (rc == RNGLD_OK && hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(RNGLD_EHIP, "hipGraphInstantiate failed");
    (void)hipStreamDestroy(cap);
    return rc;
}

}  // namespace

extern "C" int ld_autotune(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                           uint32_t n_steps, const char *cache_path, ld_tuning *out) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (!out) return fail(RNGLD_EINVAL, "out is NULL");
    if (g.kind == RNGLD_LAGFIB) return fail(RNGLD_ENOTSUP, "the lagged-Fibonacci path has no tunable launch shape");
    RNGLD_TRY(check_run_args(g, h_ens, n_ens, n_total, n_steps, nullptr));
    const std::string key = cache_key(g.kind, n_total, n_ens, n_steps, shape_hash(h_ens, n_ens));
    ld_tuning best{};
    if (cache_lookup(cache_path, key, &best)) {
        RNGLD_TRY(ld_set_tuning(g.kind, &best));
        *out = best;
        return RNGLD_OK;
    }
    // proxy runs: the same ensembles on scratch copies of x, v and the state
    DeviceScratch mem;
    const size_t xv_bytes = 3 * static_cast<size_t>(n_total) * sizeof(float);
    float *x = static_cast<float *>(mem.get(xv_bytes));
    float *v = static_cast<float *>(mem.get(xv_bytes));
    rngld_cfg c2 = *cfg;
    c2.n_streams = n_total;
    Gen g2;
    RNGLD_TRY(check_cfg(&c2, &g2));
    void *state = mem.get(g2.state_bytes);
    if (!x || !v || !state) return fail(RNGLD_EHIP, "autotune scratch allocation failed");
    TuneTimer tm;
    RNGLD_TRY(tm.init());
    RNGLD_TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(x), 3 * n_total, 0u, tm.st));
    RNGLD_TRY_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(v), 3 * n_total, 0u, tm.st));
    RNGLD_TRY(rng_init(&c2, state, g2.state_bytes, tm.st));

    // 1) launch shape (block size, oscillators per thread, blocks per CU) on a short proxy, whole run
    //    in one launch; each candidate's first repetition loads its kernel and is not counted
    const uint32_t proxy_steps = std::max<uint32_t>(1, std::min<uint32_t>(n_steps, 128));
    std::vector<ld_tuning> cands;
    for (uint32_t b : {64u, 128u, 256u, 512u})
        for (uint32_t o : {1u, 2u})
            for (uint32_t bpc : {0u, 4u, 8u}) {
                if (g.kind == RNGLD_RAN2 && o * b * kR2Tab * 4 > 64 * 1024) continue;
                cands.push_back({b, o, 0, bpc, 0});
            }
    float best_ms = 1e30f;
    for (const ld_tuning &t : cands) {
        RunLayout L;
        RNGLD_TRY(layout_run(g2, h_ens, n_ens, n_total, proxy_steps, nullptr, t, &L));
        void *ws = mem.get(L.bytes);
        if (!ws) return fail(RNGLD_EHIP, "autotune scratch allocation failed");
        float ms = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {
            float m = 0.0f;
            RNGLD_TRY(tm.time([&] { return enqueue_run(g2, state, L, t, n_total, proxy_steps, x, v, nullptr, nullptr,
                                                       ws, tm.st, true); }, &m));
            if (rep > 0) ms += m;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }

    // 2) steps per launch: each candidate chunking of a longer proxy run (up to 2500 steps, shortened
    //    for very large ensembles), captured in a graph as ld_plan_create records it and replayed;
    //    the fastest replay wins, a single launch on ties within 0.5%
    uint32_t spl_steps = std::min<uint32_t>(n_steps, 2500);
    while (spl_steps > 500 && static_cast<double>(n_total) * spl_steps > 2e11) spl_steps /= 2;
    float spl_best_ms = 1e30f;
    uint32_t spl_best = 0;
    for (uint32_t spl : {0u, 2500u, 1000u, 500u}) {
        if (spl && spl >= spl_steps) continue;
        ld_tuning t = best;
        t.steps_per_launch = spl;
        RunLayout L;
        RNGLD_TRY(layout_run(g2, h_ens, n_ens, n_total, spl_steps, nullptr, t, &L));
        void *ws = mem.get(L.bytes);
        if (!ws) return fail(RNGLD_EHIP, "autotune scratch allocation failed");
        RNGLD_TRY_HIP(launch_upload(static_cast<uint8_t *>(ws) + L.off_ens, L.ens.data(), sizeof(EnsDev) * L.ens.size(),
                                    tm.st));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int rc = capture_run(g2, state, L, t, n_total, spl_steps, x, v, ws, &graph, &exec);
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && rc == RNGLD_OK; ++rep) {
            float m = 0.0f;
            rc = tm.time([&] {
                const hipError_t e = hipGraphLaunch(exec, tm.st);
                return e == hipSuccess ? RNGLD_OK : fail(RNGLD_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
            }, &m);
            if (rep > 0) ms = std::min(ms, m);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != RNGLD_OK) return rc;
        if (spl == 0 || ms < spl_best_ms * 0.995f) {
            spl_best_ms = ms;
            spl_best = spl;
        }
    }
    best.steps_per_launch = spl_best;
    if (debug_enabled())
        fprintf(stderr, "[rngld] autotune %s: block %u, %u per thread, %u blocks per CU, %u steps per launch "
                        "(%.3f ms for %u proxy steps)\n",
                key.c_str(), best.block, best.osc_per_thread, best.blocks_per_cu, best.steps_per_launch, spl_best_ms,
                spl_steps);
    RNGLD_TRY_HIP(hipStreamSynchronize(tm.st));
    cache_store(cache_path, key, best);
    RNGLD_TRY(ld_set_tuning(g.kind, &best));
    *out = best;
    return RNGLD_OK;
}

// ---- adjoint ----------------------------------------------------------------------------------------
namespace {

constexpr uint32_t kAdjTile = 256;

int check_loss(const ld_loss *loss, uint32_t n_steps) {
    if (!loss) return fail(RNGLD_EINVAL, "loss is NULL");
    if (loss->K == 0) return fail(RNGLD_EINVAL, "checkpoint interval K must be positive");
    if (loss->flags & ~(RNGLD_ADJ_REPLAY | RNGLD_ADJ_SPREAD)) return fail(RNGLD_EINVAL, "unknown loss flags");
    if (loss->t_begin < 1 || loss->t_end < loss->t_begin || loss->t_end > n_steps)
        return fail(RNGLD_EINVAL, "loss window must satisfy 1 <= t_begin <= t_end <= n_steps");
    return RNGLD_OK;
}

struct AdjLayout {
    std::vector<EnsDev> ens;
    std::vector<AdjCoef> adj;
    uint32_t n_tiles = 0;
    bool any_replay = false, any_reg_only = false, any_sp = false, any_seq = false;
    size_t off_ens = 0, off_adj = 0, off_partials = 0, off_jump = 0, off_coef = 0, off_scratch = 0, off_seg_d = 0,
           bytes = 0;
};

// The segment-parallel forward's per-ensemble constants, in FP64 from the FP32 coefficients:
// F^K, F^len of the last segment, B^K = (F^K)^T, and the three window sums of a whole segment
// (each term from the FP32 values of a_j, b_j, as the kernels' table holds them).
void segment_constants(AdjCoef &A, uint32_t K, uint32_t len_last) {
    const double h = A.f.h, c = A.f.c, kap = A.f.kap;
    const double F[4] = {1.0 - h * kap, h * c, -kap, c};
    double pf[4] = {1, 0, 0, 1};
    for (int k = 0; k < 3; ++k) A.full[k] = 0.0;
    auto mul = [](const double *p, const double *q, double *out) {
        const double r0 = p[0] * q[0] + p[1] * q[2], r1 = p[0] * q[1] + p[1] * q[3];
        const double r2 = p[2] * q[0] + p[3] * q[2], r3 = p[2] * q[1] + p[3] * q[3];
        out[0] = r0, out[1] = r1, out[2] = r2, out[3] = r3;
    };
    for (uint32_t j = 1; j <= K; ++j) {
        mul(pf, F, pf);
        const double ca = static_cast<float>(pf[0]), cb = static_cast<float>(pf[1]);
        A.full[0] += ca * ca, A.full[1] += ca * cb, A.full[2] += cb * cb;
        if (j == len_last)
            for (int k = 0; k < 4; ++k) A.flast[k] = pf[k];
    }
    for (int k = 0; k < 4; ++k) A.fk[k] = pf[k];
    A.bk[0] = pf[0], A.bk[1] = pf[2], A.bk[2] = pf[1], A.bk[3] = pf[3];
}

// longest segment the segment-parallel forward takes (its coefficient table has K entries per
// ensemble), and the fewest segments for which it pays
constexpr uint32_t kSpMaxK = 1u << 16;
constexpr uint64_t kSpMinSegments = 2;

// B^K for the adjoint step matrix B = [[1 - kap h, -kap], [c h, c]] (row-major), the map that
// carries the adjoint (lam_x, lam_v) at a K-step segment's end to its start with no loss terms;
// evaluated as the kernels' recursion mu = lam_v + h lam_x, lam_x -= kap mu, lam_v = c mu, in FP64
void adjoint_propagator(const LdCoef &q, uint32_t K, float phi[4]) {
    const double h = q.h, c = q.c, kap = q.kap;
    double c1x = 1, c1v = 0, c2x = 0, c2v = 1;  // images of the unit vectors (columns)
    for (uint32_t j = 0; j < K; ++j) {
        const double m1 = c1v + h * c1x, m2 = c2v + h * c2x;
        c1x -= kap * m1;
        c1v = c * m1;
        c2x -= kap * m2;
        c2v = c * m2;
    }
    phi[0] = static_cast<float>(c1x);
    phi[1] = static_cast<float>(c2x);
    phi[2] = static_cast<float>(c1v);
    phi[3] = static_cast<float>(c2v);
}

// Largest growth of a perturbation over 1..K inverse steps of the underdamped integrator with
// these FP32 coefficients: max_j |M^j|_F, M the inverse of the step matrix A = [[1 - h kap, h c],
// [-kap, c]] acting on (x, v) (v' = c v - kap x, x' = x + h v').  The register-only backward
// carries the loss adjoint forward in time through a segment with B^-1 = M^T (the adjoint step is
// B = A^T), whose powers have the same norms.  Returns as soon as the growth exceeds `limit`.
double reverse_growth(const LdCoef &q, uint32_t K, double limit) {
    const double c = q.c, kap = q.kap, h = q.h;
    if (!(c > 0.0)) return HUGE_VAL;
    const double a11 = 1.0 - h * kap, a12 = h * c, a21 = -kap, a22 = c;
    const double det = a11 * a22 - a12 * a21;  // = c
    const double m11 = a22 / det, m12 = -a12 / det, m21 = -a21 / det, m22 = a11 / det;
    double p11 = 1, p12 = 0, p21 = 0, p22 = 1, worst = 0;
    for (uint32_t j = 0; j < K; ++j) {
        const double n11 = m11 * p11 + m12 * p21, n12 = m11 * p12 + m12 * p22;
        const double n21 = m21 * p11 + m22 * p21, n22 = m21 * p12 + m22 * p22;
        p11 = n11, p12 = n12, p21 = n21, p22 = n22;
        worst = std::max(worst, std::sqrt(p11 * p11 + p12 * p12 + p21 * p21 + p22 * p22));
        if (worst > limit) return worst;
    }
    return worst;
}

constexpr double kAdjGrowthLimit = 8.0;
constexpr uint32_t kAdjLamMaxK = 1u << 22;

int layout_adj(const Gen &g, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total, uint32_t n_steps,
               const ld_loss &loss, AdjLayout *L) {
    const uint32_t K = loss.K;
    L->ens.resize(n_ens);
    L->adj.resize(n_ens);
    uint64_t acc = 0;
    for (uint32_t e = 0; e < n_ens; ++e) {
        EnsDev &E = L->ens[e];
        memset(&E, 0, sizeof(E));
        E.offset = h_ens[e].offset;
        E.n = h_ens[e].n;
        E.tile_begin = static_cast<uint32_t>(acc);
        E.n_tiles = static_cast<uint32_t>((E.n + kAdjTile - 1) / kAdjTile);
        E.coef = make_coef(h_ens[e].p);
        acc += E.n_tiles;
        const ld_params &p = h_ens[e].p;
        AdjCoef &A = L->adj[e];
        A.f = E.coef;
        A.dkap_dk = static_cast<float>(static_cast<double>(p.dt) / p.m);
        A.dc_dgamma = static_cast<float>(-static_cast<double>(p.dt));
        const double sig = std::sqrt(2.0 * p.gamma * static_cast<double>(p.kT) * p.dt / p.m);
        A.dsig_dgamma = static_cast<float>(sig / (2.0 * p.gamma));
        A.dsig_dkT = static_cast<float>(sig / (2.0 * p.kT));
        A.inv_c = static_cast<float>(1.0 / static_cast<double>(A.f.c));
        A.inv_c_lo = static_cast<float>(1.0 / static_cast<double>(A.f.c) - static_cast<double>(A.inv_c));
        // the register-only backward launches one block row per segment (grid y below 2^16)
        const uint64_t nseg = (static_cast<uint64_t>(n_steps) + K - 1) / K;
        A.lam = (g.kind == RNGLD_HYBRID_TAUS || g.kind == RNGLD_RAN2) && K <= kAdjLamMaxK && nseg < 65536 &&
                reverse_growth(A.f, K, kAdjGrowthLimit) <= kAdjGrowthLimit;
        A.reg_only = A.lam && !(loss.flags & RNGLD_ADJ_REPLAY);
        // the segment-parallel forward jumps Hybrid Taus over GF(2); Ran2's shuffle table has no such jump
        A.sp = A.lam && g.kind == RNGLD_HYBRID_TAUS && K <= kSpMaxK && nseg >= kSpMinSegments;
        if (A.lam) adjoint_propagator(A.f, K, A.phi);
        if (A.sp) segment_constants(A, K, static_cast<uint32_t>(n_steps - (nseg - 1) * K));
        if (E.n) {
            L->any_reg_only |= A.reg_only != 0;
            L->any_replay |= A.reg_only == 0;
            L->any_sp |= A.sp != 0;
            L->any_seq |= A.sp == 0;
        }
    }
    if (acc >= (1ull << 31)) return fail(RNGLD_EINVAL, "too many tiles");
    L->n_tiles = static_cast<uint32_t>(acc);
    L->off_ens = 0;
    L->off_adj = align_up(sizeof(EnsDev) * n_ens);
    L->off_partials = align_up(L->off_adj + sizeof(AdjCoef) * n_ens);
    const uint64_t nseg = (static_cast<uint64_t>(n_steps) + K - 1) / K;
    L->off_jump = align_up(L->off_partials + kAdjPartW * sizeof(double) * std::max<uint32_t>(L->n_tiles, 1));
    L->off_coef = align_up(L->off_jump + (L->any_sp ? nseg * kJumpWords * sizeof(uint32_t) : 0));
    L->off_scratch = align_up(L->off_coef + (L->any_sp ? static_cast<uint64_t>(n_ens) * K * sizeof(float2) : 0));
    // the forward's segment records and the backward's scratch share the space after off_scratch;
    // both calls take the larger size, so one workspace serves both
    const size_t fwd = L->any_sp ? align_up(nseg * kFwdSegF * n_total * sizeof(float)) : 0;
    size_t bwd = L->any_replay ? align_up(9ull * K * n_total * sizeof(float)) : 0;
    L->off_seg_d = L->off_scratch + bwd;
    if (L->any_reg_only) bwd += align_up(nseg * kAdjSegD * n_total * sizeof(double));
    L->bytes = L->off_scratch + std::max(fwd, bwd);
    return RNGLD_OK;
}

int check_adj_common(const rngld_cfg *cfg, Gen *g, const ld_ensemble *h_ens, uint32_t n_ens, uint64_t n_total,
                     uint32_t n_steps, const ld_loss *loss) {
    RNGLD_TRY(check_cfg(cfg, g));
    if (g->kind != RNGLD_HYBRID_TAUS && g->kind != RNGLD_RAN2)
        return fail(RNGLD_ENOTSUP, "gradients are implemented for Hybrid Taus and Ran2");
    RNGLD_TRY(check_loss(loss, n_steps));
    RNGLD_TRY(check_ensembles(h_ens, n_ens, n_total, true));
    for (uint32_t e = 0; e < n_ens; ++e)
        if (h_ens[e].p.scheme != 0) return fail(RNGLD_ENOTSUP, "gradients use the underdamped scheme");
    if (n_total > kMaxStreams) return fail(RNGLD_EINVAL, "n_total too large");
    return RNGLD_OK;
}

// x[3], v[3], the generator rows, then the loss adjoint lam_x[3], lam_v[3]
uint32_t ckpt_lam_row(const Gen &g) { return g.kind == RNGLD_HYBRID_TAUS ? kCkptLamRow : kCkptLamRowRan2; }
size_t ckpt_record_bytes(const Gen &g, uint64_t n_total) {
    return static_cast<size_t>(n_total) * (ckpt_lam_row(g) + 6) * 4;
}

}  // namespace

extern "C" int ld_ckpt_bytes(const rngld_cfg *cfg, uint64_t n_total, uint32_t n_steps, uint32_t K, size_t *bytes) {
    Gen g;
    RNGLD_TRY(check_cfg(cfg, &g));
    if (g.kind != RNGLD_HYBRID_TAUS && g.kind != RNGLD_RAN2)
        return fail(RNGLD_ENOTSUP, "gradients are implemented for Hybrid Taus and Ran2");
    if (!bytes) return fail(RNGLD_EINVAL, "bytes is NULL");
    if (K == 0) return fail(RNGLD_EINVAL, "K must be positive");
    const uint64_t nrec = (static_cast<uint64_t>(n_steps) + K - 1) / K + 1;  // + the end state
    *bytes = nrec * ckpt_record_bytes(g, n_total);
    return RNGLD_OK;
}

extern "C" int ld_adjoint_workspace_bytes(const rngld_cfg *cfg, const ld_ensemble *h_ens, uint32_t n_ens,
                                          uint64_t n_total, uint32_t n_steps, const ld_loss *loss, size_t *bytes) {
    Gen g;
    RNGLD_TRY(check_adj_common(cfg, &g, h_ens, n_ens, n_total, n_steps, loss));
    if (!bytes) return fail(RNGLD_EINVAL, "bytes is NULL");
    AdjLayout L;
    RNGLD_TRY(layout_adj(g, h_ens, n_ens, n_total, n_steps, *loss, &L));
    *bytes = L.bytes;
    return RNGLD_OK;
}

extern "C" int ld_run_ckpt(const rngld_cfg *cfg, void *d_state, size_t state_bytes, const ld_ensemble *h_ens,
                           uint32_t n_ens, uint64_t n_total, uint32_t n_steps, float *d_x, float *d_v,
                           const ld_loss *loss, void *d_ckpt, size_t ckpt_bytes, double *d_loss, void *d_ws,
                           size_t ws_bytes, void *stream) {
    Gen g;
    RNGLD_TRY(check_adj_common(cfg, &g, h_ens, n_ens, n_total, n_steps, loss));
    RNGLD_TRY(check_state(g, d_state, state_bytes));
    if (n_total > g.S) return fail(RNGLD_ESIZE, "n_total exceeds the state's streams");
    size_t need_ck = 0;
    RNGLD_TRY(ld_ckpt_bytes(cfg, n_total, n_steps, loss->K, &need_ck));
    if (ckpt_bytes < need_ck) return fail(RNGLD_ESIZE, "checkpoint buffer %zu < %zu bytes", ckpt_bytes, need_ck);
    AdjLayout L;
    RNGLD_TRY(layout_adj(g, h_ens, n_ens, n_total, n_steps, *loss, &L));
    if (ws_bytes < L.bytes) return fail(RNGLD_ESIZE, "workspace %zu bytes < %zu required", ws_bytes, L.bytes);
    if (!d_ws || !d_loss || (n_total && (!d_x || !d_v || !d_ckpt))) return fail(RNGLD_EINVAL, "NULL buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    RNGLD_TRY_HIP(launch_upload(ws + L.off_ens, L.ens.data(), sizeof(EnsDev) * n_ens, st));
    RNGLD_TRY_HIP(launch_upload(ws + L.off_adj, L.adj.data(), sizeof(AdjCoef) * n_ens, st));
    AdjArgs a{};
    a.state = d_state;
    a.S = g.S;
    a.x = d_x;
    a.v = d_v;
    a.NT = n_total;
    a.ens = reinterpret_cast<const EnsDev *>(ws + L.off_ens);
    a.adj = reinterpret_cast<const AdjCoef *>(ws + L.off_adj);
    a.n_ens = n_ens;
    a.n_tiles = L.n_tiles;
    a.n_steps = n_steps;
    a.K = loss->K;
    a.t_begin = loss->t_begin;
    a.t_end = loss->t_end;
    a.ckpt = static_cast<uint8_t *>(d_ckpt);
    a.rec_bytes = ckpt_record_bytes(g, n_total);
    a.lam_row = ckpt_lam_row(g);
    a.partials = reinterpret_cast<double *>(ws + L.off_partials);
    a.jump = reinterpret_cast<uint32_t *>(ws + L.off_jump);
    a.coef = reinterpret_cast<float2 *>(ws + L.off_coef);
    a.fwd_seg = reinterpret_cast<float *>(ws + L.off_scratch);
    RNGLD_TRY_HIP(launch_ld_ckpt(g.kind, a, L.any_sp, L.any_seq, st));
    RNGLD_TRY_HIP(launch_adj_finalize(a.partials, L.n_tiles, 1, false, a.ens, n_ens,
                                      static_cast<double>(loss->t_end - loss->t_begin + 1), d_loss, st));
    return RNGLD_OK;
}

extern "C" int ld_run_backward(const rngld_cfg *cfg, const void *d_ckpt, size_t ckpt_bytes, const ld_ensemble *h_ens,
                               uint32_t n_ens, uint64_t n_total, uint32_t n_steps, const ld_loss *loss,
                               double *d_grad, void *d_ws, size_t ws_bytes, void *stream) {
    Gen g;
    RNGLD_TRY(check_adj_common(cfg, &g, h_ens, n_ens, n_total, n_steps, loss));
    size_t need_ck = 0;
    RNGLD_TRY(ld_ckpt_bytes(cfg, n_total, n_steps, loss->K, &need_ck));
    if (ckpt_bytes < need_ck) return fail(RNGLD_ESIZE, "checkpoint buffer %zu < %zu bytes", ckpt_bytes, need_ck);
    AdjLayout L;
    RNGLD_TRY(layout_adj(g, h_ens, n_ens, n_total, n_steps, *loss, &L));
    if (ws_bytes < L.bytes) return fail(RNGLD_ESIZE, "workspace %zu bytes < %zu required", ws_bytes, L.bytes);
    if (!d_ws || !d_grad || (n_total && !d_ckpt)) return fail(RNGLD_EINVAL, "NULL buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *ws = static_cast<uint8_t *>(d_ws);
    RNGLD_TRY_HIP(launch_upload(ws + L.off_ens, L.ens.data(), sizeof(EnsDev) * n_ens, st));
    RNGLD_TRY_HIP(launch_upload(ws + L.off_adj, L.adj.data(), sizeof(AdjCoef) * n_ens, st));
    AdjArgs a{};
    a.NT = n_total;
    a.ens = reinterpret_cast<const EnsDev *>(ws + L.off_ens);
    a.adj = reinterpret_cast<const AdjCoef *>(ws + L.off_adj);
    a.n_ens = n_ens;
    a.n_tiles = L.n_tiles;
    a.n_steps = n_steps;
    a.K = loss->K;
    a.t_begin = loss->t_begin;
    a.t_end = loss->t_end;
    a.ckpt = const_cast<uint8_t *>(static_cast<const uint8_t *>(d_ckpt));
    a.rec_bytes = ckpt_record_bytes(g, n_total);
    a.lam_row = ckpt_lam_row(g);
    a.scratch = L.any_replay ? reinterpret_cast<float *>(ws + L.off_scratch) : nullptr;
    a.seg_d = L.any_reg_only ? reinterpret_cast<double *>(ws + L.off_seg_d) : nullptr;
    a.partials = reinterpret_cast<double *>(ws + L.off_partials);
    // n_steps >= 1 (check_loss); every tile's partials are written by exactly one of the kernels
    RNGLD_TRY_HIP(launch_ld_adjoint(g.kind, a, L.any_replay, L.any_reg_only, st));
    RNGLD_TRY_HIP(launch_adj_finalize(a.partials, L.n_tiles, 3, (loss->flags & RNGLD_ADJ_SPREAD) != 0, a.ens, n_ens,
                                      static_cast<double>(loss->t_end - loss->t_begin + 1), d_grad, st));
    return RNGLD_OK;
}
