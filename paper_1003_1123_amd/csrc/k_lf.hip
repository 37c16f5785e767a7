// k_lf.hip -- additive lagged Fibonacci, one generator shared by all threads (Sec. III.C; Alg. 3).
//
// y_n = y_{n-ll} + y_{n-sl} mod 2^32 (Eq. 3).  The state is a ring of R >= ll + W 32-bit words in
// device memory; slot (slot0 + n - pos) mod R holds y_n.
//
// Three ways to run the dependency structure (a position needs the positions sl and ll back):
//  * waves: W <= sl consecutive positions per launch; every source is in an earlier wave; kernel
//    boundaries order the waves and make their writes visible across the XCDs' L2 caches.  This is
//    the device-wide synchronisation after every step of Sec. III.A, at wave granularity.
//    (Table I rows do not satisfy the paper's race-free condition ll - sl > RNS N; the ring removes
//    that condition.)
//  * producer/consumer (fused LD runs): one persistent launch in which producer waves extend the
//    sequence slice by slice in a ring of the run's own, each link on a 256-byte boundary, and
//    consumer waves drive the oscillators, synchronised by progress words (lf_flow.hpp;
//    lf_pc_kernel below).
//  * producers only (long bare streams): one persistent launch in which producer waves write the
//    sequence straight into the output, which serves as the lag table (lf_stream_kernel below).
// All reproduce the one sequential sequence exactly, for any wave width or schedule.
#include "internal.hpp"

namespace rngld {

namespace {

__device__ __forceinline__ uint32_t wrap_once(uint32_t s, uint32_t R) { return s >= R ? s - R : s; }
// slot - lag for lag <= R (slot < R)
__device__ __forceinline__ uint32_t back(uint32_t slot, uint32_t lag, uint32_t R) {
    return slot >= lag ? slot - lag : slot + (R - lag);
}
// window y_{-ll+i} = LCG^{i+1}(x0) in slots 0..ll-1 (position 0 at slot ll); the other slots are
// cleared (no position of a run ever reads them before writing them)
__global__ __launch_bounds__(kBulkBlock) void lf_seed_kernel(LfHeader *hdr, uint32_t *ring, uint32_t ll,
                                                             uint32_t sl, uint32_t R, uint32_t W, uint64_t seed) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i == 0) {
        hdr->pos = 0;
        hdr->slot = ll;
        hdr->ll = ll;
        hdr->sl = sl;
        hdr->R = R;
        hdr->W = W;
        for (int k = 0; k < 9; ++k) hdr->pad[k] = 0u;
    }
    if (i >= R) return;
    const uint32_t x0 = stream_seed_word(seed, 0, 0);
    ring[i] = i < ll ? lcg_skip(x0, i + 1) : 0u;
}

// one wave of rng_uniform: out[first + t] = y_{pos0 + first + t}; sources at or after pos0 come
// from out itself (the output doubles as the lag table), earlier ones from the ring
__global__ __launch_bounds__(kBulkBlock) void lf_uniform_phase_kernel(LfRing L, uint32_t *out, uint64_t first,
                                                                      uint32_t count) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= count) return;
    const uint64_t i = first + t;
    const uint32_t base = L.hdr->slot;
    const uint32_t a = i >= L.ll ? out[i - L.ll] : L.ring[back(base, L.ll - static_cast<uint32_t>(i), L.R)];
    const uint32_t b = i >= L.sl ? out[i - L.sl] : L.ring[back(base, L.sl - static_cast<uint32_t>(i), L.R)];
    out[i] = a + b;
}

// after a bulk call: the last min(count, ll) outputs become the ring's newest values
__global__ __launch_bounds__(kBulkBlock) void lf_ring_store_kernel(LfRing L, const uint32_t *out, uint64_t count,
                                                                   uint32_t m, uint32_t base_mod) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= m) return;
    const uint32_t slot = wrap_once(wrap_once(L.hdr->slot + base_mod, L.R) + t, L.R);
    const uint64_t i = count - m + t;
    L.ring[slot] = out[i];
}

// one wave of rng_gaussian: positions first + 2t, +1 (ring slots off_mod + 2t, +1 from pos0's)
__global__ __launch_bounds__(kBulkBlock) void lf_gauss_phase_kernel(LfRing L, float *out, uint64_t first,
                                                                    uint32_t off_mod, uint32_t pairs) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= pairs) return;
    const uint32_t s0 = wrap_once(wrap_once(L.hdr->slot + off_mod, L.R) + 2 * t, L.R);
    const uint32_t s1 = wrap_once(s0 + 1, L.R);
    const uint32_t w0 = L.ring[back(s0, L.ll, L.R)] + L.ring[back(s0, L.sl, L.R)];
    const uint32_t w1 = L.ring[back(s1, L.ll, L.R)] + L.ring[back(s1, L.sl, L.R)];
    L.ring[s0] = w0;
    L.ring[s1] = w1;
    const float r = box_muller_radius(w0);
    float c, s;
    box_muller_angle(w1, c, s);
    out[first + 2 * t] = r * c;
    out[first + 2 * t + 1] = r * s;
}

// one wave of the seeding discard: positions pos0 + first + t, t < count, generated into the ring
// only (slots off_mod + t from pos0's); the header is advanced afterwards
__global__ __launch_bounds__(kBulkBlock) void lf_discard_phase_kernel(LfRing L, uint32_t off_mod, uint32_t count) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= count) return;
    const uint32_t s = wrap_once(wrap_once(L.hdr->slot + off_mod, L.R) + t, L.R);
    L.ring[s] = L.ring[back(s, L.ll, L.R)] + L.ring[back(s, L.sl, L.R)];
}

__global__ void lf_advance_kernel(LfHeader *hdr, uint64_t count, uint32_t count_mod) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        hdr->pos += count;
        uint32_t s = hdr->slot + count_mod;
        hdr->slot = s >= hdr->R ? s - hdr->R : s;
    }
}

// one wave of an LD step: thread t owns oscillator osc_begin + t and positions 4t..4t+3 of the
// wave (Alg. 3: thread j takes y_{(j + N t) RNS + r}); the observables of the step's starting
// state are recorded first when the step is an observation point
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void lf_ld_phase_kernel(LfLdPhase ph) {
    __shared__ double red[BLOCK / 64][6];
    const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
    const bool act = t < ph.osc_count;
    const uint64_t o = ph.osc_begin + t;
    float x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    if (act)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = ph.x[d * ph.N + o];
            v[d] = ph.v[d * ph.N + o];
        }
    if (ph.stride && ph.step % ph.stride == 0) {
        float x0[3] = {0, 0, 0}, v0[3] = {0, 0, 0};
        if (act && ph.step == ph.t0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x0[d] = x[d];
                v0[d] = v[d];
            }
        } else if (act && ph.step > ph.t0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x0[d] = ph.t0buf[d * ph.N + o];
                v0[d] = ph.t0buf[(3 + d) * ph.N + o];
            }
        }
        double q[6] = {0, 0, 0, 0, 0, 0};
        if (act) add_observables(q, x, v, x0, v0, ph.step >= ph.t0);
        double *dst = ph.partials +
                      (static_cast<uint64_t>(ph.step / ph.stride) * ph.n_tiles + ph.tile_base + blockIdx.x) * 6;
        block_sum6<BLOCK>(q, red, dst);
    }
    if (!act) return;
    if (ph.stride && ph.step == ph.t0)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ph.t0buf[d * ph.N + o] = x[d];
            ph.t0buf[(3 + d) * ph.N + o] = v[d];
        }
    const uint32_t R = ph.L.R;
    uint32_t slot = wrap_once(wrap_once(ph.L.hdr->slot + ph.off_mod, R) + 4 * t, R);
    uint32_t w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w[r] = ph.L.ring[back(slot, ph.L.ll, R)] + ph.L.ring[back(slot, ph.L.sl, R)];
        ph.L.ring[slot] = w[r];
        slot = wrap_once(slot + 1, R);
    }
    float g[3];
    gaussian_forces(w[0], w[1], w[2], w[3], g[0], g[1], g[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ld_update(ph.coef, x[d], v[d], g[d]);
        ph.x[d * ph.N + o] = x[d];
        ph.v[d * ph.N + o] = v[d];
    }
}

// observables of the final state, with the same tiling as the waves (one tile per wave block)
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void lf_observe_kernel(LfLdPhase ph, uint32_t bpp, uint64_t phase_osc,
                                                           uint32_t point, bool t0_now) {
    __shared__ double red[BLOCK / 64][6];
    const uint32_t phase = blockIdx.x / bpp, b = blockIdx.x % bpp;
    const uint64_t begin = static_cast<uint64_t>(phase) * phase_osc;
    const uint64_t count = (begin + phase_osc <= ph.n_osc) ? phase_osc : ph.n_osc - begin;
    const uint64_t t = static_cast<uint64_t>(b) * BLOCK + threadIdx.x;
    const bool act = t < count;
    const uint64_t o = begin + t;
    double q[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        float x[3], v[3], x0[3], v0[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = ph.x[d * ph.N + o];
            v[d] = ph.v[d * ph.N + o];
            x0[d] = t0_now ? x[d] : ph.t0buf[d * ph.N + o];
            v0[d] = t0_now ? v[d] : ph.t0buf[(3 + d) * ph.N + o];
        }
        add_observables(q, x, v, x0, v0, true);
    }
    block_sum6<BLOCK>(q, red, ph.partials + (static_cast<uint64_t>(point) * ph.n_tiles + blockIdx.x) * 6);
}

// ---- persistent producer/consumer run ----------------------------------------------------------
// One cooperative launch of one 1024-thread block per CU runs every LD step.  The first np waves of
// a block are producers, the others consumers (roles, waits and the no-deadlock argument:
// lf_flow.hpp).  No block-wide barrier: every wave works on its own.
//  * Ring words and progress words are read and written with device-scope (agent) atomics, which
//    bypass the XCDs' mutually non-coherent L2 caches.  A producer waits for its ring stores to
//    complete (s_waitcnt) before it stores its progress word; a reader issues its ring loads only
//    after the progress words it waits for have been seen.  No cache-wide release or acquire fence
//    is needed.
//  * A consumer publishes a tile only after its loads have returned, so the slots may then be
//    rewritten.
//  * Every wait is bounded: after spin_limit polls, or once another wave has given up, the wave
//    stops, status[0] is set and the run's results are invalid.
__device__ __forceinline__ uint32_t agent_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ring word `idx` (the dataflow run's ring is below 2^29 words, so the byte offset fits 31 bits and
// the store takes the ring base from scalar registers and one 32-bit offset register)
__device__ __forceinline__ void ring_put(uint32_t *ring, uint32_t idx, uint32_t v) {
    agent_store(reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(ring) + (idx << 2)), v);
}

constexpr int kFlowM = kLfFlowSliceMax / 64;  // producer positions per lane per link
constexpr int kFlowG = kFlowM / 4;             // ... in groups of four consecutive offsets

// The persistent run moves ring words four at a time: 16-byte buffer loads and stores with the
// sc1 cache policy (device scope, the same policy as the agent-scope word accesses above), lane l
// taking four consecutive words.  A wave then moves 1 KiB per instruction, which on MI355X
// sustains the run's two-loads-per-store mix about 10% faster than 4-byte accesses and issues a
// quarter of the memory instructions.  The resource's size bounds every access (an access past it
// reads zeros and writes nothing); a 16-byte access needs only 4-byte alignment.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Box-Muller pairs of four consecutive words (two whole pairs), as their bit patterns
__device__ __forceinline__ u32x4 box_muller_pairs4(const u32x4 &wv) {
    u32x4 gv;
    float c, sn;
    float r = box_muller_radius(wv[0]);
    box_muller_angle(wv[1], c, sn);
    gv[0] = __float_as_uint(r * c);
    gv[1] = __float_as_uint(r * sn);
    r = box_muller_radius(wv[2]);
    box_muller_angle(wv[3], c, sn);
    gv[2] = __float_as_uint(r * c);
    gv[3] = __float_as_uint(r * sn);
    return gv;
}
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 encoding
constexpr int kCachePolicySc1 = 16;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ring_rsrc(uint32_t *ring, uint32_t words) {
    return __builtin_amdgcn_make_buffer_rsrc(ring, 0, static_cast<int>(words * 4u), kBufferWord3);
}
__device__ __forceinline__ u32x4 ring_get4(__amdgpu_buffer_rsrc_t r, uint32_t word) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(word << 2), 0, kCachePolicySc1);
}
// the first three words at `word` (a straddling group's second part: at most three words, and a
// load whose result is all used keeps the compiler from reusing a register it still writes)
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
__device__ __forceinline__ u32x3 ring_get3(__amdgpu_buffer_rsrc_t r, uint32_t word) {
    return __builtin_amdgcn_raw_buffer_load_b96(r, static_cast<int>(word << 2), 0, kCachePolicySc1);
}
__device__ __forceinline__ void ring_put4(__amdgpu_buffer_rsrc_t r, uint32_t word, u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, static_cast<int>(word << 2), 0, kCachePolicySc1);
}

// up to 64 waits of one wave, one per lane; `tile` tags a consumer's wait with its tile
struct FlowWaits {
    const uint32_t *flag;
    uint32_t need;
    uint32_t tile;
    uint32_t n;  // collected so far (the same in every lane)
};

__device__ __forceinline__ void wait_add(FlowWaits &w, uint32_t lane, const uint32_t *flag, uint32_t need,
                                         uint32_t tile) {
    if (lane == w.n) {
        w.flag = flag;
        w.need = need;
        w.tile = tile;
    }
    ++w.n;
}

// pause between polls, growing with the number of failed polls up to about 0.4 us: pollers
// must not flood the memory path that the waited-for stores travel on
__device__ __forceinline__ void poll_pause(uint32_t spins) {
    const uint32_t n = spins < 16u ? spins : 16u;
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(8);
}

// block until every collected wait holds; false if the run gave up
__device__ __forceinline__ bool wait_all(FlowWaits &w, uint32_t lane, const LfFlowArgs &a) {
    bool ok = true;
    if (lane < w.n) {
        uint32_t spins = 0;
        while (agent_load(w.flag) < w.need) {
            if (++spins > a.spin_limit || ((spins & 15u) == 0 && agent_load(a.status) != 0u)) {
                agent_store(a.status, 1u);
                ok = false;
                break;
            }
            poll_pause(spins);
        }
    }
    w.n = 0;
    return __all(ok);
}

// Producer p: offsets [p T, min((p+1) T, sl)) of every link; lane takes the four-offset groups
// 4 lane + 256 r.  Software-pipelined over links.  When link j is summed, one read of the progress
// words link j+1 waits for and then link j's long-lag loads were issued during link j-1.  If those
// waits hold, link j's stores are followed at once by the read for link j+2 and link j+1's loads,
// and s_waitcnt vmcnt(kFlowG + 1) then means that every store of link j has completed (vector
// memory operations complete in issue order), so link j can be published while link j+1's loads
// are in flight.  Otherwise link j is published first and only then does the producer block on link
// j+1's waits: it never blocks with an earlier link unpublished (the no-deadlock argument of
// lf_flow.hpp with one link per iteration).
// The waits of link j, 64 per round: from the steady link on, a full slice takes the fixed
// template of waits (a) and (c) and walks only the consumers (b); otherwise the general form.
__device__ __forceinline__ uint32_t producer_waits(const LfFlowArgs &a, uint32_t p, uint32_t j, uint32_t o_lo,
                                                   uint32_t len, uint32_t width, const LfWaitTemplate &tpl,
                                                   int64_t step_R, uint64_t off_R, FlowWaits &w, uint32_t lane,
                                                   uint32_t round) {
    uint32_t idx = 0;
    auto add = [&](const uint32_t *f, uint32_t need) {
        if (idx - 64u * round < 64u) wait_add(w, lane, f, need, 0);
        ++idx;
        return true;
    };
    if (!len) return 0;
    if (len == width && j >= lf_steady_link(a.geom)) {
#pragma unroll
        for (uint32_t i = 0; i < 6; ++i)  // constant indices keep the template in registers
            if (i < tpl.n)
                add(a.prod + tpl.slice[i] * kLfFlagStride, static_cast<uint32_t>(static_cast<int64_t>(j) + tpl.d[i]));
        lf_walk_consumers(a.geom, step_R, off_R, len,
                          [&](uint32_t c, uint32_t need) { return add(a.cons + c * kLfFlagStride, need); });
    } else {
        lf_producer_waits(
            a.geom, p, j, o_lo, len, step_R, off_R,
            [&](uint32_t s, uint32_t need) { return add(a.prod + s * kLfFlagStride, need); },
            [&](uint32_t c, uint32_t need) { return add(a.cons + c * kLfFlagStride, need); });
    }
    return idx;  // waits in all
}

// block until every wait of link j holds (64 per round); false if the run gave up
__device__ __forceinline__ bool producer_wait_link(const LfFlowArgs &a, uint32_t p, uint32_t j, uint32_t o_lo,
                                                   uint32_t len, uint32_t width, const LfWaitTemplate &tpl,
                                                   int64_t step_R, uint64_t off_R, FlowWaits &w, uint32_t lane) {
    for (uint32_t round = 0;; ++round) {
        const uint32_t total = producer_waits(a, p, j, o_lo, len, width, tpl, step_R, off_R, w, lane, round);
        if (!wait_all(w, lane, a)) return false;
        if (total <= 64u * (round + 1)) return true;
    }
}

__device__ __forceinline__ void lf_producer(const LfFlowArgs &a, uint32_t p, uint32_t lane) {
    const LfFlowGeom &g = a.geom;
    if (p >= g.n_slices) return;
    const uint32_t sl = g.sl, lla = g.ll.a, llb = g.ll.b;  // ll = lla sl + llb
    const uint32_t slp = a.pr.slp, ring_words = a.pr.nr * a.pr.slp;
    const uint32_t o_lo = p << g.slice_log2;
    const uint32_t width = ((1u << g.slice_log2) < sl - o_lo) ? (1u << g.slice_log2) : sl - o_lo;
    uint32_t *ring = a.pring;
    auto link_len = [&](uint32_t j) -> uint32_t {
        if (j >= g.n_links) return 0u;
        const uint64_t P_lo = static_cast<uint64_t>(j) * sl + o_lo;
        return P_lo >= g.Ptot ? 0u : (g.Ptot - P_lo < width ? static_cast<uint32_t>(g.Ptot - P_lo) : width);
    };
    // words of link j and of link j - lla, the long lag's link for offsets >= llb (advanced
    // together, link by link)
    uint32_t base = 0, base_ll = lf_pad_base(a.pr, -static_cast<int64_t>(lla));
    const __amdgpu_buffer_rsrc_t rr = ring_rsrc(ring, ring_words);
    // lane takes the groups of offsets o_lo + 256 r + 4 lane + (0..3), r < kFlowG; a group that
    // starts at or past the slice's width is not stored
    // y_{P - sl} of link 0 comes from the ring (link -1), afterwards from the previous link in
    // registers
    u32x4 chain[kFlowG], src[kFlowG];
    u32x3 src_x;
    {
        const uint32_t base_prev = lf_pad_base(a.pr, -1);
#pragma unroll
        for (int r = 0; r < kFlowG; ++r) chain[r] = ring_get4(rr, base_prev + o_lo + 256u * r + 4u * lane);
    }
    int64_t step_R;
    uint64_t off_R;
    // consumer coordinate of (link j, o_lo) - R, R = nr sl
    lf_consumer_coord0(g, o_lo, static_cast<uint64_t>(a.pr.nr) * sl, step_R, off_R);
    LfWaitTemplate tpl;
    lf_wait_template(g, p, o_lo, width, tpl);
    FlowWaits w;
    w.n = 0;
    // Long-lag sources: offset o reads (link - lla, o - llb) when o >= llb, else (link - lla - 1,
    // o + sl - llb), so a group's four sources are consecutive words unless the group straddles llb
    // (o < llb < o + 4): that one group, in lane xl of load xr, takes its words from o = llb on out
    // of a second load, of the first three words of link - lla.  kFlowG + 1 loads per lane, always
    // all issued; a group past the slice's width reads words it never uses.
    const uint32_t xo = llb > o_lo && llb < o_lo + width && (llb - o_lo) % 4u ? (llb - o_lo) / 4u : ~0u;
    const uint32_t xr = xo / 64u, xl = xo % 64u, xk = llb - o_lo - 4u * xo;
    const bool x_here = xo != ~0u && lane == xl;
    auto load_link = [&](uint32_t bll) {
        const uint32_t bll1 = bll >= slp ? bll - slp : bll + ring_words - slp;
#pragma unroll
        for (int r = 0; r < kFlowG; ++r) {
            const uint32_t o = o_lo + 256u * r + 4u * lane;
            src[r] = ring_get4(rr, o >= llb ? bll + (o - llb) : bll1 + (o + (sl - llb)));
        }
        // issued in every lane so that the count is fixed: past the ring's end (zeros, no memory
        // access) except in lane xl
        src_x = ring_get3(rr, x_here ? bll : ring_words);
    };
    // y_P = y_{P-sl} + y_{P-ll} for the lane's groups
    auto sum_link = [&]() {
#pragma unroll
        for (int r = 0; r < kFlowG; ++r) {
            u32x4 s = src[r];
            if (x_here && xr == static_cast<uint32_t>(r)) {
                // words k >= xk are offsets k - xk of link - lla
                if (xk == 1u) {
                    s.y = src_x.x;
                    s.z = src_x.y;
                    s.w = src_x.z;
                } else if (xk == 2u) {
                    s.z = src_x.x;
                    s.w = src_x.y;
                } else {
                    s.w = src_x.x;
                }
            }
            chain[r] += s;
        }
    };
    // one read of the first 64 progress words link j1 waits for (lanes without a wait read the
    // status word); it is issued just before a link's loads, so it has returned once they have
    uint32_t total_poll = 0, seen = 0;
    auto poll_link = [&](uint32_t j1, int64_t sR, uint64_t oR) {
        const uint32_t len_j1 = link_len(j1);
        total_poll = producer_waits(a, p, j1, o_lo, len_j1, width, tpl, sR, oR, w, lane, 0);
        seen = agent_load(lane < w.n ? w.flag : a.status);
    };
    uint32_t len = link_len(0);
    if (!producer_wait_link(a, p, 0, o_lo, len, width, tpl, step_R, off_R, w, lane)) return;
    {
        int64_t sR1 = step_R;
        uint64_t oR1 = off_R;
        lf_consumer_coord_next(g, sR1, oR1);
        poll_link(1, sR1, oR1);
    }
    load_link(base_ll);
    for (uint32_t j = 0; j < g.n_links; ++j) {
        const uint32_t next_base = base + slp < ring_words ? base + slp : 0u;
        const uint32_t next_base_ll = base_ll + slp < ring_words ? base_ll + slp : 0u;
        int64_t next_sR = step_R;
        uint64_t next_oR = off_R;
        lf_consumer_coord_next(g, next_sR, next_oR);
        const uint32_t next_len = link_len(j + 1);
        sum_link();
        // link j+1's waits, read before link j's loads (a partial next link takes the plain path)
        const bool ready = next_len == width && total_poll <= 64u && __all(lane >= w.n || seen >= w.need);
        w.n = 0;
        if (len == kLfFlowSliceMax) {
            // a full slice: straight-line stores, so that no store waits for another (a store in
            // a branch of its own can make the compiler wait for the previous one)
#pragma unroll
            for (int r = 0; r < kFlowG; ++r) ring_put4(rr, base + o_lo + 256u * r + 4u * lane, chain[r]);
        } else if (len == width) {
            // the last slice of a link: a group that reaches past sl writes into the link's
            // padding (slp is a multiple of 64 words, so round_up(sl, 4) <= slp)
#pragma unroll
            for (int r = 0; r < kFlowG; ++r)
                if (256u * r + 4u * lane < width) ring_put4(rr, base + o_lo + 256u * r + 4u * lane, chain[r]);
        } else {
            // the end of the run: word by word, nothing past the last position
#pragma unroll
            for (int r = 0; r < kFlowG; ++r) {
                const uint32_t q = 256u * r + 4u * lane;
                if (q < len) ring_put(ring, base + o_lo + q, chain[r].x);
                if (q + 1u < len) ring_put(ring, base + o_lo + q + 1u, chain[r].y);
                if (q + 2u < len) ring_put(ring, base + o_lo + q + 2u, chain[r].z);
                if (q + 3u < len) ring_put(ring, base + o_lo + q + 3u, chain[r].w);
            }
        }
        if (!ready) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0) agent_store(a.prod + p * kLfFlagStride, j + 1);
            if (!next_len) break;
            if (!producer_wait_link(a, p, j + 1, o_lo, next_len, width, tpl, next_sR, next_oR, w, lane)) return;
        }
        {
            int64_t sR2 = next_sR;
            uint64_t oR2 = next_oR;
            lf_consumer_coord_next(g, sR2, oR2);
            poll_link(j + 2, sR2, oR2);
        }
        load_link(next_base_ll);
        if (ready) {
            // only the poll and link j+1's kFlowG + 1 loads, issued after link j's stores, may
            // still be outstanding: link j is stored
            static_assert(kFlowG == 4, "the wait count below");
            asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
            if (lane == 0) agent_store(a.prod + p * kLfFlagStride, j + 1);
        }
        base = next_base;
        base_ll = next_base_ll;
        step_R = next_sR;
        off_R = next_oR;
        len = next_len;
    }
}

// observables of one 64-oscillator tile; lane 0 writes the tile's partial sums
__device__ __forceinline__ void tile_observe(const LfFlowArgs &a, const float *t0buf, const float *xv, uint32_t lane,
                                             uint64_t o, bool act, uint32_t s, uint32_t c) {
    double q[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        float x[3], v[3], x0[3] = {0, 0, 0}, v0[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = xv[d * 64 + lane];
            v[d] = xv[(3 + d) * 64 + lane];
            if (s >= a.t0) {
                x0[d] = s == a.t0 ? x[d] : t0buf[d * a.N + o];
                v0[d] = s == a.t0 ? v[d] : t0buf[(3 + d) * a.N + o];
            }
        }
        add_observables(q, x, v, x0, v0, s >= a.t0);
    }
    double *dst = a.partials + (static_cast<uint64_t>(s / a.stride) * a.pstride + c) * 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double t = wave_sum(q[i]);
        if (lane == 0) dst[i] = t;
    }
}

// s_waitcnt immediates (gfx9 encoding) that wait for vector memory only: vmcnt(1), vmcnt(0)
constexpr int kWaitVm1 = 0xF71, kWaitVm0 = 0xF70;

// Consumer wave cw: the Kc consecutive tiles cw Kc .. (64 oscillators each, lane l of tile k
// drives oscillator 64 (cw Kc + k) + l); x, v in LDS as xv[k][6][64].  A step's positions for the
// wave are the 4 (o1 - o0) consecutive ones from 4 o0 + s 4n, and lane l of tile k loads its
// oscillator's four as one group.  Per step: wait for the producers of the wave's positions, load
// them, publish, then drive the oscillators.  Up to 4 tiles per wave the steps are
// software-pipelined: the next step's loads go out before this step's LD update whenever a poll
// issued one step earlier shows its producers published (a second set of word registers, which 8
// tiles do not have).
// MODE kFlowGauss (bare Gaussian streams): no oscillators; lane l of tile k writes its group of four
// positions 4 (o + n s) .. + 3 to out as two Box-Muller pairs, with one 16-byte nontemporal store
// (the output is not read again here, and the ring it would otherwise push out of the caches is).
template <int KC, int MODE>
__device__ __forceinline__ void lf_consumer(const LfFlowArgs &a, uint32_t cw, uint32_t lane, float *xv) {
    constexpr bool kPipe = KC <= 4;
    const LfFlowGeom &g = a.geom;
    const uint32_t Kc = g.Kc, sl = g.sl, slp = a.pr.slp, nr = a.pr.nr, ring_words = nr * slp;
    const __amdgpu_buffer_rsrc_t rr = ring_rsrc(a.pring, ring_words);
    const uint64_t o0 = 64ull * cw * Kc < a.n ? 64ull * cw * Kc : a.n;
    const uint64_t o1 = 64ull * (cw + 1) * Kc < a.n ? 64ull * (cw + 1) * Kc : a.n;
    if (o0 >= o1) return;  // no oscillators: no producer ever waits for this wave
    const uint32_t cnt = static_cast<uint32_t>(4 * (o1 - o0));  // positions per step
    const uint32_t Kw = static_cast<uint32_t>((o1 - o0 + 63) / 64);
    if constexpr (MODE == kFlowLd) {
#pragma unroll 1
        for (uint32_t k = 0; k < Kw; ++k) {
            const uint64_t o = o0 + 64ull * k + lane;
            const bool act = o < o1;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xv[(k * 6 + d) * 64 + lane] = act ? a.x[d * a.N + o] : 0.0f;
                xv[(k * 6 + 3 + d) * 64 + lane] = act ? a.v[d * a.N + o] : 0.0f;
            }
        }
    }
    // coordinates of a step's first position 4 o0 + s 4n: its link, offset and the link's first
    // word (a step's positions span at most two links: 256 Kc <= sl)
    struct Coord {
        int64_t link;
        uint32_t off, lbase;
    };
    auto advance = [&](Coord &c) {
        const int64_t link_before = c.link;
        lf_link_coord_next_step(g, c.link, c.off);
        c.lbase += (static_cast<uint32_t>(c.link - link_before) % nr) * slp;
        if (c.lbase >= ring_words) c.lbase -= ring_words;
    };
    auto collect = [&](FlowWaits &w, const Coord &c) {
        w.n = 0;
        lf_walk_producers(g, c.link, c.off, cnt, [&](uint32_t sl_, uint32_t l) {
            wait_add(w, lane, a.prod + sl_ * kLfFlagStride, l + 1, 0);
            return true;
        });
    };
    // A step's words: lane l of tile k takes positions 256 k + 4 l .. + 3 of the step (a lane past
    // the wave's positions reads the step's first group).  The one group that may straddle the end
    // of the step's first link (o < sl < o + 4) takes its words from sl on from the next link's
    // first three words: a load of its own, issued once the step's loads have returned and waited
    // for at once (a few steps in a thousand), before the step is published.
    struct Words {
        u32x4 q[KC];
        uint32_t xk, xt, xw;  // xk > 0: group xt's words k >= xk are the words from xw on
    };
    auto load = [&](Words &W, const Coord &c) {
        const uint32_t nbase = c.lbase + slp < ring_words ? c.lbase + slp : 0u;
        W.xk = 0u;
        W.xt = 0u;
        W.xw = nbase;
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const uint32_t g0 = 256u * k + 4u * lane;
            const uint32_t o = c.off + (g0 < cnt ? g0 : 0u);
            W.q[k] = ring_get4(rr, o < sl ? c.lbase + o : nbase + (o - sl));
            // only a group the wave uses: a lane past the wave's positions reads the step's first
            // group, which may straddle too, and must not take the place of the lane's own
            if (g0 < cnt && o < sl && sl - o < 4u) {
                W.xk = sl - o;
                W.xt = k;
            }
        }
    };
    auto fix = [&](Words &W) {
        if (__any(W.xk != 0u)) {
            const u32x3 x = ring_get3(rr, W.xk ? W.xw : ring_words);
#pragma unroll
            for (int k = 0; k < KC; ++k)
                if (W.xk && W.xt == static_cast<uint32_t>(k)) {
                    if (W.xk == 1u) {
                        W.q[k].y = x.x;
                        W.q[k].z = x.y;
                        W.q[k].w = x.z;
                    } else if (W.xk == 2u) {
                        W.q[k].z = x.x;
                        W.q[k].w = x.y;
                    } else {
                        W.q[k].w = x.x;
                    }
                }
        }
    };
    auto observe = [&](uint32_t s) {
        if constexpr (MODE != kFlowLd) return;
        float *t0buf = a.t0buf;
        asm volatile("" : "+s"(t0buf));
        if (a.stride && s % a.stride == 0) {
#pragma unroll 1
            for (uint32_t k = 0; k < Kw; ++k) {
                const uint64_t o = o0 + 64ull * k + lane;
                tile_observe(a, t0buf, xv + k * 384, lane, o, o < o1, s, cw * Kc + k);
            }
        }
        if (a.stride && s == a.t0) {
#pragma unroll 1
            for (uint32_t k = 0; k < Kw; ++k) {
                const uint64_t o = o0 + 64ull * k + lane;
                if (o < o1)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        t0buf[d * a.N + o] = xv[(k * 6 + d) * 64 + lane];
                        t0buf[(3 + d) * a.N + o] = xv[(k * 6 + 3 + d) * 64 + lane];
                    }
            }
        }
    };
    // stream modes: step s of the wave's words to out
    auto emit = [&](const Words &W, uint32_t s) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k >= static_cast<int>(Kw)) break;
            const uint64_t o = o0 + 64ull * k + lane;
            if (o < o1) {
                u32x4 *dst = reinterpret_cast<u32x4 *>(a.out + 4 * (o + a.n * s));
                __builtin_nontemporal_store(box_muller_pairs4(W.q[k]), dst);
            }
        }
    };
    auto update = [&](const Words &W) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k >= static_cast<int>(Kw)) break;
            if (o0 + 64ull * k + lane < o1) {
                const u32x4 u = W.q[k];
                float gf[3];
                gaussian_forces(u.x, u.y, u.z, u.w, gf[0], gf[1], gf[2]);
                float *t = xv + k * 384;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float x = t[d * 64 + lane], v = t[(3 + d) * 64 + lane];
                    ld_update(a.coef, x, v, gf[d]);
                    t[d * 64 + lane] = x;
                    t[(3 + d) * 64 + lane] = v;
                }
            }
        }
    };
    Coord nxt{static_cast<int64_t>((4 * o0) / g.sl), static_cast<uint32_t>((4 * o0) % g.sl), 0u};
    nxt.lbase = lf_pad_base(a.pr, nxt.link);
    FlowWaits w;
    if constexpr (kPipe) {
        Words wa, wb;
        uint32_t seen = 0;
        if (a.n_steps > 0) {
            collect(w, nxt);
            if (!wait_all(w, lane, a)) return;
            load(wa, nxt);
            advance(nxt);
            if (a.n_steps > 1) {
                collect(w, nxt);
                seen = agent_load(lane < w.n ? w.flag : a.status);
            }
        }
        // Step s with its words X in flight (loaded after the producers published them) and, if
        // there is a step s+1, the poll of its producers issued after them: wait for X (and the
        // poll), and if the poll shows step s+1 published, issue its loads into Y and the poll of
        // step s+2 before the LD update of step s, else wait and load after it.  The loads of step
        // s+1 are issued before this wave publishes s+1, so their slots still hold them.
        auto step = [&](uint32_t s, Words &X, Words &Y) -> int {
            if (s >= a.n_steps) return 0;
            observe(s);
            const bool more = s + 1 < a.n_steps;
            // the builtin, unlike inline asm, is known to the compiler's wait insertion
            if (more) __builtin_amdgcn_s_waitcnt(kWaitVm1);
            else __builtin_amdgcn_s_waitcnt(kWaitVm0);
            fix(X);
            // X's registers pass through an empty asm statement: the compiler's wait insertion then
            // sees them written here, after their loads have returned, and does not hold the LD
            // update below for the loads of step s+1 issued in between
#pragma unroll
            for (int k = 0; k < KC; ++k) asm volatile("" : "+v"(X.q[k]));
            const bool ready = more && w.n <= 64u && __all(lane >= w.n || seen >= w.need);
            Coord far = nxt;
            advance(far);
            if (ready) {
                load(Y, nxt);
                if (s + 2 < a.n_steps) {
                    collect(w, far);
                    seen = agent_load(lane < w.n ? w.flag : a.status);
                }
            }
            // X's slots are free (published before any wait for step s+1)
            if (lane == 0) agent_store(a.cons + cw * kLfFlagStride, s + 1);
            if constexpr (MODE == kFlowLd)
                update(X);
            else
                emit(X, s);
            if (more && !ready) {
                collect(w, nxt);
                if (!wait_all(w, lane, a)) return -1;
                load(Y, nxt);
                if (s + 2 < a.n_steps) {
                    collect(w, far);
                    seen = agent_load(lane < w.n ? w.flag : a.status);
                }
            }
            nxt = far;
            return 1;
        };
        for (uint32_t s = 0;; s += 2) {
            int r = step(s, wa, wb);
            if (r > 0) r = step(s + 1, wb, wa);
            if (r < 0) return;
            if (r == 0) break;
        }
    } else {
        Words W;
        for (uint32_t s = 0; s < a.n_steps; ++s) {
            observe(s);
            // the producers of this step's positions (a few slices: one wait per lane)
            collect(w, nxt);
            if (!wait_all(w, lane, a)) return;
            load(W, nxt);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the loads have returned
            fix(W);
            // the step's slots are free
            if (lane == 0) agent_store(a.cons + cw * kLfFlagStride, s + 1);
            if constexpr (MODE == kFlowLd)
                update(W);
            else
                emit(W, s);
            advance(nxt);
        }
    }
    if constexpr (MODE != kFlowLd) return;
    float *t0buf = a.t0buf, *xo = a.x, *vo = a.v;
    asm volatile("" : "+s"(t0buf), "+s"(xo), "+s"(vo));
    if (a.stride && a.n_steps % a.stride == 0) {
#pragma unroll 1
        for (uint32_t k = 0; k < Kw; ++k) {
            const uint64_t o = o0 + 64ull * k + lane;
            tile_observe(a, t0buf, xv + k * 384, lane, o, o < o1, a.n_steps, cw * Kc + k);
        }
    }
#pragma unroll 1
    for (uint32_t k = 0; k < Kw; ++k) {
        const uint64_t o = o0 + 64ull * k + lane;
        if (o < o1)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xo[d * a.N + o] = xv[(k * 6 + d) * 64 + lane];
                vo[d * a.N + o] = xv[(k * 6 + 3 + d) * 64 + lane];
            }
    }
}

template <int KC, int MODE>
__global__ __launch_bounds__(kLfFlowBlock) void lf_pc_kernel(LfFlowArgs a) {
    extern __shared__ float flow_lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid < a.np) {
        lf_producer(a, __builtin_amdgcn_readfirstlane(blockIdx.x * a.np + wid), lane);
    } else {
        const uint32_t nc = kLfFlowBlock / 64 - a.np, k = wid - a.np;
        lf_consumer<KC, MODE>(a, __builtin_amdgcn_readfirstlane(blockIdx.x * nc + k), lane,
                        flow_lds + static_cast<size_t>(k) * a.geom.Kc * 384u);
    }
}

// the window before a persistent run: run positions -ll..-1 from the state's ring (slot
// hdr->slot is run position 0) into the run's ring
__global__ __launch_bounds__(kBulkBlock) void lf_pad_in_kernel(LfRing L, uint32_t *pring, LfPadRing pr) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= L.ll) return;
    const int64_t P = static_cast<int64_t>(i) - L.ll;
    // (slot + P) mod R with -ll <= P < 0 and ll <= R
    const uint64_t s = static_cast<uint64_t>(L.hdr->slot) + L.R - L.ll + i;
    pring[lf_pad_slot(pr, L.sl, P)] = L.ring[s >= L.R ? s - L.R : s];
}

// after the run: run positions Ptot - ll .. Ptot - 1 back into the state's ring, at the slots
// relative to run position 0 (still hdr->slot)
__global__ __launch_bounds__(kBulkBlock) void lf_pad_out_kernel(LfRing L, const uint32_t *pring, LfPadRing pr,
                                                                uint64_t Ptot) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= L.ll) return;
    const int64_t P = static_cast<int64_t>(Ptot) - L.ll + static_cast<int64_t>(i);
    int64_t s = (static_cast<int64_t>(L.hdr->slot) + P % static_cast<int64_t>(L.R)) % static_cast<int64_t>(L.R);
    if (s < 0) s += L.R;
    L.ring[s] = pring[lf_pad_slot(pr, L.sl, P)];
}

__global__ __launch_bounds__(kBulkBlock) void fill_u32_kernel(uint32_t *dst, uint64_t count, uint32_t value) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i < count) dst[i] = value;
}

template <int KC>
const void *lf_pc_fn() {
    return reinterpret_cast<const void *>(&lf_pc_kernel<KC, kFlowLd>);
}

template <int MODE>
const void *lf_stream_pc_fn(uint32_t kc) {
    switch (kc) {
        case 1: return reinterpret_cast<const void *>(&lf_pc_kernel<1, MODE>);
        case 2: return reinterpret_cast<const void *>(&lf_pc_kernel<2, MODE>);
        case 4: return reinterpret_cast<const void *>(&lf_pc_kernel<4, MODE>);
        default: return nullptr;
    }
}

const void *lf_pc_fn_for(uint32_t kc, int mode) {
    if (mode == kFlowGauss) return lf_stream_pc_fn<kFlowGauss>(kc);
    switch (kc) {
        case 1: return lf_pc_fn<1>();
        case 2: return lf_pc_fn<2>();
        case 4: return lf_pc_fn<4>();
        case 8: return lf_pc_fn<8>();
        default: return nullptr;
    }
}

inline dim3 grid_for(uint64_t n, int block = kBulkBlock) {
    return dim3(static_cast<unsigned>((n + block - 1) / block));
}

}  // namespace

hipError_t launch_lf_seed(void *state, uint32_t ll, uint32_t sl, uint32_t R, uint32_t W, uint64_t seed,
                          hipStream_t st) {
    LfHeader *hdr = static_cast<LfHeader *>(state);
    uint32_t *ring = reinterpret_cast<uint32_t *>(hdr + 1);
    lf_seed_kernel<<<grid_for(R), kBulkBlock, 0, st>>>(hdr, ring, ll, sl, R, W, seed);
    return hipGetLastError();
}

hipError_t launch_lf_uniform_phase(const LfRing &L, uint32_t *out, uint64_t first, uint32_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    lf_uniform_phase_kernel<<<grid_for(count), kBulkBlock, 0, st>>>(L, out, first, count);
    return hipGetLastError();
}

hipError_t launch_lf_ring_store(const LfRing &L, const uint32_t *out, uint64_t count, uint32_t base_mod,
                                hipStream_t st) {
    const uint32_t m = static_cast<uint32_t>(count < L.ll ? count : L.ll);
    if (m == 0) return hipSuccess;
    lf_ring_store_kernel<<<grid_for(m), kBulkBlock, 0, st>>>(L, out, count, m, base_mod);
    return hipGetLastError();
}

hipError_t launch_lf_gauss_phase(const LfRing &L, float *out, uint64_t first, uint32_t off_mod, uint32_t count,
                                 hipStream_t st) {
    const uint32_t pairs = count / 2;
    if (pairs == 0) return hipSuccess;
    lf_gauss_phase_kernel<<<grid_for(pairs), kBulkBlock, 0, st>>>(L, out, first, off_mod, pairs);
    return hipGetLastError();
}

hipError_t launch_lf_pad_in(const LfRing &L, uint32_t *pring, const LfPadRing &pr, hipStream_t st) {
    lf_pad_in_kernel<<<grid_for(L.ll), kBulkBlock, 0, st>>>(L, pring, pr);
    return hipGetLastError();
}

hipError_t launch_lf_pad_out(const LfRing &L, const uint32_t *pring, const LfPadRing &pr, uint64_t Ptot,
                             hipStream_t st) {
    lf_pad_out_kernel<<<grid_for(L.ll), kBulkBlock, 0, st>>>(L, pring, pr, Ptot);
    return hipGetLastError();
}

hipError_t launch_lf_discard_phase(const LfRing &L, uint32_t off_mod, uint32_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    lf_discard_phase_kernel<<<(count + kBulkBlock - 1) / kBulkBlock, kBulkBlock, 0, st>>>(L, off_mod, count);
    return hipGetLastError();
}

hipError_t launch_lf_advance(LfHeader *hdr, uint64_t count, uint32_t count_mod, hipStream_t st) {
    lf_advance_kernel<<<1, 64, 0, st>>>(hdr, count, count_mod);
    return hipGetLastError();
}

hipError_t launch_lf_ld_phase(const LfLdPhase &ph, hipStream_t st) {
    if (ph.osc_count == 0) return hipSuccess;
    lf_ld_phase_kernel<kLfLdBlock><<<grid_for(ph.osc_count, kLfLdBlock), kLfLdBlock, 0, st>>>(ph);
    return hipGetLastError();
}

hipError_t launch_lf_observe(const LfLdPhase &ph0, uint32_t n_phases, uint64_t phase_osc, uint32_t point,
                             bool t0_now, hipStream_t st) {
    const uint32_t bpp = static_cast<uint32_t>((phase_osc + kLfLdBlock - 1) / kLfLdBlock);
    if (bpp == 0 || n_phases == 0) return hipSuccess;
    lf_observe_kernel<kLfLdBlock><<<dim3(n_phases * bpp), kLfLdBlock, 0, st>>>(ph0, bpp, phase_osc, point, t0_now);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *dst, uint64_t count, uint32_t value, hipStream_t st) {
    if (count == 0) return hipSuccess;
    fill_u32_kernel<<<grid_for(count), kBulkBlock, 0, st>>>(dst, count, value);
    return hipGetLastError();
}

namespace {

// ---- persistent bare stream --------------------------------------------------------------------------
// One cooperative launch writes out[0, count) = y_{pos} .. y_{pos+count-1}; the output doubles as
// the lag table.  Producer p (one wave) owns offsets [p T, (p+1) T), T = 64 M, of every sl-long link
// (link j = positions [j sl, (j+1) sl) of the call); its short-lag source is its own number of the
// previous link, kept in registers, and its long-lag source y_{n-ll} is read from out, or for n < ll
// from the state's ring (the ll values before the call).  Nothing is overwritten, so the only waits
// are for the producers of the long-lag sources, which lie in earlier links or, when ll < 2 sl, in
// the same link of other producers; a producer publishes link j before it blocks on link j+1, so
// every wait is for work that is published before its producer blocks, and with all waves resident
// the run always progresses.

__device__ __forceinline__ bool stream_wait(FlowWaits &w, uint32_t lane, const LfStreamArgs &a) {
    bool ok = true;
    if (lane < w.n) {
        uint32_t spins = 0;
        while (agent_load(w.flag) < w.need) {
            if (++spins > a.spin_limit || ((spins & 15u) == 0 && agent_load(a.status) != 0u)) {
                agent_store(a.status, 1u);
                ok = false;
                break;
            }
            poll_pause(spins);
        }
    }
    w.n = 0;
    return __all(ok);
}

// Lane l of producer p holds the offsets 4 (l + 64 g) + r of its slice, g < M / 4, r < 4: four
// consecutive words, moved with one 16-byte buffer access (sc1, as the ring of the fused run) wherever
// the four lie inside the slice's valid part and, for loads, inside the output; word by word
// otherwise (the first links, whose long-lag sources are in the state's ring, and ragged ends).
// Software-pipelined over links: when the waits of link j+1 are already seen to hold, link j's stores
// are followed at once by the poll for link j+2 and link j+1's loads, and link j is published as soon
// as only those can still be outstanding (vector memory operations complete in issue order, and a
// store counts until it has completed); otherwise link j is published first, then the producer blocks
// on link j+1's waits.
// (A Gaussian variant that kept the integers in a ring and wrote each pair to the output from the
// producers ran at 2.8e11 values/s against the uint32 stream's 5e11: the output stores complete in
// issue order with the ring stores, so every link's publication waited for the previous link's
// output writes.  Long Gaussian streams take the producer/consumer run instead, whose consumers
// write the pairs.)

template <int M>
__global__ __launch_bounds__(kLfFlowBlock) void lf_stream_kernel(LfStreamArgs a) {
    static_assert(M % 4 == 0, "groups of four words");
    constexpr int G = M / 4;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t p = __builtin_amdgcn_readfirstlane(blockIdx.x * (kLfFlowBlock / 64) + (threadIdx.x >> 6));
    if (p >= a.n_slices) return;
    constexpr uint32_t T = 64u * M;
    const LfFlowGeom &g = a.geom;
    const uint32_t sl = g.sl, o_lo = p * T;
    const uint32_t width = T < sl - o_lo ? T : sl - o_lo;
    const uint64_t count = g.Ptot;
    uint32_t *out = a.out;
    const uint32_t *ring = a.L.ring;
    const uint32_t R = a.L.R, ll = a.L.ll;
    const uint32_t slot0 = a.L.hdr->slot;  // ring slot of y_{pos}
    // the word holding y_{pos + P}: out for P >= 0, the ring for -ll <= P < 0
    auto word = [&](int64_t P) -> const uint32_t * {
        if (P >= 0) return out + P;
        int64_t s = static_cast<int64_t>(slot0) + P;
        if (s < 0) s += R;
        return ring + s;
    };
    auto link_len = [&](uint32_t j) -> uint32_t {
        if (j >= a.n_links) return 0u;
        const uint64_t n0 = static_cast<uint64_t>(j) * sl + o_lo;
        return n0 >= count ? 0u : (count - n0 < width ? static_cast<uint32_t>(count - n0) : width);
    };
    auto q_of = [&](int gi, int r) -> uint32_t { return 4u * (lane + 64u * gi) + r; };
    u32x4 chain[G], src[G];
#pragma unroll
    for (int gi = 0; gi < G; ++gi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t q = q_of(gi, r);
            chain[gi][r] = q < width ? agent_load(word(static_cast<int64_t>(o_lo + q) - sl)) : 0u;
        }
    FlowWaits w;
    w.n = 0;
    // the producers of link j's long-lag sources (positions >= 0 only)
    auto collect = [&](uint32_t j, uint32_t len) {
        int64_t link;
        uint32_t off;
        lf_back(j, o_lo, LfLag{a.lla, a.llb}, sl, link, off);
        lf_walk_producers(g, link, off, len, [&](uint32_t slice, uint32_t l) {
            wait_add(w, lane, a.prod + slice * kLfFlagStride, l + 1, 0);
            return true;
        });
    };
    // link j's long-lag sources y_{n - ll}, n = j sl + o_lo + q.  With every source in the output
    // (j sl + o_lo >= ll) the slice's whole window of T sources is read, 16 bytes per group: it lies
    // inside the output (it ends before position j sl + o_lo); values past len are not used.
    auto load = [&](uint32_t j, uint32_t len, u32x4 (&dst)[G]) {
        const int64_t base = static_cast<int64_t>(j) * sl + o_lo - ll;
        if (base >= 0) {
            const __amdgpu_buffer_rsrc_t rs = ring_rsrc(out + base, T);
#pragma unroll
            for (int gi = 0; gi < G; ++gi) dst[gi] = ring_get4(rs, 4u * (lane + 64u * gi));
        } else {
#pragma unroll
            for (int gi = 0; gi < G; ++gi)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t q = q_of(gi, r);
                    dst[gi][r] = agent_load(word(base + (q < len ? q : 0u)));
                }
        }
    };
    // link j's values chain into out[j sl + o_lo + q], q < len
    auto store = [&](uint32_t j, uint32_t len) {
        uint32_t *dst = out + static_cast<uint64_t>(j) * sl + o_lo;
        const __amdgpu_buffer_rsrc_t rs = ring_rsrc(dst, T);
#pragma unroll
        for (int gi = 0; gi < G; ++gi) {
            const uint32_t q0 = 4u * (lane + 64u * gi);
            if (q0 + 4u <= len) {
                ring_put4(rs, q0, chain[gi]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (q0 + r < len) agent_store(dst + q0 + r, chain[gi][r]);
            }
        }
    };
    uint32_t len = link_len(0);
    if (len == 0) return;
    collect(0, len);
    if (!stream_wait(w, lane, a)) return;
    // one read of the first progress word each lane waits for (the status word in lanes without a
    // wait), for link j1
    uint32_t seen = 0;
    auto poll = [&](uint32_t j1) {
        w.n = 0;
        collect(j1, link_len(j1));
        seen = agent_load(lane < w.n ? w.flag : a.status);
    };
    poll(1);
    load(0, len, src);
    for (uint32_t j = 0; j < a.n_links; ++j) {
        const uint32_t next_len = link_len(j + 1);
#pragma unroll
        for (int gi = 0; gi < G; ++gi) chain[gi] += src[gi];
        // link j+1's waits, as read by the last poll (before link j's loads)
        const bool ready = next_len > 0 && w.n <= 64u && __all(lane >= w.n || seen >= w.need);
        store(j, len);
        if (!ready) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (lane == 0) agent_store(a.prod + p * kLfFlagStride, j + 1);
            if (!next_len) break;
            // link j+1's waits, in full (a link's sources span at most two slices of each of two
            // links, so they fit the 64 lanes)
            w.n = 0;
            collect(j + 1, next_len);
            if (!stream_wait(w, lane, a)) return;
        }
        poll(j + 2);
        const bool fast = static_cast<int64_t>(j + 1) * sl + o_lo >= static_cast<int64_t>(ll);
        load(j + 1, next_len, src);
        if (ready) {
            // only the poll and link j+1's loads, issued after link j's stores, may still be
            // outstanding (vector memory operations complete in issue order): link j is stored
            if (fast)
                asm volatile("s_waitcnt vmcnt(%0)" ::"n"(G + 1) : "memory");
            else
                asm volatile("s_waitcnt vmcnt(%0)" ::"n"(M + 1) : "memory");
            if (lane == 0) agent_store(a.prod + p * kLfFlagStride, j + 1);
        }
        len = next_len;
    }
}

}  // namespace

hipError_t launch_lf_stream(const LfStreamArgs &a, uint32_t grid, uint32_t m, hipStream_t st) {
    const void *fn = nullptr;
    if (m == 4) fn = reinterpret_cast<const void *>(&lf_stream_kernel<4>);
    else if (m == 16) fn = reinterpret_cast<const void *>(&lf_stream_kernel<16>);
    else return hipErrorInvalidValue;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kLfFlowBlock, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
    LfStreamArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kLfFlowBlock), args, 0, st);
}

hipError_t launch_lf_flow(const LfFlowArgs &a, uint32_t grid, uint32_t kc, uint32_t lds, hipStream_t st, int mode) {
    const void *fn = lf_pc_fn_for(kc, mode);
    if (!fn) return hipErrorInvalidValue;
    // allow more than 64 KiB of dynamic LDS where the runtime asks for it; the occupancy query
    // below decides whether the block fits
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        (void)hipGetLastError();
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kLfFlowBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
    LfFlowArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kLfFlowBlock), args, lds, st);
}

}  // namespace rngld
