// k_lf.hip -- additive lagged Fibonacci, one generator shared by all threads (Sec. III.C; Alg. 3).
//
// y_n = y_{n-ll} + y_{n-sl} mod 2^32 (Eq. 3).  The state is a ring of R >= ll + W 64-bit slots in
// device memory; slot (slot0 + n - pos) mod R holds y_n in its low half and the low 32 bits of n
// (its "tag") in its high half, written by one 64-bit store.  The tags let a consumer recognise
// whether a slot already holds the position it needs, which the persistent dataflow run relies on.
//
// Two ways to run the dependency structure (a position needs the positions sl and ll back):
//  * waves: W <= sl consecutive positions per launch; every source is in an earlier wave; kernel
//    boundaries order the waves and make their writes visible across the XCDs' L2 caches.  This is
//    the device-wide "synchronisation at the end of each step" of Sec. III.A at wave granularity.
//    (Table I rows do not satisfy the paper's race-free condition ll - sl > RNS N; the ring removes
//    that condition.)
//  * dataflow (fused LD runs, R = ll + sl): one persistent launch; each tile of 1024 positions
//    waits only for the tags of its own sources (see lf_ld_flow_kernel).
// Both reproduce the one sequential sequence exactly, for any wave width or schedule.
#include "internal.hpp"

namespace rngld {

namespace {

__device__ __forceinline__ uint32_t wrap_once(uint32_t s, uint32_t R) { return s >= R ? s - R : s; }
// slot - lag for lag <= R (slot < R)
__device__ __forceinline__ uint32_t back(uint32_t slot, uint32_t lag, uint32_t R) {
    return slot >= lag ? slot - lag : slot + (R - lag);
}
__device__ __forceinline__ uint64_t pack(uint32_t value, uint32_t tag) {
    return static_cast<uint64_t>(value) | (static_cast<uint64_t>(tag) << 32);
}
__device__ __forceinline__ uint32_t value_of(uint64_t s) { return static_cast<uint32_t>(s); }
__device__ __forceinline__ uint32_t tag_of(uint64_t s) { return static_cast<uint32_t>(s >> 32); }

// window y_{-ll+i} = LCG^{i+1}(x0) in slots 0..ll-1 (position 0 at slot ll); the other slots get
// tags one lap back, which no position of the run will ever expect
__global__ __launch_bounds__(kBulkBlock) void lf_seed_kernel(LfHeader *hdr, uint64_t *ring, uint32_t ll,
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
    const int64_t position = static_cast<int64_t>(i) - ll - (i < ll ? 0 : static_cast<int64_t>(R));
    ring[i] = pack(i < ll ? lcg_skip(x0, i + 1) : 0u, static_cast<uint32_t>(position));
}

// one wave of rng_uniform: out[first + t] = y_{pos0 + first + t}; sources at or after pos0 come
// from out itself (the output doubles as the lag table), earlier ones from the ring
__global__ __launch_bounds__(kBulkBlock) void lf_uniform_phase_kernel(LfRing L, uint32_t *out, uint64_t first,
                                                                      uint32_t count) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= count) return;
    const uint64_t i = first + t;
    const uint32_t base = L.hdr->slot;
    const uint32_t a = i >= L.ll ? out[i - L.ll] : value_of(L.ring[back(base, L.ll - static_cast<uint32_t>(i), L.R)]);
    const uint32_t b = i >= L.sl ? out[i - L.sl] : value_of(L.ring[back(base, L.sl - static_cast<uint32_t>(i), L.R)]);
    out[i] = a + b;
}

// after a bulk call: the last min(count, ll) outputs become the ring's newest values
__global__ __launch_bounds__(kBulkBlock) void lf_ring_store_kernel(LfRing L, const uint32_t *out, uint64_t count,
                                                                   uint32_t m, uint32_t base_mod) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= m) return;
    const uint32_t slot = wrap_once(wrap_once(L.hdr->slot + base_mod, L.R) + t, L.R);
    const uint64_t i = count - m + t;
    L.ring[slot] = pack(out[i], static_cast<uint32_t>(L.hdr->pos + i));
}

// one wave of rng_gaussian: positions first + 2t, +1 (ring slots off_mod + 2t, +1 from pos0's)
__global__ __launch_bounds__(kBulkBlock) void lf_gauss_phase_kernel(LfRing L, float *out, uint64_t first,
                                                                    uint32_t off_mod, uint32_t pairs) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= pairs) return;
    const uint32_t s0 = wrap_once(wrap_once(L.hdr->slot + off_mod, L.R) + 2 * t, L.R);
    const uint32_t s1 = wrap_once(s0 + 1, L.R);
    const uint32_t w0 = value_of(L.ring[back(s0, L.ll, L.R)]) + value_of(L.ring[back(s0, L.sl, L.R)]);
    const uint32_t w1 = value_of(L.ring[back(s1, L.ll, L.R)]) + value_of(L.ring[back(s1, L.sl, L.R)]);
    const uint32_t tag0 = static_cast<uint32_t>(L.hdr->pos + first + 2 * t);
    L.ring[s0] = pack(w0, tag0);
    L.ring[s1] = pack(w1, tag0 + 1);
    const float r = box_muller_radius(w0);
    float c, s;
    box_muller_angle(w1, c, s);
    out[first + 2 * t] = r * c;
    out[first + 2 * t + 1] = r * s;
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
    const uint32_t tag0 = static_cast<uint32_t>(ph.L.hdr->pos + ph.pos_rel) + 4 * t;
    uint32_t w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        w[r] = value_of(ph.L.ring[back(slot, ph.L.ll, R)]) + value_of(ph.L.ring[back(slot, ph.L.sl, R)]);
        ph.L.ring[slot] = pack(w[r], tag0 + r);
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

// ---- persistent dataflow run ----------------------------------------------------------------------
// One cooperative launch runs every LD step.  Block g owns tiles c = g, g + G, ... of every step
// (a tile = 256 oscillators = 1024 consecutive positions) and keeps their x, v in LDS.  It handles
// its tiles in sequence order.  For a tile, lane t takes positions t + 256 r: it loads the two
// source slots of each, and re-loads any whose tag is not yet the expected position, until all
// sources are present; then it stores the tile's numbers with their tags and, after an LDS
// transpose, oscillator t's four words drive its Box-Muller forces and LD update.
//  * No flags and no fences: a slot's tag says whether it holds the position a reader needs.
//    Ring accesses are device-scope (agent) loads and stores, so they bypass the XCDs' mutually
//    non-coherent L2 caches; a 64-bit slot is written and read in one access.
//  * No ring hazard (R = ll + sl): slot(p) previously held p - ll - sl, read only by positions
//    p - sl and p - ll.  Position p is written only after their tags were seen, and each of them
//    was stored only after its own sources (p - ll - sl among them) had been loaded.  Symmetrically,
//    the slots read for p can be rewritten only by p + ll and p + sl, whose producers must first
//    see position p itself.
//  * No deadlock: every source lies >= sl >= 1024 positions back, so outside the tile; blocks run
//    their tiles in position order and are all co-resident (cooperative launch), so the earliest
//    unfinished tile always has its sources and can run.
//  * Every wait is bounded: after spin_limit polls, or once another block has given up, a lane
//    stops waiting, status[0] is set and the run stops (its results are then invalid).
__device__ __forceinline__ uint64_t ring_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ring_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int BLOCK, int KMAX>
__global__ __launch_bounds__(BLOCK) void lf_ld_flow_kernel(LfFlowArgs a) {
    // x, v of the block's tiles stay on chip in LDS ([tile][component][lane], conflict-free), so
    // the register count does not grow with the tiles a block owns; x(t0), v(t0) live in t0buf
    __shared__ float xv[KMAX][6][BLOCK];
    __shared__ uint32_t words[4 * BLOCK];  // the current tile's numbers, in sequence order
    __shared__ double red[BLOCK / 64][6];
    __shared__ uint32_t s_abort;
    __shared__ uint32_t s_toff[KMAX];  // (4 B c) mod R of the block's k-th tile
    const uint32_t G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const uint32_t R = a.L.R, Ct = a.geom.n_ctiles;
    if (tid == 0) {
        uint32_t off = static_cast<uint32_t>((4ull * BLOCK * g) % R);
        const uint32_t step = static_cast<uint32_t>((4ull * BLOCK * G) % R);
        for (int k = 0; k < KMAX; ++k) {
            s_toff[k] = off;
            off = wrap_once(off + step, R);
        }
        s_abort = 0u;
    }
    for (int k = 0; k < KMAX; ++k) {
        const uint32_t c = g + k * G;
        const uint64_t o = static_cast<uint64_t>(c) * BLOCK + tid;
        const bool act = c < Ct && o < a.n;
        for (int d = 0; d < 3; ++d) {
            xv[k][d][tid] = act ? a.x[d * a.N + o] : 0.0f;
            xv[k][3 + d][tid] = act ? a.v[d * a.N + o] : 0.0f;
        }
    }
    uint32_t slot_s = a.L.hdr->slot;                        // ring slot of the step's first position
    uint32_t tag_s = static_cast<uint32_t>(a.L.hdr->pos);  // low 32 bits of that position
    const uint32_t tag_adv = static_cast<uint32_t>(a.geom.four_n);
    __syncthreads();
    bool stop = false;
    for (uint32_t s = 0; s < a.n_steps && !stop; ++s) {
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t c = g + k * G;
            if (c >= Ct) break;
            const uint64_t first = static_cast<uint64_t>(c) * BLOCK;
            const uint32_t count = static_cast<uint32_t>(first + BLOCK <= a.n ? BLOCK : a.n - first);
            const bool act = tid < count;
            const uint64_t o = first + tid;
            if (a.stride && s % a.stride == 0) {  // observables of the tile's state before this step
                double q[6] = {0, 0, 0, 0, 0, 0};
                if (act) {
                    float x[3], v[3], x0[3] = {0, 0, 0}, v0[3] = {0, 0, 0};
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        x[d] = xv[k][d][tid];
                        v[d] = xv[k][3 + d][tid];
                        if (s >= a.t0) {
                            x0[d] = s == a.t0 ? x[d] : a.t0buf[d * a.N + o];
                            v0[d] = s == a.t0 ? v[d] : a.t0buf[(3 + d) * a.N + o];
                        }
                    }
                    add_observables(q, x, v, x0, v0, s >= a.t0);
                }
                block_sum6<BLOCK>(q, red, a.partials + (static_cast<uint64_t>(s / a.stride) * a.pstride + c) * 6);
            }
            if (a.stride && s == a.t0 && act)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    a.t0buf[d * a.N + o] = xv[k][d][tid];
                    a.t0buf[(3 + d) * a.N + o] = xv[k][3 + d][tid];
                }
            // the tile's 4 count numbers: lane t takes positions q = t + 256 r
            {
                const uint32_t base = wrap_once(slot_s + s_toff[k], R);
                const uint32_t tag0 = tag_s + static_cast<uint32_t>(4ull * BLOCK * c);
                uint32_t src_l[4], src_s[4];
                uint64_t vl[4], vs[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t q = r * BLOCK + tid;
                    if (q < 4 * count) {
                        const uint32_t slot = wrap_once(base + q, R);
                        src_l[r] = back(slot, a.L.ll, R);
                        src_s[r] = back(slot, a.L.sl, R);
                        vl[r] = ring_load(a.L.ring + src_l[r]);
                        vs[r] = ring_load(a.L.ring + src_s[r]);
                    }
                }
                bool ok = true;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t q = r * BLOCK + tid;
                    if (ok && q < 4 * count) {
                        const uint32_t want_l = tag0 + q - a.L.ll, want_s = tag0 + q - a.L.sl;
                        uint32_t spins = 0;
                        while (tag_of(vl[r]) != want_l || tag_of(vs[r]) != want_s) {
                            if (++spins > a.spin_limit ||
                                __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                                __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                ok = false;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            if (tag_of(vl[r]) != want_l) vl[r] = ring_load(a.L.ring + src_l[r]);
                            if (tag_of(vs[r]) != want_s) vs[r] = ring_load(a.L.ring + src_s[r]);
                        }
                        if (ok) {
                            const uint32_t w = value_of(vl[r]) + value_of(vs[r]);
                            ring_store(a.L.ring + wrap_once(base + q, R), pack(w, tag0 + q));
                            words[q] = w;
                        }
                    }
                }
                if (!ok) s_abort = 1u;
            }
            __syncthreads();  // words[] complete: oscillator t's four words are words[4t .. 4t+3]
            if (s_abort) {
                stop = true;
                break;
            }
            if (act) {
                const uint32_t *w = words + 4 * tid;
                float gf[3];
                gaussian_forces(w[0], w[1], w[2], w[3], gf[0], gf[1], gf[2]);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float x = xv[k][d][tid], v = xv[k][3 + d][tid];
                    ld_update(a.coef, x, v, gf[d]);
                    xv[k][d][tid] = x;
                    xv[k][3 + d][tid] = v;
                }
            }
            __syncthreads();  // words[] is free for the next tile
        }
        slot_s = wrap_once(slot_s + a.step_adv, R);
        tag_s += tag_adv;
    }
    if (!stop && a.stride && a.n_steps % a.stride == 0) {
        const uint32_t s = a.n_steps;
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t c = g + k * G;
            if (c >= Ct) break;
            const uint64_t o = static_cast<uint64_t>(c) * BLOCK + tid;
            double q[6] = {0, 0, 0, 0, 0, 0};
            if (o < a.n) {
                float x[3], v[3], x0[3], v0[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x[d] = xv[k][d][tid];
                    v[d] = xv[k][3 + d][tid];
                    x0[d] = s == a.t0 ? x[d] : a.t0buf[d * a.N + o];
                    v0[d] = s == a.t0 ? v[d] : a.t0buf[(3 + d) * a.N + o];
                }
                add_observables(q, x, v, x0, v0, s >= a.t0);
            }
            block_sum6<BLOCK>(q, red, a.partials + (static_cast<uint64_t>(s / a.stride) * a.pstride + c) * 6);
        }
    }
    for (int k = 0; k < KMAX; ++k) {
        const uint32_t c = g + k * G;
        const uint64_t o = static_cast<uint64_t>(c) * BLOCK + tid;
        if (c < Ct && o < a.n)
            for (int d = 0; d < 3; ++d) {
                a.x[d * a.N + o] = xv[k][d][tid];
                a.v[d * a.N + o] = xv[k][3 + d][tid];
            }
    }
}

__global__ __launch_bounds__(kBulkBlock) void fill_u32_kernel(uint32_t *dst, uint64_t count, uint32_t value) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i < count) dst[i] = value;
}

template <int KMAX>
const void *lf_flow_fn() {
    return reinterpret_cast<const void *>(&lf_ld_flow_kernel<(1 << kLfFlowBlockLog2), KMAX>);
}

const void *lf_flow_fn_for(uint32_t kmax) {
    switch (kmax) {
        case 1: return lf_flow_fn<1>();
        case 2: return lf_flow_fn<2>();
        case 4: return lf_flow_fn<4>();
        case 8: return lf_flow_fn<8>();
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
    uint64_t *ring = reinterpret_cast<uint64_t *>(hdr + 1);
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

uint32_t lf_flow_max_grid(uint32_t kmax) {
    const void *fn = lf_flow_fn_for(kmax);
    if (!fn) return 0;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 1 << kLfFlowBlockLog2, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return static_cast<uint32_t>(per_cu) * static_cast<uint32_t>(cus);
}

hipError_t launch_lf_flow(const LfFlowArgs &a, uint32_t grid, uint32_t kmax, hipStream_t st) {
    const void *fn = lf_flow_fn_for(kmax);
    if (!fn) return hipErrorInvalidValue;
    LfFlowArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(1 << kLfFlowBlockLog2), args, 0, st);
}

}  // namespace rngld
