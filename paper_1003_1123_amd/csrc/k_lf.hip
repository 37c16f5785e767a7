// k_lf.hip -- additive lagged Fibonacci, one generator shared by all threads (Sec. III.C; Alg. 3).
//
// y_n = y_{n-ll} + y_{n-sl} mod 2^32 (Eq. 3).  The state is a ring of R >= ll + W words in device
// memory.  A "wave" computes W <= sl consecutive positions concurrently: every source is at least
// sl positions back, so it belongs to an earlier wave, and no write of the wave overwrites a value
// a later reader still needs (R >= ll + W).  Waves are separated by kernel boundaries, which on
// gfx950 also make each wave's writes visible across all XCDs' L2 caches.  This is the
// device-wide "synchronisation at the end of each step" of Sec. III.A, at wave granularity, and
// it reproduces the one sequential sequence for any wave width (the paper's Table I rows do not
// satisfy its own race-free condition ll - sl > RNS N; the ring removes that condition).
#include "internal.hpp"

namespace rngld {

namespace {

__device__ __forceinline__ uint32_t wrap_once(uint32_t s, uint32_t R) { return s >= R ? s - R : s; }
// slot - lag for lag <= R (slot < R)
__device__ __forceinline__ uint32_t back(uint32_t slot, uint32_t lag, uint32_t R) {
    return slot >= lag ? slot - lag : slot + (R - lag);
}

// window y_{-ll+i} = LCG^{i+1}(x0) in slots 0..ll-1, position 0 at slot ll; other slots zero
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
    uint32_t a, b;
    if (i >= L.ll)
        a = out[i - L.ll];
    else
        a = L.ring[back(base, L.ll - static_cast<uint32_t>(i), L.R)];
    if (i >= L.sl)
        b = out[i - L.sl];
    else
        b = L.ring[back(base, L.sl - static_cast<uint32_t>(i), L.R)];
    out[i] = a + b;
}

// after a bulk call: the last min(count, ll) outputs become the ring's newest values
__global__ __launch_bounds__(kBulkBlock) void lf_ring_store_kernel(LfRing L, const uint32_t *out, uint64_t count,
                                                                   uint32_t m, uint32_t base_mod) {
    const uint32_t t = blockIdx.x * kBulkBlock + threadIdx.x;
    if (t >= m) return;
    const uint32_t slot = wrap_once(wrap_once(L.hdr->slot + base_mod, L.R) + t, L.R);
    L.ring[slot] = out[count - m + t];
}

// one wave of rng_gaussian: positions off_mod + 2t, +1 (ring slots relative to pos0's slot)
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

__global__ void lf_advance_kernel(LfHeader *hdr, uint64_t count, uint32_t count_mod) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        hdr->pos += count;
        uint32_t s = hdr->slot + count_mod;
        hdr->slot = s >= hdr->R ? s - hdr->R : s;
    }
}

// one phase of an LD step: thread t owns oscillator osc_begin + t and positions 4t..4t+3 of the
// phase (Alg. 3: thread j takes y_{(j + N t) RNS + r}); the observables of the step's starting
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

// observables of the final state, with the same tiling as the phases (one tile per phase block)
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
// One cooperative launch runs every LD step.  Block g owns tiles c = g, g + G, ... of every step (a
// tile = 256 oscillators = 1024 consecutive positions) and keeps their x, v in registers.  It
// processes its tiles in sequence order; before a tile it waits until the tiles holding the
// tile's sources (positions sl and ll back) have been completed, then generates the tile's 1024
// numbers into the ring, updates its oscillators and publishes progress[c] = step + 1.
//  * No deadlock: dependencies point to earlier positions, each block handles its tiles in
//    position order, and all blocks are co-resident (cooperative launch), so the earliest
//    unfinished tile can always run.
//  * No ring hazard: with R = ll + sl, slot(p) holds p - ll - sl, whose only readers are the
//    positions p - sl and p - ll -- exactly the sources this tile waits for.  Any schedule the
//    flags allow therefore reproduces the sequential sequence.
//  * Visibility across the 8 XCDs' (mutually non-coherent) L2 caches: every access to the shared
//    ring is a device-scope (agent) access, so ring stores write through to the device coherence
//    point and ring loads read from it, never from a stale XCD L2 line.  A producer waits for its
//    block's ring stores to complete (s_waitcnt, then a block barrier) before storing the
//    progress flag; a consumer observes the flag before a block barrier and only then issues its
//    ring loads.  This avoids agent-scope release/acquire fences, which write back / invalidate
//    a whole XCD L2 each time and made every tile cost tens of microseconds.
//  * Every wait is bounded: after spin_limit polls, or when another block has given up, the
//    block stops, and status[0] records the failure.
__device__ __forceinline__ uint32_t ring_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ring_store(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool lf_wait_progress(uint32_t *progress, uint32_t c, uint32_t need, uint32_t *status,
                                                 uint32_t spin_limit) {
    uint32_t spins = 0;
    while (__hip_atomic_load(progress + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++spins > spin_limit ||
            __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
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
    if (tid == 0) s_abort = 0u;
    uint32_t slot_s = a.L.hdr->slot;  // ring slot of the current step's first position
    __syncthreads();
    bool stop = false;
    for (uint32_t s = 0; s < a.n_steps && !stop; ++s) {
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t c = g + k * G;
            if (c >= Ct) break;
            const uint64_t first = static_cast<uint64_t>(c) * BLOCK;
            const uint32_t count = static_cast<uint32_t>(first + BLOCK <= a.n ? BLOCK : a.n - first);
            // the first wave polls the tile's source tiles in parallel, lane i the i-th of them
            if (tid < 64) {
                uint32_t idx = 0, my_c = 0, my_need = 0;
                lf_tile_sources(a.geom, s, c, count, [&](uint32_t s2, uint32_t c2) {
                    if (idx == tid) {
                        my_c = c2;
                        my_need = s2 + 1;
                    }
                    ++idx;
                    return true;
                });
                if (tid < idx && !lf_wait_progress(a.progress, my_c, my_need, a.status, a.spin_limit))
                    s_abort = 1u;
            }
            __syncthreads();
            if (s_abort) {
                stop = true;
                break;
            }
            const bool act = tid < count;
            const uint64_t o = first + tid;
            float x[3], v[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x[d] = xv[k][d][tid];
                v[d] = xv[k][3 + d][tid];
            }
            if (a.stride && s == a.t0 && act)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    a.t0buf[d * a.N + o] = x[d];
                    a.t0buf[(3 + d) * a.N + o] = v[d];
                }
            if (a.stride && s % a.stride == 0) {
                double q[6] = {0, 0, 0, 0, 0, 0};
                if (act) {
                    float x0[3] = {0, 0, 0}, v0[3] = {0, 0, 0};
                    if (s >= a.t0)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            x0[d] = s == a.t0 ? x[d] : a.t0buf[d * a.N + o];
                            v0[d] = s == a.t0 ? v[d] : a.t0buf[(3 + d) * a.N + o];
                        }
                    add_observables(q, x, v, x0, v0, s >= a.t0);
                }
                block_sum6<BLOCK>(q, red, a.partials + (static_cast<uint64_t>(s / a.stride) * a.pstride + c) * 6);
            }
            // generate the tile's 4 count numbers: lane t takes positions t + 256 r (each load and
            // store instruction is contiguous across the wave); all loads are issued before any
            // store, which is safe because sl >= 1024 keeps every source outside the tile
            {
                const uint32_t base = wrap_once(slot_s + s_toff[k], R);
                uint32_t sa[4], sb[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t q = r * BLOCK + tid;
                    if (q < 4 * count) {
                        const uint32_t slot = wrap_once(base + q, R);
                        sa[r] = ring_load(a.L.ring + back(slot, a.L.ll, R));
                        sb[r] = ring_load(a.L.ring + back(slot, a.L.sl, R));
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t q = r * BLOCK + tid;
                    if (q < 4 * count) {
                        const uint32_t w = sa[r] + sb[r];
                        ring_store(a.L.ring + wrap_once(base + q, R), w);
                        words[q] = w;
                    }
                }
            }
            __syncthreads();  // words[] complete: oscillator t's four words are words[4t .. 4t+3]
            if (act) {
                const uint32_t *w = words + 4 * tid;
                float gf[3];
                gaussian_forces(w[0], w[1], w[2], w[3], gf[0], gf[1], gf[2]);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    ld_update(a.coef, x[d], v[d], gf[d]);
                    xv[k][d][tid] = x[d];
                    xv[k][3 + d][tid] = v[d];
                }
            }
            __builtin_amdgcn_s_waitcnt(0);  // this wave's ring stores have completed
            __syncthreads();                // ... and so have every other wave's
            if (tid == 0) __hip_atomic_store(a.progress + c, s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        slot_s = wrap_once(slot_s + a.step_adv, R);
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
