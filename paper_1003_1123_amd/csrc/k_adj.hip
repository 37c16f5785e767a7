// k_adj.hip -- pathwise reverse-mode gradients of an LD loss w.r.t. (k, gamma, kT).
//
// Not in the paper; it differentiates the paper's LD model (Sec. I, Sec. IV) with the noise held
// fixed.  Underdamped semi-implicit step per component, z = (x, v):
//     v' = c v - kap x + sig g,  x' = x + h v'.
// With mu = lam_v' + h lam_x' (adjoints of the step's outputs), one reverse step is
//     lam_x = lam_x' - kap mu + dL/dx,  lam_v = c mu,
//     dL/dtheta += mu (dc/dtheta v - dkap/dtheta x + dsig/dtheta g).
// The forward kernel writes (x, v, generator state) every K steps and at the end.  The backward
// kernels walk the segments last to first, in one of two ways per ensemble:
//  * register-only (Hybrid Taus): start from the checkpoint at the segment's end and step both
//    the generator (inverse Tausworthe and LCG steps, so the noise is bit-identical) and the
//    integrator backward, x = x' - h v', v = (v' + kap x - sig g) / c, while sweeping the adjoint;
//    the next segment restarts from its own end checkpoint, which bounds the growth of rounding
//    errors in the reconstructed path to K steps (the host admits an ensemble only if that growth
//    stays small).  Nothing is stored.
//  * replay: restore the checkpoint at the segment's start, rerun the segment with the same
//    generator, Box-Muller and update code, keep its path in a per-thread scratch column, and
//    sweep it backward.
// Gradients accumulate in FP64 per thread and reduce in a fixed order (no atomics).
#include <type_traits>

#include "internal.hpp"

namespace rngld {

namespace {

template <class Gen>
struct IsRan2A : std::false_type {};
template <>
struct IsRan2A<Ran2> : std::true_type {};

template <class Gen>
__device__ __forceinline__ void bind_tab(Gen &g, int32_t *lds, int tid, int block) {
    if constexpr (IsRan2A<Gen>::value) {
        g.tab = lds + tid;
        g.tstride = block;
    }
}
template <class Gen>
__device__ __forceinline__ void park(Gen &g) {
    if constexpr (IsRan2A<Gen>::value) {
        g.idum = g.idum2 = g.iy = 1;
        for (int t = 0; t < kR2Tab; ++t) g.tab[t * g.tstride] = 1;
    } else {
        g.t1 = g.t2 = g.t3 = g.lcg = 0x9E3779B9u;
    }
}
template <class Gen>
__device__ __forceinline__ void load_state(Gen &g, const void *st, uint64_t S, uint64_t j) {
    if constexpr (IsRan2A<Gen>::value)
        g.load(static_cast<const int32_t *>(st), S, j);
    else
        g.load(static_cast<const uint32_t *>(st), S, j);
}
template <class Gen>
__device__ __forceinline__ void store_state(const Gen &g, void *st, uint64_t S, uint64_t j) {
    if constexpr (IsRan2A<Gen>::value)
        g.store(static_cast<int32_t *>(st), S, j);
    else
        g.store(static_cast<uint32_t *>(st), S, j);
}

__device__ __forceinline__ uint32_t find_ensemble(const EnsDev *ens, uint32_t n_ens, uint32_t tile) {
    uint32_t lo = 0, hi = n_ens - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (ens[mid].tile_begin <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// reduce up to three FP64 values per thread into partial[tile][0..2]
template <int BLOCK>
__device__ __forceinline__ void block_sum3(const double (&q)[3], double (*red)[3], double *dst) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double s = wave_sum(q[i]);
        if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
    __syncthreads();
}

// forward run from the current state with checkpoints every K steps; loss partial = sum of x^2
// over the loss window (scaled on finalisation)
template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_ckpt_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];
    __shared__ double red[BLOCK / 64][3];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const LdCoef q = a.adj[e].f;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    Gen g;
    bind_tab(g, lds, threadIdx.x, BLOCK);
    float x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    if (act) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = a.x[d * a.NT + i];
            v[d] = a.v[d * a.NT + i];
        }
        load_state(g, a.state, a.S, i);
    } else {
        park(g);
    }
    double lsum = 0.0;
    for (uint32_t s = 0; s < a.n_steps; ++s) {
        if (s % a.K == 0 && act) {
            uint8_t *rec = a.ckpt + static_cast<uint64_t>(s / a.K) * a.rec_bytes;
            float *rx = reinterpret_cast<float *>(rec);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                rx[d * a.NT + i] = x[d];
                rx[(3 + d) * a.NT + i] = v[d];
            }
            store_state(g, rx + 6 * a.NT, a.NT, i);
        }
        const uint32_t w0 = g.next(), w1 = g.next(), w2 = g.next(), w3 = g.next();
        float gf[3];
        gaussian_forces(w0, w1, w2, w3, gf[0], gf[1], gf[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) ld_update(q, x[d], v[d], gf[d]);
        if (s + 1 >= a.t_begin && s + 1 <= a.t_end)
#pragma unroll
            for (int d = 0; d < 3; ++d) lsum += static_cast<double>(x[d]) * x[d];
    }
    if (act) {
        // the end state: the live buffers and the last checkpoint record
        float *rx = reinterpret_cast<float *>(a.ckpt + static_cast<uint64_t>((a.n_steps + a.K - 1) / a.K) * a.rec_bytes);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.x[d * a.NT + i] = x[d];
            a.v[d * a.NT + i] = v[d];
            rx[d * a.NT + i] = x[d];
            rx[(3 + d) * a.NT + i] = v[d];
        }
        store_state(g, a.state, a.S, i);
        store_state(g, rx + 6 * a.NT, a.NT, i);
    }
    double qv[3] = {act ? lsum : 0.0, 0.0, 0.0};
    block_sum3<BLOCK>(qv, red, a.partials + static_cast<uint64_t>(tile) * 3);
}

template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];
    __shared__ double red[BLOCK / 64][3];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef A = a.adj[e];
    if (A.inverse) return;  // the register-only kernel owns this tile
    const float h = A.f.h, c = A.f.c, kap = A.f.kap;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t col = act ? i : E.offset;  // inactive lanes replay a valid column, store nothing
    Gen g;
    bind_tab(g, lds, threadIdx.x, BLOCK);
    float lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
    double gk = 0.0, gg = 0.0, gT = 0.0;
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    const uint64_t NT = a.NT;
    for (uint32_t seg = nseg; seg-- > 0;) {
        const uint32_t s0 = seg * a.K;
        const uint32_t s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
        const float *rec = reinterpret_cast<const float *>(a.ckpt + static_cast<uint64_t>(seg) * a.rec_bytes);
        float x[3], v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = rec[d * NT + col];
            v[d] = rec[(3 + d) * NT + col];
        }
        load_state(g, rec + 6 * NT, NT, col);
        // replay: scratch row r holds x_s, v_s, g_s of step s = s0 + r
        for (uint32_t s = s0; s < s1; ++s) {
            float *row = a.scratch + static_cast<uint64_t>(s - s0) * 9 * NT + i;
            const uint32_t w0 = g.next(), w1 = g.next(), w2 = g.next(), w3 = g.next();
            float gf[3];
            gaussian_forces(w0, w1, w2, w3, gf[0], gf[1], gf[2]);
            if (act)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    row[d * NT] = x[d];
                    row[(3 + d) * NT] = v[d];
                    row[(6 + d) * NT] = gf[d];
                }
#pragma unroll
            for (int d = 0; d < 3; ++d) ld_update(A.f, x[d], v[d], gf[d]);
        }
        // reverse sweep; x holds x_{s+1} on entry to step s
        for (uint32_t s = s1; s-- > s0;) {
            const bool in_loss = (s + 1 >= a.t_begin) && (s + 1 <= a.t_end);
            const float *row = a.scratch + static_cast<uint64_t>(s - s0) * 9 * NT + i;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (in_loss) lx[d] += 2.0f * x[d];
                const float xs = act ? row[d * NT] : 0.0f;
                const float vs = act ? row[(3 + d) * NT] : 0.0f;
                const float gs = act ? row[(6 + d) * NT] : 0.0f;
                const float mu = lv[d] + h * lx[d];
                gk += static_cast<double>(mu) * static_cast<double>(-A.dkap_dk * xs);
                gg += static_cast<double>(mu) * static_cast<double>(A.dc_dgamma * vs + A.dsig_dgamma * gs);
                gT += static_cast<double>(mu) * static_cast<double>(A.dsig_dkT * gs);
                lx[d] = lx[d] - kap * mu;
                lv[d] = c * mu;
                x[d] = xs;
            }
        }
    }
    double qv[3] = {act ? gk : 0.0, act ? gg : 0.0, act ? gT : 0.0};
    block_sum3<BLOCK>(qv, red, a.partials + static_cast<uint64_t>(tile) * 3);
}

// register-only backward sweep (Hybrid Taus): no replay and no scratch
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_inv_kernel(AdjArgs a) {
    __shared__ double red[BLOCK / 64][3];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef A = a.adj[e];
    if (!A.inverse) return;  // the replay kernel owns this tile
    const float h = A.f.h, c = A.f.c, kap = A.f.kap, sig = A.f.sig, inv_c = A.inv_c;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t col = act ? i : E.offset;  // inactive lanes follow a valid column
    const uint64_t NT = a.NT;
    HybridTaus g;
    float lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
    double gk = 0.0, gg = 0.0, gT = 0.0;
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    for (uint32_t seg = nseg; seg-- > 0;) {
        const uint32_t s0 = seg * a.K;
        const uint32_t s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
        // record seg + 1 holds the state at s1 (the end state for the last segment)
        const float *rec = reinterpret_cast<const float *>(a.ckpt + static_cast<uint64_t>(seg + 1) * a.rec_bytes);
        float x[3], v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = rec[d * NT + col];
            v[d] = rec[(3 + d) * NT + col];
        }
        g.load(reinterpret_cast<const uint32_t *>(rec + 6 * NT), NT, col);
        // x, v hold the state after step s on entry to step s
        for (uint32_t s = s1; s-- > s0;) {
            const bool in_loss = (s + 1 >= a.t_begin) && (s + 1 <= a.t_end);
            const uint32_t w3 = g.prev();
            const uint32_t w2 = g.prev();
            const uint32_t w1 = g.prev();
            const uint32_t w0 = g.prev();
            float gf[3];
            gaussian_forces(w0, w1, w2, w3, gf[0], gf[1], gf[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (in_loss) lx[d] += 2.0f * x[d];
                const float xs = x[d] - h * v[d];
                const float vs = (v[d] + kap * xs - sig * gf[d]) * inv_c;
                const float mu = lv[d] + h * lx[d];
                gk += static_cast<double>(mu) * static_cast<double>(-A.dkap_dk * xs);
                gg += static_cast<double>(mu) * static_cast<double>(A.dc_dgamma * vs + A.dsig_dgamma * gf[d]);
                gT += static_cast<double>(mu) * static_cast<double>(A.dsig_dkT * gf[d]);
                lx[d] = lx[d] - kap * mu;
                lv[d] = c * mu;
                x[d] = xs;
                v[d] = vs;
            }
        }
    }
    double qv[3] = {act ? gk : 0.0, act ? gg : 0.0, act ? gT : 0.0};
    block_sum3<BLOCK>(qv, red, a.partials + static_cast<uint64_t>(tile) * 3);
}

__global__ __launch_bounds__(64) void adj_finalize_kernel(const double *partials, uint32_t width, const EnsDev *ens,
                                                          double denom_steps, double *out) {
    const uint32_t e = blockIdx.x;
    const EnsDev &E = ens[e];
    const double denom = denom_steps * 3.0 * static_cast<double>(E.n);
    for (uint32_t qi = 0; qi < width; ++qi) {
        double acc = 0.0;
        for (uint32_t t = threadIdx.x; t < E.n_tiles; t += 64) acc += partials[(E.tile_begin + t) * 3ull + qi];
        acc = wave_sum(acc);
        if (threadIdx.x == 0) out[static_cast<uint64_t>(e) * width + qi] = E.n ? acc / denom : 0.0;
    }
}

constexpr int kAdjBlock = 256;

}  // namespace

hipError_t launch_ld_ckpt(int kind, const AdjArgs &a, uint32_t block, hipStream_t st) {
    (void)block;
    if (a.n_tiles == 0) return hipSuccess;
    if (kind == RNGLD_RAN2)
        ld_ckpt_kernel<Ran2, kAdjBlock><<<a.n_tiles, kAdjBlock, kR2Tab * kAdjBlock * 4, st>>>(a);
    else
        ld_ckpt_kernel<HybridTaus, kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_ld_adjoint(int kind, const AdjArgs &a, bool any_replay, bool any_inverse, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    if (any_replay) {
        if (kind == RNGLD_RAN2)
            ld_adjoint_kernel<Ran2, kAdjBlock><<<a.n_tiles, kAdjBlock, kR2Tab * kAdjBlock * 4, st>>>(a);
        else
            ld_adjoint_kernel<HybridTaus, kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (any_inverse && kind == RNGLD_HYBRID_TAUS) ld_adjoint_inv_kernel<kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_adj_finalize(const double *partials, uint32_t n_tiles, uint32_t width, const EnsDev *ens,
                               uint32_t n_ens, double denom_steps, double *out, hipStream_t st) {
    (void)n_tiles;
    if (n_ens == 0) return hipSuccess;
    adj_finalize_kernel<<<n_ens, 64, 0, st>>>(partials, width, ens, denom_steps, out);
    return hipGetLastError();
}

}  // namespace rngld
