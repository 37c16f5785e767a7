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
//    each segment restarts from its own end checkpoint, which bounds the growth of rounding
//    errors in the reconstructed path to K steps (the host admits an ensemble only if that growth
//    stays small).  The segments run in parallel, one thread per (oscillator, segment): the
//    reverse recursion is linear with a step matrix B that is the same for every step of an
//    ensemble, so a segment swept with a zero adjoint at its end yields its own contribution, and
//    the contribution of the adjoint that arrives from later segments is linear in that adjoint:
//    with mu^hom_s = a_s lam_x + b_s lam_v the part of mu at step s driven by the end adjoint, the
//    gradient gains sum_s (a_s, b_s) f_s . lam_end, f_s = dc v_s - dkap x_s + dsig g_s.  Each
//    thread records its segment's own adjoint at the start, its gradient sums and the sums
//    sum_s a_s z_s, sum_s b_s z_s for z = x, v, g; a per-oscillator pass then walks the segments
//    from last to first, carrying lam_end(previous) = lam_own + B^K lam_end.
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
        g.idum = g.idum2 = 1;
        g.iym1 = 0;
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

// one oscillator's three gradient sums and their squares, summed over the block (fixed order)
template <int BLOCK>
__device__ __forceinline__ void block_grad_partials(bool act, double gk, double gg, double gT, double (*red)[6],
                                                    double *dst) {
    const double q[6] = {act ? gk : 0.0, act ? gg : 0.0, act ? gT : 0.0,
                         act ? gk * gk : 0.0, act ? gg * gg : 0.0, act ? gT * gT : 0.0};
    block_sum6<BLOCK>(q, red, dst);
}

// one step of the adjoint recursion with no loss term: (lam_x, lam_v) <- B (lam_x, lam_v),
// mu = lam_v + h lam_x, lam_x' = lam_x - kap mu, lam_v' = c mu
__device__ __forceinline__ void adjoint_step(const LdCoef &q, float &lx, float &lv) {
    const float mu = lv + q.h * lx;
    lx = lx - q.kap * mu;
    lv = q.c * mu;
}

// the loss window's step range [lo, hi) within steps [s0, s1): the loss takes the positions after
// steps t_begin..t_end, i.e. steps s in [t_begin - 1, t_end)
__device__ __forceinline__ void window_part(const AdjArgs &a, uint32_t s0, uint32_t s1, uint32_t &lo, uint32_t &hi) {
    const uint32_t w_lo = a.t_begin - 1, w_hi = a.t_end;
    lo = s0 > w_lo ? s0 : (w_lo < s1 ? w_lo : s1);
    hi = lo > w_hi ? lo : (w_hi < s1 ? w_hi : s1);
}

// forward run from the current state with checkpoints every K steps; loss partial = sum of x^2
// over the loss window (scaled on finalisation).
// For ensembles with lam each record also gets the loss adjoint of its state, the starting point
// of the register-only backward sweep of the segment that ends there.  The adjoint recursion is
// linear with the constant matrix B, so what a segment's own loss terms hand to the adjoint at its
// start is the sum over its window steps j = 1..K of B^j (2 x_j, 0); it is accumulated here from
// the forward positions (B^j e1 advanced alongside), and a last pass over the records, latest
// first, adds what the later segments hand back: lam(start) = own + B^K lam(end), in FP64.
template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_ckpt_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];
    __shared__ double red[BLOCK / 64][6];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef &A = a.adj[e];
    const LdCoef q = A.f;
    const bool lam = A.lam != 0;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t NT = a.NT;
    Gen g;
    bind_tab(g, lds, threadIdx.x, BLOCK);
    float x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    if (act) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d] = a.x[d * NT + i];
            v[d] = a.v[d * NT + i];
        }
        load_state(g, a.state, a.S, i);
    } else {
        park(g);
    }
    // B^j e1 of the current step and the segment's own adjoint sums (without the factor 2)
    float al = 0.0f, be = 0.0f, ox[3] = {0, 0, 0}, ov[3] = {0, 0, 0};
    // steps [s, e) of the run, adding x^2 after each step to lseg when LOSS and the step's own
    // adjoint terms when LAM
    auto steps = [&](auto loss_tag, auto lam_tag, uint32_t s, uint32_t e, float &lseg) {
        constexpr bool LOSS = decltype(loss_tag)::value;
        constexpr bool LAM = decltype(lam_tag)::value;
        for (; s < e; ++s) {
            const uint32_t w0 = g.next_top24(), w1 = g.next_top24(), w2 = g.next_top24(), w3 = g.next_top24();
            float gf[3];
            gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2], Gen::kTopScale);
#pragma unroll
            for (int d = 0; d < 3; ++d) ld_update(q, x[d], v[d], gf[d]);
            if constexpr (LOSS) {
#pragma unroll
                for (int d = 0; d < 3; ++d) lseg += x[d] * x[d];
            }
            if constexpr (LAM) {
                adjoint_step(q, al, be);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    ox[d] += al * x[d];
                    ov[d] += be * x[d];
                }
            }
        }
    };
    auto rec_f = [&](uint32_t r) { return reinterpret_cast<float *>(a.ckpt + static_cast<uint64_t>(r) * a.rec_bytes); };
    // the loss sum: FP32 within each K-step segment (at most 3K terms of x^2), FP64 across segments
    double lsum = 0.0;
    for (uint32_t s0 = 0; s0 < a.n_steps; s0 += a.K) {
        float *rx = rec_f(s0 / a.K);
        if (act) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                rx[d * NT + i] = x[d];
                rx[(3 + d) * NT + i] = v[d];
            }
            store_state(g, rx + 6 * NT, NT, i);
        }
        const uint32_t s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
        uint32_t lo, hi;
        window_part(a, s0, s1, lo, hi);
        float lseg = 0.0f;
        steps(std::false_type{}, std::false_type{}, s0, lo, lseg);
        if (lam && hi > lo) {
            // B^(lo - s0) e1 before the first window step
            al = 1.0f;
            be = 0.0f;
            for (uint32_t j = s0; j < lo; ++j) adjoint_step(q, al, be);
#pragma unroll
            for (int d = 0; d < 3; ++d) ox[d] = ov[d] = 0.0f;
            steps(std::true_type{}, std::true_type{}, lo, hi, lseg);
            // the segment's own adjoint, parked in its start record until the last pass
            if (act)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rx[(kCkptLamRow + d) * NT + i] = 2.0f * ox[d];
                    rx[(kCkptLamRow + 3 + d) * NT + i] = 2.0f * ov[d];
                }
        } else {
            steps(std::true_type{}, std::false_type{}, lo, hi, lseg);
        }
        steps(std::false_type{}, std::false_type{}, hi, s1, lseg);
        lsum += static_cast<double>(lseg);
    }
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    if (act) {
        // the end state: the live buffers and the last checkpoint record
        float *rx = rec_f(nseg);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.x[d * NT + i] = x[d];
            a.v[d * NT + i] = v[d];
            rx[d * NT + i] = x[d];
            rx[(3 + d) * NT + i] = v[d];
        }
        store_state(g, a.state, a.S, i);
        store_state(g, rx + 6 * NT, NT, i);
    }
    if (lam && act) {
        // latest record first: the end state's adjoint is 0; each segment's start adjoint is its
        // own part plus B^K times its end adjoint (every segment but the last is K steps long, and
        // the last one's end adjoint is 0)
        double lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
        for (uint32_t seg = nseg; seg-- > 0;) {
            float *r_end = rec_f(seg + 1), *r_start = rec_f(seg);
            const uint32_t s0 = seg * a.K, s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
            uint32_t lo, hi;
            window_part(a, s0, s1, lo, hi);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                r_end[(kCkptLamRow + d) * NT + i] = static_cast<float>(lx[d]);
                r_end[(kCkptLamRow + 3 + d) * NT + i] = static_cast<float>(lv[d]);
                double nx = A.phi[0] * lx[d] + A.phi[1] * lv[d];
                double nv = A.phi[2] * lx[d] + A.phi[3] * lv[d];
                if (hi > lo) {
                    nx += r_start[(kCkptLamRow + d) * NT + i];
                    nv += r_start[(kCkptLamRow + 3 + d) * NT + i];
                }
                lx[d] = nx;
                lv[d] = nv;
            }
        }
        float *r0 = rec_f(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r0[(kCkptLamRow + d) * NT + i] = static_cast<float>(lx[d]);
            r0[(kCkptLamRow + 3 + d) * NT + i] = static_cast<float>(lv[d]);
        }
    }
    // the loss sum and its square (the per-oscillator spread of the loss)
    const double qv[6] = {act ? lsum : 0.0, act ? lsum * lsum : 0.0, 0.0, 0.0, 0.0, 0.0};
    block_sum6<BLOCK>(qv, red, a.partials + static_cast<uint64_t>(tile) * kAdjPartW);
}

template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];
    __shared__ double red[BLOCK / 64][6];
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
            const uint32_t w0 = g.next_top24(), w1 = g.next_top24(), w2 = g.next_top24(), w3 = g.next_top24();
            float gf[3];
            gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2], Gen::kTopScale);
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
    block_grad_partials<BLOCK>(act, gk, gg, gT, red, a.partials + static_cast<uint64_t>(tile) * kAdjPartW);
}

// register-only backward sweep (Hybrid Taus), one thread per (oscillator, segment): blockIdx.y is
// the segment.  The sweep starts from the loss adjoint that the forward run left in the record at
// the segment's end, so each thread's sums are its segment's share of the gradient; they go to
// seg_d and a second pass adds an oscillator's segments in order.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_seg_kernel(AdjArgs a) {
    const uint32_t tile = blockIdx.x, seg = blockIdx.y;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef A = a.adj[e];
    if (!A.inverse) return;  // the replay kernel owns this tile
    const float h = A.f.h, c = A.f.c, kap = A.f.kap, sig = A.f.sig, inv_c = A.inv_c, inv_c_lo = A.inv_c_lo;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t col = act ? i : E.offset;  // inactive lanes follow a valid column
    const uint64_t NT = a.NT;
    const uint32_t s0 = seg * a.K;
    const uint32_t s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
    // record seg + 1 holds the state at s1 (the end state for the last segment) and its adjoint
    const float *rec = reinterpret_cast<const float *>(a.ckpt + static_cast<uint64_t>(seg + 1) * a.rec_bytes);
    float x[3], v[3], lx[3], lv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = rec[d * NT + col];
        v[d] = rec[(3 + d) * NT + col];
        lx[d] = rec[(kCkptLamRow + d) * NT + col];
        lv[d] = rec[(kCkptLamRow + 3 + d) * NT + col];
    }
    HybridTaus g;
    g.load(reinterpret_cast<const uint32_t *>(rec + 6 * NT), NT, col);
    // the segment's gradient as sums over its steps and the three components of mu x, mu v and
    // mu g, scaled by the partials at the end: K terms per component in FP32
    float smx = 0.0f, smv = 0.0f, smg = 0.0f;
    // x, v hold the state after step s on entry to step s
    for (uint32_t s = s1; s-- > s0;) {
        const bool in_loss = (s + 1 >= a.t_begin) && (s + 1 <= a.t_end);
        const uint32_t w3 = g.prev_top24();
        const uint32_t w2 = g.prev_top24();
        const uint32_t w1 = g.prev_top24();
        const uint32_t w0 = g.prev_top24();
        float gf[3];
        gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (in_loss) lx[d] += 2.0f * x[d];
            const float xs = x[d] - h * v[d];
            const float t = v[d] + kap * xs - sig * gf[d];
            const float vs = __builtin_fmaf(t, inv_c, t * inv_c_lo);
            const float mu = lv[d] + h * lx[d];
            smx += mu * xs;
            smv += mu * vs;
            smg += mu * gf[d];
            lx[d] = lx[d] - kap * mu;
            lv[d] = c * mu;
            x[d] = xs;
            v[d] = vs;
        }
    }
    if (!act) return;
    double *rd = a.seg_d + static_cast<uint64_t>(seg) * kAdjSegD * NT + i;
    rd[0] = -static_cast<double>(A.dkap_dk) * smx;
    rd[NT] = static_cast<double>(A.dc_dgamma) * smv + static_cast<double>(A.dsig_dgamma) * smg;
    rd[2 * NT] = static_cast<double>(A.dsig_dkT) * smg;
}

// per-oscillator sum of the segments' gradient shares in segment order, then the block's partials
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_sum_kernel(AdjArgs a) {
    __shared__ double red[BLOCK / 64][6];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    if (!a.adj[e].inverse) return;  // the replay kernel owns this tile
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t NT = a.NT;
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    double gk = 0.0, gg = 0.0, gT = 0.0;
    if (act)
        for (uint32_t seg = 0; seg < nseg; ++seg) {
            const double *rd = a.seg_d + static_cast<uint64_t>(seg) * kAdjSegD * NT + i;
            gk += rd[0];
            gg += rd[NT];
            gT += rd[2 * NT];
        }
    block_grad_partials<BLOCK>(act, gk, gg, gT, red, a.partials + static_cast<uint64_t>(tile) * kAdjPartW);
}

__global__ __launch_bounds__(64) void adj_finalize_kernel(const double *partials, uint32_t width, bool spread,
                                                          const EnsDev *ens, double denom_steps, double *out) {
    const uint32_t e = blockIdx.x;
    const EnsDev &E = ens[e];
    const double n = static_cast<double>(E.n);
    const double per_osc = denom_steps * 3.0;  // a per-oscillator sum over this is its contribution
    const uint32_t ow = spread ? 2 * width : width;
    for (uint32_t qi = 0; qi < width; ++qi) {
        double acc = 0.0, acc2 = 0.0;
        for (uint32_t t = threadIdx.x; t < E.n_tiles; t += 64) {
            acc += partials[(E.tile_begin + t) * static_cast<uint64_t>(kAdjPartW) + qi];
            acc2 += partials[(E.tile_begin + t) * static_cast<uint64_t>(kAdjPartW) + width + qi];
        }
        acc = wave_sum(acc);
        acc2 = wave_sum(acc2);
        if (threadIdx.x == 0) {
            const double mean = E.n ? acc / (per_osc * n) : 0.0;
            out[static_cast<uint64_t>(e) * ow + qi] = mean;
            if (spread) {
                // standard error of the mean of the per-oscillator contributions c_i = g_i / per_osc
                double se = 0.0;
                if (E.n > 1) {
                    const double var = (acc2 / (per_osc * per_osc) - n * mean * mean) / (n - 1.0);
                    se = var > 0.0 ? sqrt(var / n) : 0.0;
                }
                out[static_cast<uint64_t>(e) * ow + width + qi] = se;
            }
        }
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
    if (any_inverse && kind == RNGLD_HYBRID_TAUS) {
        const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
        ld_adjoint_seg_kernel<kAdjBlock><<<dim3(a.n_tiles, nseg), kAdjBlock, 0, st>>>(a);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        ld_adjoint_sum_kernel<kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_adj_finalize(const double *partials, uint32_t n_tiles, uint32_t width, bool spread,
                               const EnsDev *ens, uint32_t n_ens, double denom_steps, double *out, hipStream_t st) {
    (void)n_tiles;
    if (n_ens == 0) return hipSuccess;
    adj_finalize_kernel<<<n_ens, 64, 0, st>>>(partials, width, spread, ens, denom_steps, out);
    return hipGetLastError();
}

}  // namespace rngld
