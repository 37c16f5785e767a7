// k_adj.hip -- pathwise reverse-mode gradients of an LD loss w.r.t. (k, gamma, kT).
//
// Not in the paper; it differentiates the paper's LD model (Sec. I, Sec. IV) with the noise held
// fixed.  Underdamped semi-implicit step per component, z = (x, v):
//     v' = c v - kap x + sig g,  x' = x + h v'.
// With mu = lam_v' + h lam_x' (adjoints of the step's outputs), one reverse step is
//     lam_x = lam_x' - kap mu + dL/dx,  lam_v = c mu,
//     dL/dtheta += mu (dc/dtheta v - dkap/dtheta x + dsig/dtheta g).
// The forward kernels write (x, v, generator state) every K steps and at the end.  The backward
// kernels take one of two ways per ensemble:
//  * register-only (Hybrid Taus, Ran2): the forward run also leaves in each record the loss
//    adjoint of the record's state (the recursion is linear with a step matrix B that is the same
//    for every step of an ensemble, so each segment's own share, summed over its window steps,
//    plus B^K times the adjoint at its end gives the adjoint at its start, walked last to first
//    in FP64).  Every segment then runs on its own, one thread per (oscillator, segment), forward
//    in time from its start record: the same generator, Box-Muller and update code give the noise
//    and the path bit for bit, and the adjoint is carried forward by solving the reverse step for
//    lam'.  Nothing is stored per step.
//  * replay: restore the checkpoint at the segment's start, rerun the segment with the same
//    generator, Box-Muller and update code, keep its path in a per-thread scratch column, and
//    sweep it backward, segments last to first.
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

// one step of the adjoint recursion with no loss term, in FP64 with the ensemble's binary32
// coefficients: (lam_x, lam_v) <- B (lam_x, lam_v), mu = lam_v + h lam_x, lam_x' = lam_x - kap mu,
// lam_v' = c mu
__device__ __forceinline__ void adjoint_step(const LdCoef &q, double &lx, double &lv) {
    const double mu = lv + static_cast<double>(q.h) * lx;
    lx = lx - static_cast<double>(q.kap) * mu;
    lv = static_cast<double>(q.c) * mu;
}

// the loss window's step range [lo, hi) within steps [s0, s1): the loss takes the positions after
// steps t_begin..t_end, i.e. steps s in [t_begin - 1, t_end)
__device__ __forceinline__ void window_part(const AdjArgs &a, uint32_t s0, uint32_t s1, uint32_t &lo, uint32_t &hi) {
    const uint32_t w_lo = a.t_begin - 1, w_hi = a.t_end;
    lo = s0 > w_lo ? s0 : (w_lo < s1 ? w_lo : s1);
    hi = lo > w_hi ? lo : (w_hi < s1 ? w_hi : s1);
}

// The last pass of a forward run over component d of oscillator i's checkpoint records, latest
// first: the end state's adjoint is 0, and each segment's start adjoint is its own part (parked in
// the adjoint rows of its start record by the forward run, for segments with window steps) plus
// bk = B^K times its end adjoint (every segment but the last is K steps long, and the last one's
// end adjoint is 0).  The parked values of the next segment down are loaded one iteration ahead.
__device__ void adjoint_walk(const AdjArgs &a, uint64_t i, int d, const double bk[4]) {
    const uint64_t NT = a.NT;
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    auto rec_f = [&](uint32_t r) { return reinterpret_cast<float *>(a.ckpt + static_cast<uint64_t>(r) * a.rec_bytes); };
    auto has_window = [&](uint32_t seg) {
        const uint32_t s0 = seg * a.K, s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
        uint32_t lo, hi;
        window_part(a, s0, s1, lo, hi);
        return hi > lo;
    };
    auto own = [&](uint32_t seg, float &ox, float &ov) {
        ox = ov = 0.0f;
        if (has_window(seg)) {
            const float *r = rec_f(seg);
            ox = r[(a.lam_row + d) * NT + i];
            ov = r[(a.lam_row + 3 + d) * NT + i];
        }
    };
    double lx = 0.0, lv = 0.0;
    float ox, ov;
    own(nseg - 1, ox, ov);
    for (uint32_t seg = nseg; seg-- > 0;) {
        float px = 0.0f, pv = 0.0f;
        if (seg > 0) own(seg - 1, px, pv);
        float *r_end = rec_f(seg + 1);
        r_end[(a.lam_row + d) * NT + i] = static_cast<float>(lx);
        r_end[(a.lam_row + 3 + d) * NT + i] = static_cast<float>(lv);
        const double nx = bk[0] * lx + bk[1] * lv + ox;
        const double nv = bk[2] * lx + bk[3] * lv + ov;
        lx = nx;
        lv = nv;
        ox = px;
        ov = pv;
    }
    float *r0 = rec_f(0);
    r0[(a.lam_row + d) * NT + i] = static_cast<float>(lx);
    r0[(a.lam_row + 3 + d) * NT + i] = static_cast<float>(lv);
}

// forward run from the current state with checkpoints every K steps; loss partial = sum of x^2
// over the loss window (scaled on finalisation).
// For ensembles with lam each record also gets the loss adjoint of its state, the starting point
// of the register-only backward of the segment that starts there.  The adjoint recursion is
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
    if (A.sp) return;  // the segment-parallel kernels own this tile
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
    // B^j e1 of the current step and the segment's own adjoint sums (without the factor 2), in FP64:
    // they are the starting adjoint of the register-only backward, carried over up to K steps
    double al = 0.0, be = 0.0, ox[3] = {0, 0, 0}, ov[3] = {0, 0, 0};
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
            al = 1.0;
            be = 0.0;
            for (uint32_t j = s0; j < lo; ++j) adjoint_step(q, al, be);
#pragma unroll
            for (int d = 0; d < 3; ++d) ox[d] = ov[d] = 0.0;
            steps(std::true_type{}, std::true_type{}, lo, hi, lseg);
            // the segment's own adjoint, parked in its start record until the last pass
            if (act)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    rx[(a.lam_row + d) * NT + i] = static_cast<float>(2.0 * ox[d]);
                    rx[(a.lam_row + 3 + d) * NT + i] = static_cast<float>(2.0 * ov[d]);
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
        const double bk[4] = {A.phi[0], A.phi[1], A.phi[2], A.phi[3]};
        for (int d = 0; d < 3; ++d) adjoint_walk(a, i, d, bk);
    }
    // the loss sum and its square (the per-oscillator spread of the loss)
    const double qv[6] = {act ? lsum : 0.0, act ? lsum * lsum : 0.0, 0.0, 0.0, 0.0, 0.0};
    block_sum6<BLOCK>(qv, red, a.partials + static_cast<uint64_t>(tile) * kAdjPartW);
}

// ---- segment-parallel forward (Hybrid Taus) ---------------------------------------------------------
// Every Tausworthe step is linear over GF(2) on the 32-bit word (shifts, masks and xors), and the
// LCG step is affine, so the generator's state after n draws is a fixed 32 x 32 bit matrix per
// component applied to the state now, plus the LCG's n-step map.  The LD step is linear too:
// (x, v) after j steps from (x0, v0) is the zero-start run plus F^j (x0, v0).  So each segment runs
// from a zero state with its generator jumped to the segment's start, all segments at once, and a
// join pass per oscillator walks the segments in order in FP64, adding F^len times the true start
// state to each segment's end and the matching terms to its loss and adjoint sums.

// z -> M z over GF(2), M given by its 32 columns
__device__ __forceinline__ uint32_t gf2_apply(const uint32_t *col, uint32_t z) {
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) r ^= static_cast<uint32_t>(__builtin_amdgcn_sbfe(static_cast<int32_t>(z), b, 1)) & col[b];
    return r;
}

// one draw's step of Tausworthe component c of Hybrid Taus
__device__ __forceinline__ uint32_t taus_component_step(int c, uint32_t z) {
    return c == 0 ? tausworthe<13, 12, 31>(z) : (c == 1 ? tausworthe<2, 4, 29>(z) : tausworthe<3, 17, 28>(z));
}

// 2 x 2 row-major products in FP64
__device__ __forceinline__ void mat2_mul(const double *p, const double *q, double *out) {
    const double r0 = p[0] * q[0] + p[1] * q[2], r1 = p[0] * q[1] + p[1] * q[3];
    const double r2 = p[2] * q[0] + p[3] * q[2], r3 = p[2] * q[1] + p[3] * q[3];
    out[0] = r0, out[1] = r1, out[2] = r2, out[3] = r3;
}

// Tables of the segment-parallel forward.  Blocks [0, nseg): the jump of segment seg, 4 seg K draws:
// thread t < 96 follows column t % 32 of component t / 32 through binary powering, with the matrix
// M^(2^k) squared in LDS each round; thread 96 the LCG's map.  Blocks [nseg, nseg + n_ens): the
// ensemble's coefficients for j = 1..K, (a_j, b_j) the first row of F^j (also B^j e1, since the
// adjoint step is B = F^T), each by binary powering in FP64 and rounded once.
__global__ __launch_bounds__(128) void adj_prep_kernel(AdjArgs a, uint32_t nseg) {
    __shared__ uint32_t P[3][32];
    const uint32_t t = threadIdx.x;
    if (blockIdx.x < nseg) {
        const uint64_t n = 4ull * blockIdx.x * a.K;
        const int c = static_cast<int>(t / 32), b = static_cast<int>(t % 32);
        uint32_t v = t < 96 ? (1u << b) : 0u;
        if (t < 96) P[c][b] = taus_component_step(c, 1u << b);
        __syncthreads();
        for (uint64_t m = n; m != 0; m >>= 1) {
            if ((m & 1) && t < 96) v = gf2_apply(P[c], v);
            const uint32_t sq = t < 96 ? gf2_apply(P[c], P[c][b]) : 0u;
            __syncthreads();
            if (t < 96) P[c][b] = sq;
            __syncthreads();
        }
        uint32_t *J = a.jump + static_cast<uint64_t>(blockIdx.x) * kJumpWords;
        if (t < 96) J[t] = v;
        if (t == 96) {
            const uint32_t add = lcg_skip(0u, n);
            J[96] = lcg_skip(1u, n) - add;
            J[97] = add;
            J[98] = J[99] = 0u;
        }
        return;
    }
    const uint32_t e = blockIdx.x - nseg;
    const AdjCoef &A = a.adj[e];
    if (!A.sp) return;
    const LdCoef q = A.f;
    const double h = q.h, c = q.c, kap = q.kap;
    const double F[4] = {1.0 - h * kap, h * c, -kap, c};
    for (uint32_t j = 1 + t; j <= a.K; j += 128) {
        double pf[4] = {1, 0, 0, 1}, sf[4];
        for (int k = 0; k < 4; ++k) sf[k] = F[k];
        for (uint32_t m = j; m != 0; m >>= 1) {
            if (m & 1) mat2_mul(pf, sf, pf);
            mat2_mul(sf, sf, sf);
        }
        a.coef[static_cast<uint64_t>(e) * a.K + j - 1] =
            make_float2(static_cast<float>(pf[0]), static_cast<float>(pf[1]));
    }
}

// Zero-start run of one segment, one thread per (oscillator, segment), blockIdx.y the segment: the
// generator jumped to the segment's start (also written to the segment's start record; the last
// segment writes its end state to the end record), the window sums of the join in kFwdSegF rows.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_fwd_seg_kernel(AdjArgs a) {
    const uint32_t tile = blockIdx.x, seg = blockIdx.y;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef &A = a.adj[e];
    if (!A.sp) return;
    const LdCoef q = A.f;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t col = act ? i : E.offset;  // inactive lanes follow a valid column, store nothing
    const uint64_t NT = a.NT;
    const uint32_t nseg = gridDim.y;
    const uint32_t s0 = seg * a.K, s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
    HybridTaus g;
    g.load(static_cast<const uint32_t *>(a.state), a.S, col);
    const uint32_t *J = a.jump + static_cast<uint64_t>(seg) * kJumpWords;
    g.t1 = gf2_apply(J, g.t1);
    g.t2 = gf2_apply(J + 32, g.t2);
    g.t3 = gf2_apply(J + 64, g.t3);
    g.lcg = J[96] * g.lcg + J[97];
    auto rec_f = [&](uint32_t r) { return reinterpret_cast<float *>(a.ckpt + static_cast<uint64_t>(r) * a.rec_bytes); };
    if (act) g.store(reinterpret_cast<uint32_t *>(rec_f(seg) + 6 * NT), NT, i);
    float x[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    float sxx = 0.0f, sa[3] = {0, 0, 0}, sb[3] = {0, 0, 0};
    const float2 *cf = a.coef + static_cast<uint64_t>(e) * a.K;
    auto steps = [&](auto win_tag, uint32_t s, uint32_t end) {
        constexpr bool WIN = decltype(win_tag)::value;
        for (; s < end; ++s) {
            const uint32_t w0 = g.next_top24(), w1 = g.next_top24(), w2 = g.next_top24(), w3 = g.next_top24();
            float gf[3];
            gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) ld_update_s<0>(q, x[d], v[d], gf[d]);
            if constexpr (WIN) {
                const float2 k = cf[s - s0];  // j = s - s0 + 1
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    sxx += x[d] * x[d];
                    sa[d] += k.x * x[d];
                    sb[d] += k.y * x[d];
                }
            }
        }
    };
    uint32_t lo, hi;
    window_part(a, s0, s1, lo, hi);
    steps(std::false_type{}, s0, lo);
    steps(std::true_type{}, lo, hi);
    steps(std::false_type{}, hi, s1);
    if (!act) return;
    float *fr = a.fwd_seg + static_cast<uint64_t>(seg) * kFwdSegF * NT + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fr[d * NT] = x[d];
        fr[(3 + d) * NT] = v[d];
        fr[(7 + d) * NT] = sa[d];
        fr[(10 + d) * NT] = sb[d];
    }
    fr[6 * NT] = sxx;
    if (seg + 1 == nseg) g.store(reinterpret_cast<uint32_t *>(rec_f(nseg) + 6 * NT), NT, i);
}

// Join of the segment-parallel forward, FP64, one thread per (oscillator, component): a block of
// 3 x TILE threads covers one tile, thread t taking component t / TILE of oscillator t % TILE.  It
// walks the segments in order from the live x, v, writing each record's x, v, the segment's loss
// and own adjoint (the zero-start sums plus their response to the start state), the end state to
// the end record and the live buffers, the end record's generator rows to the live state; then the
// adjoint walk.  The next segment's sums are loaded one iteration ahead.
template <int TILE>
__global__ __launch_bounds__(3 * TILE) void ld_fwd_join_kernel(AdjArgs a) {
    __shared__ double red[3 * TILE / 64][6];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef &A = a.adj[e];
    if (!A.sp) return;
    const int d = static_cast<int>(threadIdx.x / TILE);
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * TILE + threadIdx.x % TILE;
    const bool act = i < E.offset + E.n;
    const uint64_t NT = a.NT;
    const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
    auto rec_f = [&](uint32_t r) { return reinterpret_cast<float *>(a.ckpt + static_cast<uint64_t>(r) * a.rec_bytes); };
    // the zero-start run's rows of one segment for this component (and the x^2 sum for d = 0)
    struct Rows {
        float xp, vp, sa, sb, sxx;
    };
    auto load = [&](uint32_t seg) {
        const float *fr = a.fwd_seg + static_cast<uint64_t>(seg) * kFwdSegF * NT + i;
        return Rows{fr[d * NT], fr[(3 + d) * NT], fr[(7 + d) * NT], fr[(10 + d) * NT], d == 0 ? fr[6 * NT] : 0.0f};
    };
    double lsum = 0.0;
    if (act) {
        const float2 *cf = a.coef + static_cast<uint64_t>(e) * a.K;
        double x = a.x[d * NT + i], v = a.v[d * NT + i];
        Rows cur = load(0);
        for (uint32_t seg = 0; seg < nseg; ++seg) {
            const Rows nxt = seg + 1 < nseg ? load(seg + 1) : cur;
            const uint32_t s0 = seg * a.K, s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
            float *rx = rec_f(seg);
            rx[d * NT + i] = static_cast<float>(x);
            rx[(3 + d) * NT + i] = static_cast<float>(v);
            uint32_t lo, hi;
            window_part(a, s0, s1, lo, hi);
            if (hi > lo) {
                // the sums of a_j^2, a_j b_j, b_j^2 over the window steps j = lo - s0 + 1 .. hi - s0
                double P[3];
                if (lo == s0 && hi - s0 == a.K) {
                    for (int k = 0; k < 3; ++k) P[k] = A.full[k];
                } else {
                    for (int k = 0; k < 3; ++k) P[k] = 0.0;
                    for (uint32_t s = lo; s < hi; ++s) {
                        const float2 k2 = cf[s - s0];
                        const double ca = k2.x, cb = k2.y;
                        P[0] += ca * ca, P[1] += ca * cb, P[2] += cb * cb;
                    }
                }
                // the segment's loss terms sum_j (x0_j + a_j x + b_j v)^2 (x0 the zero-start path)
                // and their gradient with respect to the start state (x, v), its own adjoint
                lsum += cur.sxx + 2.0 * (x * cur.sa + v * cur.sb) + x * x * P[0] + 2.0 * x * v * P[1] + v * v * P[2];
                rx[(a.lam_row + d) * NT + i] = static_cast<float>(2.0 * (cur.sa + P[0] * x + P[1] * v));
                rx[(a.lam_row + 3 + d) * NT + i] = static_cast<float>(2.0 * (cur.sb + P[1] * x + P[2] * v));
            }
            const double *M = (s1 - s0 == a.K) ? A.fk : A.flast;
            const double nx = cur.xp + M[0] * x + M[1] * v;
            const double nv = cur.vp + M[2] * x + M[3] * v;
            x = nx;
            v = nv;
            cur = nxt;
        }
        float *rx = rec_f(nseg);
        const float xf = static_cast<float>(x), vf = static_cast<float>(v);
        rx[d * NT + i] = xf;
        rx[(3 + d) * NT + i] = vf;
        a.x[d * NT + i] = xf;
        a.v[d * NT + i] = vf;
        // the generator rows of the end record to the live state: rows d, and row 3 with d = 0
        const uint32_t *rs = reinterpret_cast<const uint32_t *>(rx + 6 * NT);
        uint32_t *live = static_cast<uint32_t *>(a.state);
        live[d * a.S + i] = rs[d * NT + i];
        if (d == 0) live[3 * a.S + i] = rs[3 * NT + i];
        adjoint_walk(a, i, d, A.bk);
    }
    const double qv[6] = {act ? lsum : 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    block_sum6<3 * TILE>(qv, red, a.partials + static_cast<uint64_t>(tile) * kAdjPartW);
}

template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];
    __shared__ double red[BLOCK / 64][6];
    const uint32_t tile = blockIdx.x;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef A = a.adj[e];
    if (A.reg_only) return;  // the register-only kernel owns this tile
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

// register-only backward (Hybrid Taus, Ran2), one thread per (oscillator, segment): blockIdx.y is
// the segment.  The record at the segment's start holds its state and the loss adjoint A_s0 of that
// state (the gradient of the loss terms after it), so the segment runs forward in time: the same
// generator, Box-Muller and update steps as the forward run give the noise and the path, and the
// adjoint recursion A_s = B A'_{s+1} is solved for the adjoint of the step's outputs,
//     mu = lam_v / c,  A'_x = lam_x + kap mu,  A'_v = mu - h A'_x,
// then the loss term of the step's end position is taken off, A_{s+1} = A' - (2 x_{s+1}, 0).  The
// powers of B's inverse have the norms of the forward step matrix's inverse powers (B is its
// transpose): the error growth the host bounds over K steps.  Each thread's sums are its segment's share of the gradient;
// they go to seg_d and a second pass adds an oscillator's segments in order.
template <class Gen, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ld_adjoint_seg_kernel(AdjArgs a) {
    extern __shared__ int32_t lds[];  // Ran2: the threads' shuffle tables, [32][BLOCK]
    const uint32_t tile = blockIdx.x, seg = blockIdx.y;
    const uint32_t e = find_ensemble(a.ens, a.n_ens, tile);
    const EnsDev &E = a.ens[e];
    const AdjCoef A = a.adj[e];
    if (!A.reg_only) return;  // the replay kernel owns this tile
    const LdCoef q = A.f;
    const float h = q.h, kap = q.kap, inv_c = A.inv_c, inv_c_lo = A.inv_c_lo;
    const uint64_t i = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * BLOCK + threadIdx.x;
    const bool act = i < E.offset + E.n;
    const uint64_t col = act ? i : E.offset;  // inactive lanes follow a valid column
    const uint64_t NT = a.NT;
    const uint32_t s0 = seg * a.K;
    const uint32_t s1 = (s0 + a.K < a.n_steps) ? s0 + a.K : a.n_steps;
    const float *rec = reinterpret_cast<const float *>(a.ckpt + static_cast<uint64_t>(seg) * a.rec_bytes);
    float x[3], v[3], lx[3], lv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = rec[d * NT + col];
        v[d] = rec[(3 + d) * NT + col];
        lx[d] = rec[(a.lam_row + d) * NT + col];
        lv[d] = rec[(a.lam_row + 3 + d) * NT + col];
    }
    Gen g;
    bind_tab(g, lds, threadIdx.x, BLOCK);
    load_state(g, rec + 6 * NT, NT, col);
    // the segment's gradient as sums over its steps and the three components of mu x, mu v and
    // mu g, scaled by the partials at the end: K terms per component in FP32
    float smx = 0.0f, smv = 0.0f, smg = 0.0f;
    // steps [b, e); LOSS: the steps whose end position is a loss term
    auto sweep = [&](auto loss_tag, uint32_t b, uint32_t e) {
        constexpr bool LOSS = decltype(loss_tag)::value;
        for (uint32_t s = b; s < e; ++s) {
            const uint32_t w0 = g.next_top24(), w1 = g.next_top24(), w2 = g.next_top24(), w3 = g.next_top24();
            float gf[3];
            gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2], Gen::kTopScale);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float mu = __builtin_fmaf(lv[d], inv_c, lv[d] * inv_c_lo);
                const float ax = lx[d] + kap * mu;
                lv[d] = mu - h * ax;
                smx += mu * x[d];
                smv += mu * v[d];
                smg += mu * gf[d];
                ld_update_s<0>(q, x[d], v[d], gf[d]);
                lx[d] = LOSS ? ax - 2.0f * x[d] : ax;
            }
        }
    };
    uint32_t lo, hi;
    window_part(a, s0, s1, lo, hi);
    sweep(std::false_type{}, s0, lo);
    sweep(std::true_type{}, lo, hi);
    sweep(std::false_type{}, hi, s1);
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
    if (!a.adj[e].reg_only) return;  // the replay kernel owns this tile
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

hipError_t launch_ld_ckpt(int kind, const AdjArgs &a, bool any_sp, bool any_seq, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    if (any_sp && kind == RNGLD_HYBRID_TAUS) {
        const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
        adj_prep_kernel<<<nseg + a.n_ens, 128, 0, st>>>(a, nseg);
        ld_fwd_seg_kernel<kAdjBlock><<<dim3(a.n_tiles, nseg), kAdjBlock, 0, st>>>(a);
        ld_fwd_join_kernel<kAdjBlock><<<a.n_tiles, 3 * kAdjBlock, 0, st>>>(a);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (any_seq) {
        if (kind == RNGLD_RAN2)
            ld_ckpt_kernel<Ran2, kAdjBlock><<<a.n_tiles, kAdjBlock, kR2Tab * kAdjBlock * 4, st>>>(a);
        else
            ld_ckpt_kernel<HybridTaus, kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_ld_adjoint(int kind, const AdjArgs &a, bool any_replay, bool any_reg_only, hipStream_t st) {
    if (a.n_tiles == 0) return hipSuccess;
    if (any_replay) {
        if (kind == RNGLD_RAN2)
            ld_adjoint_kernel<Ran2, kAdjBlock><<<a.n_tiles, kAdjBlock, kR2Tab * kAdjBlock * 4, st>>>(a);
        else
            ld_adjoint_kernel<HybridTaus, kAdjBlock><<<a.n_tiles, kAdjBlock, 0, st>>>(a);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (any_reg_only) {
        const uint32_t nseg = (a.n_steps + a.K - 1) / a.K;
        if (kind == RNGLD_RAN2)
            ld_adjoint_seg_kernel<Ran2, kAdjBlock><<<dim3(a.n_tiles, nseg), kAdjBlock, kR2Tab * kAdjBlock * 4, st>>>(a);
        else
            ld_adjoint_seg_kernel<HybridTaus, kAdjBlock><<<dim3(a.n_tiles, nseg), kAdjBlock, 0, st>>>(a);
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
