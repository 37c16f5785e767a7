// k_ld.hip -- fused RNG + Langevin-dynamics kernels for the per-thread generators.
//
// The paper launches one kernel per LD step and keeps generator state in global memory between
// steps (Sec. III.B; Fig. 2; Sec. IV, where all threads synchronise after every step).  Here one launch runs
// many steps: every thread keeps its oscillators' x, v and its generator state in VGPRs (Ran2's
// shuffle table in LDS) from the first step of the launch to the last, so device memory is
// touched once per launch, not once per step.  ld_step_* keeps the paper's per-step protocol.
//
// Observables (Sec. IV's <R(t)>, <R(t)R(0)> per component) are reduced without atomics: FP64 wave
// sums, then a fixed-order sum over the block's waves into one partial per (point, tile), then a
// fixed-order sum over an ensemble's tiles.  The order depends only on the tile shape, so runs are
// reproducible and a batched ensemble equals its plain run bit for bit.
#include <cstring>
#include <type_traits>

#include "internal.hpp"

namespace rngld {

namespace {

constexpr int kNobs = RNGLD_NOBS;

template <class Gen>
struct IsRan2 : std::false_type {};
template <>
struct IsRan2<Ran2> : std::true_type {};

template <class Gen>
struct IsLcg : std::false_type {};
template <>
struct IsLcg<Lcg32> : std::true_type {};

template <class Gen>
struct IsNoNoise : std::false_type {};
template <>
struct IsNoNoise<NoNoise> : std::true_type {};

// one oscillator-step's three force components: four words through Box-Muller, or zero
template <class Gen>
__device__ __forceinline__ void draw_forces(Gen &g, float &gx, float &gy, float &gz) {
    if constexpr (IsNoNoise<Gen>::value) {
        gx = gy = gz = 0.0f;
    } else {
        const uint32_t m0 = g.next_top24();
        const uint32_t m1 = g.next_top24();
        const uint32_t m2 = g.next_top24();
        const uint32_t m3 = g.next_top24();
        gaussian_forces_top24(m0, m1, m2, m3, gx, gy, gz, Gen::kTopScale);
    }
}

template <class Gen>
__device__ __forceinline__ void gen_park(Gen &g) {
    if constexpr (IsRan2<Gen>::value) {
        g.idum = 1;
        g.idum2 = 1;
        g.iym1 = 0;
        for (int t = 0; t < kR2Tab; ++t) g.tab[t * g.tstride] = 1;
    } else if constexpr (IsLcg<Gen>::value) {
        g.x = 0x9E3779B9u;
    } else if constexpr (IsNoNoise<Gen>::value) {
    } else {
        g.t1 = g.t2 = g.t3 = g.lcg = 0x9E3779B9u;
    }
}

template <class Gen>
__device__ __forceinline__ void gen_load(Gen &g, const void *st, uint64_t S, uint64_t j) {
    if constexpr (IsRan2<Gen>::value)
        g.load(static_cast<const int32_t *>(st), S, j);
    else
        g.load(static_cast<const uint32_t *>(st), S, j);
}

template <class Gen>
__device__ __forceinline__ void gen_store(const Gen &g, void *st, uint64_t S, uint64_t j) {
    if constexpr (IsRan2<Gen>::value)
        g.store(static_cast<int32_t *>(st), S, j);
    else
        g.store(static_cast<uint32_t *>(st), S, j);
}

// FP64 sums of the six observables over the block's active oscillators, one partial per tile
template <int BLOCK, int OPT>
__device__ __forceinline__ void record_point(const float (&x)[OPT][3], const float (&v)[OPT][3],
                                             const float (&x0)[OPT][3], const float (&v0)[OPT][3],
                                             const bool (&act)[OPT], bool after_t0, double (*red)[kNobs],
                                             double *dst) {
    double q[kNobs] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < OPT; ++k)
        if (act[k]) add_observables(q, x[k], v[k], x0[k], v0[k], after_t0);
    block_sum6<BLOCK>(q, red, dst);
}

// the step loop of one tile, with the integrator scheme fixed at compile time
template <int SCHEME, int BLOCK, int OPT, class Gen>
__device__ __forceinline__ void run_steps(const LdArgs &a, const LdCoef &q, uint32_t tile, Gen (&g)[OPT],
                                          float (&x)[OPT][3], float (&v)[OPT][3], float (&x0)[OPT][3],
                                          float (&v0)[OPT][3], const bool (&act)[OPT], double (*red)[kNobs]) {
    uint32_t next_obs = 0xFFFFFFFFu;
    if (a.stride) next_obs = ((a.step_begin + a.stride - 1) / a.stride) * a.stride;
    uint32_t s = a.step_begin;
    while (s < a.step_end) {
        if (s == a.t0) {
#pragma unroll
            for (int k = 0; k < OPT; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x0[k][d] = x[k][d];
                    v0[k][d] = v[k][d];
                }
        }
        if (s == next_obs) {
            double *dst = a.partials + (static_cast<uint64_t>(s / a.stride) * a.n_tiles + tile) * kNobs;
            record_point<BLOCK, OPT>(x, v, x0, v0, act, s >= a.t0, red, dst);
            next_obs += a.stride;
        }
        // steps up to the next event run without any per-step test (stop > s always)
        uint32_t stop = a.step_end < next_obs ? a.step_end : next_obs;
        if (a.t0 > s && a.t0 < stop) stop = a.t0;
        for (; s < stop; ++s) {
#pragma unroll
            for (int k = 0; k < OPT; ++k) {
                float gx, gy, gz;
                draw_forces(g[k], gx, gy, gz);
                ld_update_s<SCHEME>(q, x[k][0], v[k][0], gx);
                ld_update_s<SCHEME>(q, x[k][1], v[k][1], gy);
                ld_update_s<SCHEME>(q, x[k][2], v[k][2], gz);
            }
        }
    }
}

template <class Gen, int BLOCK, int OPT>
__global__ __launch_bounds__(BLOCK) void ld_run_kernel(LdArgs a) {
    extern __shared__ int32_t lds_tables[];  // Ran2: [OPT][32][BLOCK]
    __shared__ double red[BLOCK / 64][kNobs];
    const int tid = threadIdx.x;

    for (uint32_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        // ensemble owning this tile
        uint32_t lo = 0, hi = a.n_ens - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (a.ens[mid].tile_begin <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        const EnsDev &E = a.ens[lo];
        const LdCoef q = E.coef;
        const uint64_t first = E.offset + static_cast<uint64_t>(tile - E.tile_begin) * (BLOCK * OPT);
        const uint64_t end = E.offset + E.n;

        float x[OPT][3], v[OPT][3], x0[OPT][3], v0[OPT][3];
        bool act[OPT];
        Gen g[OPT];
        const bool have_t0 = a.stride && a.step_begin > a.t0;
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            const uint64_t i = first + tid + static_cast<uint64_t>(k) * BLOCK;
            act[k] = i < end;
            if constexpr (IsRan2<Gen>::value) {
                g[k].tab = lds_tables + k * kR2Tab * BLOCK + tid;
                g[k].tstride = BLOCK;
            }
            if (act[k]) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x[k][d] = a.x[d * a.NT + i];
                    v[k][d] = a.v[d * a.NT + i];
                    x0[k][d] = have_t0 ? a.t0buf[d * a.NT + i] : 0.0f;
                    v0[k][d] = have_t0 ? a.t0buf[(3 + d) * a.NT + i] : 0.0f;
                }
                gen_load(g[k], a.state, a.S, i);
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) x[k][d] = v[k][d] = x0[k][d] = v0[k][d] = 0.0f;
                gen_park(g[k]);
            }
        }

        if (q.scheme == 0)
            run_steps<0, BLOCK, OPT>(a, q, tile, g, x, v, x0, v0, act, red);
        else
            run_steps<1, BLOCK, OPT>(a, q, tile, g, x, v, x0, v0, act, red);
        if (a.step_end == a.n_steps) {
            const uint32_t s = a.n_steps;
            if (s == a.t0) {
#pragma unroll
                for (int k = 0; k < OPT; ++k)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        x0[k][d] = x[k][d];
                        v0[k][d] = v[k][d];
                    }
            }
            if (a.stride && s % a.stride == 0) {
                double *dst = a.partials + (static_cast<uint64_t>(s / a.stride) * a.n_tiles + tile) * kNobs;
                record_point<BLOCK, OPT>(x, v, x0, v0, act, s >= a.t0, red, dst);
            }
        }
        const bool keep_t0 = a.stride && a.t0 < a.step_end && a.step_end < a.n_steps;
#pragma unroll
        for (int k = 0; k < OPT; ++k) {
            if (!act[k]) continue;
            const uint64_t i = first + tid + static_cast<uint64_t>(k) * BLOCK;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a.x[d * a.NT + i] = x[k][d];
                a.v[d * a.NT + i] = v[k][d];
                if (keep_t0) {
                    a.t0buf[d * a.NT + i] = x0[k][d];
                    a.t0buf[(3 + d) * a.NT + i] = v0[k][d];
                }
            }
            gen_store(g[k], a.state, a.S, i);
        }
    }
}

// ---- paper protocol: one launch per step, state through device memory ------------------------------
// generators whose state is uint32 rows (Hybrid Taus, LCG) or absent (no random force)
template <class Gen>
__global__ __launch_bounds__(kBulkBlock) void u32_step_kernel(uint32_t *st, uint64_t S, LdCoef q, uint64_t n,
                                                              float *x, float *v) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= n) return;
    Gen g;
    g.load(st, S, i);
    float gf[3];
    draw_forces(g, gf[0], gf[1], gf[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float xd = x[d * n + i], vd = v[d * n + i];
        ld_update(q, xd, vd, gf[d]);
        x[d * n + i] = xd;
        v[d * n + i] = vd;
    }
    g.store(st, S, i);
}

// Ran2 with its shuffle table left in device memory and touched at the selected entry only
// (Alg. 2 keeps each thread's part of the generator state in global memory between steps).
__global__ __launch_bounds__(kBulkBlock) void ran2_step_kernel(int32_t *st, uint64_t S, LdCoef q, uint64_t n,
                                                               float *x, float *v) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= n) return;
    Ran2 g;
    g.idum = st[i];
    g.idum2 = st[S + i];
    g.iym1 = static_cast<uint32_t>(st[2 * S + i]) - 1u;
    g.tab = st + 3 * S + i;
    g.tstride = S;
    const uint32_t w0 = g.next_top24(), w1 = g.next_top24(), w2 = g.next_top24(), w3 = g.next_top24();
    st[i] = g.idum;
    st[S + i] = g.idum2;
    st[2 * S + i] = static_cast<int32_t>(g.iym1 + 1u);
    float gf[3];
    gaussian_forces_top24(w0, w1, w2, w3, gf[0], gf[1], gf[2], Ran2::kTopScale);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float xd = x[d * n + i], vd = v[d * n + i];
        ld_update(q, xd, vd, gf[d]);
        x[d * n + i] = xd;
        v[d * n + i] = vd;
    }
}

// One block per (point, ensemble): thread j sums the six observables of the ensemble's tiles j,
// j + 256, ... in tile order (one tile's six partials are 48 contiguous bytes, so a wave reads
// consecutive tiles' whole records), then the block adds its threads' sums in a fixed order.  The
// order depends only on the ensemble's tile count.
constexpr int kFinBlock = 256;
__global__ __launch_bounds__(kFinBlock) void obs_finalize_kernel(const double *partials, uint32_t n_tiles,
                                                                 uint32_t P, const EnsDev *ens, double *out) {
    __shared__ double red[kFinBlock / 64][kNobs];
    const uint32_t p = blockIdx.x, e = blockIdx.y;
    const EnsDev &E = ens[e];
    const double *src = partials + (static_cast<uint64_t>(p) * n_tiles + E.tile_begin) * kNobs;
    double acc[kNobs] = {0, 0, 0, 0, 0, 0};
#pragma unroll 4
    for (uint32_t t = threadIdx.x; t < E.n_tiles; t += kFinBlock)
#pragma unroll
        for (int qi = 0; qi < kNobs; ++qi) acc[qi] += src[static_cast<uint64_t>(t) * kNobs + qi];
    double *dst = out + (static_cast<uint64_t>(e) * P + p) * kNobs;
    block_sum6<kFinBlock>(acc, red, dst);
    if (threadIdx.x < kNobs) dst[threadIdx.x] = E.n ? dst[threadIdx.x] / (3.0 * static_cast<double>(E.n)) : 0.0;
}

struct UploadBlob {
    uint32_t w[480];
};

__global__ __launch_bounds__(64) void upload_kernel(uint32_t *dst, UploadBlob b, uint32_t nwords) {
    for (uint32_t i = threadIdx.x; i < nwords; i += 64) dst[i] = b.w[i];
}

template <class Gen>
struct KernelTable {
    template <int B, int O>
    static const void *ptr() {
        return reinterpret_cast<const void *>(&ld_run_kernel<Gen, B, O>);
    }
    static const void *get(const ld_tuning &t) {
        const bool two = t.osc_per_thread == 2;
        switch (t.block) {
            case 64: return two ? ptr<64, 2>() : ptr<64, 1>();
            case 128: return two ? ptr<128, 2>() : ptr<128, 1>();
            case 256: return two ? ptr<256, 2>() : ptr<256, 1>();
            case 512: return two ? ptr<512, 2>() : ptr<512, 1>();
            default: return nullptr;
        }
    }
};

}  // namespace

const void *ld_run_kernel_ptr(int kind, const ld_tuning &t) {
    if (kind == RNGLD_RAN2) return KernelTable<Ran2>::get(t);
    if (kind == RNGLD_LCG) return KernelTable<Lcg32>::get(t);
    if (kind == RNGLD_NO_NOISE) return KernelTable<NoNoise>::get(t);
    return KernelTable<HybridTaus>::get(t);
}

size_t ld_run_lds_bytes(int kind, const ld_tuning &t) {
    return kind == RNGLD_RAN2 ? static_cast<size_t>(t.osc_per_thread) * kR2Tab * t.block * sizeof(int32_t) : 0;
}

hipError_t launch_ld_run(int kind, const LdArgs &a, const ld_tuning &t, uint32_t grid, hipStream_t st) {
    const void *fn = ld_run_kernel_ptr(kind, t);
    if (!fn) return hipErrorInvalidValue;
    LdArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchKernel(fn, dim3(grid), dim3(t.block), args, ld_run_lds_bytes(kind, t), st);
}

hipError_t launch_obs_finalize(const double *partials, uint32_t n_tiles, uint32_t P, const EnsDev *ens,
                               uint32_t n_ens, double *out, hipStream_t st) {
    if (P == 0 || n_ens == 0) return hipSuccess;
    obs_finalize_kernel<<<dim3(P, n_ens), kFinBlock, 0, st>>>(partials, n_tiles, P, ens, out);
    return hipGetLastError();
}

hipError_t launch_ld_step(int kind, void *state, uint64_t S, const LdCoef &coef, uint64_t n, float *x, float *v,
                          hipStream_t st) {
    if (n == 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((n + kBulkBlock - 1) / kBulkBlock));
    if (kind == RNGLD_HYBRID_TAUS)
        u32_step_kernel<HybridTaus><<<grid, kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, coef, n, x, v);
    else if (kind == RNGLD_LCG)
        u32_step_kernel<Lcg32><<<grid, kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, coef, n, x, v);
    else if (kind == RNGLD_NO_NOISE)
        u32_step_kernel<NoNoise><<<grid, kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, coef, n, x, v);
    else
        ran2_step_kernel<<<grid, kBulkBlock, 0, st>>>(static_cast<int32_t *>(state), S, coef, n, x, v);
    return hipGetLastError();
}

// copy small host data into device memory through kernel arguments (no memcpy node, so the copy
// can sit inside a captured graph and needs no pinned staging buffer)
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    const size_t words = (bytes + 3) / 4;
    const uint32_t *s = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    for (size_t off = 0; off < words; off += 480) {
        UploadBlob b{};
        const uint32_t nw = static_cast<uint32_t>(words - off < 480 ? words - off : 480);
        const size_t tail_bytes = bytes - off * 4;
        std::memcpy(b.w, s + off, nw * 4 <= tail_bytes ? nw * 4 : tail_bytes);
        upload_kernel<<<1, 64, 0, st>>>(d + off, b, nw);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rngld
