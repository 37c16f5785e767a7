// k_rng.hip -- seeding and bare-generator kernels for the per-thread generators.
//
// One thread owns one stream (Sec. III.B, one generator per thread).  State rows are
// component-major ([row][S]) so that consecutive threads touch consecutive words (coalesced; the
// paper asks for coalesced seed arrays in Sec. III.B).  Ran2's 32-entry shuffle table lives in LDS
// as tab[t][lane] while a thread runs, so a data-dependent entry never leaves the chip and
// different lanes never share a bank row.
#include "internal.hpp"

namespace rngld {

namespace {

__global__ __launch_bounds__(kBulkBlock) void taus_seed_kernel(uint32_t *st, uint64_t S, uint64_t seed,
                                                               uint64_t stream_base, uint64_t col_offset,
                                                               uint64_t count) {
    const uint64_t t = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (t >= count) return;
    HybridTaus g;
    g.seed(seed, stream_base + t);
    g.store(st, S, col_offset + t);
}

__global__ __launch_bounds__(kBulkBlock) void ran2_seed_kernel(int32_t *st, uint64_t S, uint64_t seed,
                                                               uint64_t stream_base, uint64_t col_offset,
                                                               uint64_t count) {
    __shared__ int32_t tab[kR2Tab * kBulkBlock];
    const uint64_t t = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (t >= count) return;  // no block-wide synchronisation below
    Ran2 g;
    g.tab = tab + threadIdx.x;
    g.tstride = kBulkBlock;
    g.seed(seed, stream_base + t);
    g.store(st, S, col_offset + t);
}

__global__ __launch_bounds__(kBulkBlock) void lcg_seed_kernel(uint32_t *st, uint64_t S, uint64_t seed,
                                                              uint64_t stream_base, uint64_t col_offset,
                                                              uint64_t count, uint64_t leap) {
    const uint64_t t = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (t >= count) return;
    Lcg32 g;
    g.seed(seed, stream_base + t, leap);
    g.store(st, S, col_offset + t);
}

// generators whose state is uint32 rows (Hybrid Taus, LCG)
template <class Gen>
__global__ __launch_bounds__(kBulkBlock) void u32_uniform_kernel(uint32_t *st, uint64_t S, uint64_t per_stream,
                                                                 uint32_t *out) {
    const uint64_t j = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (j >= S) return;
    Gen g;
    g.load(st, S, j);
    uint32_t *o = out + j;
    for (uint64_t t = 0; t < per_stream; ++t) o[t * S] = g.next();
    g.store(st, S, j);
}

__global__ __launch_bounds__(kBulkBlock) void ran2_uniform_kernel(int32_t *st, uint64_t S, uint64_t per_stream,
                                                                  uint32_t *out) {
    __shared__ int32_t tab[kR2Tab * kBulkBlock];
    const uint64_t j = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (j >= S) return;
    Ran2 g;
    g.tab = tab + threadIdx.x;
    g.tstride = kBulkBlock;
    g.load(st, S, j);
    uint32_t *o = out + j;
    // streaming stores: 1.24-1.29e12 values/s at 2^20 streams x 1024 against 1.14e12 with ordinary
    // ones (the Hybrid Taus, LCG and Gaussian kernels measured no faster or slower with them)
    for (uint64_t t = 0; t < per_stream; ++t) __builtin_nontemporal_store(g.next_iym1() + 1u, o + t * S);
    g.store(st, S, j);
}

template <class Gen>
__device__ __forceinline__ void gaussian_pairs(Gen &g, uint64_t S, uint64_t per_stream, float *o) {
    for (uint64_t t = 0; t < per_stream; t += 2) {
        const uint32_t w0 = g.next();
        const uint32_t w1 = g.next();
        const float r = box_muller_radius(w0);
        float c, s;
        box_muller_angle(w1, c, s);
        o[t * S] = r * c;
        o[(t + 1) * S] = r * s;
    }
}

template <class Gen>
__global__ __launch_bounds__(kBulkBlock) void u32_gaussian_kernel(uint32_t *st, uint64_t S, uint64_t per_stream,
                                                                  float *out) {
    const uint64_t j = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (j >= S) return;
    Gen g;
    g.load(st, S, j);
    gaussian_pairs(g, S, per_stream, out + j);
    g.store(st, S, j);
}

__global__ __launch_bounds__(kBulkBlock) void ran2_gaussian_kernel(int32_t *st, uint64_t S, uint64_t per_stream,
                                                                   float *out) {
    __shared__ int32_t tab[kR2Tab * kBulkBlock];
    const uint64_t j = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (j >= S) return;
    Ran2 g;
    g.tab = tab + threadIdx.x;
    g.tstride = kBulkBlock;
    g.load(st, S, j);
    gaussian_pairs(g, S, per_stream, out + j);
    g.store(st, S, j);
}

__global__ __launch_bounds__(kBulkBlock) void box_muller_kernel(const uint32_t *words, uint64_t n_pairs,
                                                                float *out) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= n_pairs) return;
    const float r = box_muller_radius(words[2 * i]);
    float c, s;
    box_muller_angle(words[2 * i + 1], c, s);
    out[2 * i] = r * c;
    out[2 * i + 1] = r * s;
}

// the same transform in place: word pair i becomes Gaussian pair i (each thread reads its two
// words before it writes)
__global__ __launch_bounds__(kBulkBlock) void box_muller_inplace_kernel(uint32_t *buf, uint64_t n_pairs) {
    const uint64_t i = blockIdx.x * static_cast<uint64_t>(kBulkBlock) + threadIdx.x;
    if (i >= n_pairs) return;
    const uint32_t w0 = buf[2 * i], w1 = buf[2 * i + 1];
    const float r = box_muller_radius(w0);
    float c, s;
    box_muller_angle(w1, c, s);
    float *out = reinterpret_cast<float *>(buf);
    out[2 * i] = r * c;
    out[2 * i + 1] = r * s;
}

inline dim3 grid_for(uint64_t n) { return dim3(static_cast<unsigned>((n + kBulkBlock - 1) / kBulkBlock)); }

}  // namespace

hipError_t launch_seed(int kind, void *state, uint64_t S, uint64_t seed, uint64_t stream_base, uint64_t col_offset,
                       uint64_t count, uint64_t leap, hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (kind == RNGLD_LCG)
        lcg_seed_kernel<<<grid_for(count), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, seed, stream_base,
                                                                col_offset, count, leap);
    else if (kind == RNGLD_HYBRID_TAUS)
        taus_seed_kernel<<<grid_for(count), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, seed,
                                                                 stream_base, col_offset, count);
    else
        ran2_seed_kernel<<<grid_for(count), kBulkBlock, 0, st>>>(static_cast<int32_t *>(state), S, seed,
                                                                 stream_base, col_offset, count);
    return hipGetLastError();
}

hipError_t launch_bulk_uniform(int kind, void *state, uint64_t S, uint64_t per_stream, uint32_t *out,
                               hipStream_t st) {
    if (S == 0 || per_stream == 0) return hipSuccess;
    if (kind == RNGLD_LCG)
        u32_uniform_kernel<Lcg32><<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, per_stream, out);
    else if (kind == RNGLD_HYBRID_TAUS)
        u32_uniform_kernel<HybridTaus><<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, per_stream,
                                                                          out);
    else
        ran2_uniform_kernel<<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<int32_t *>(state), S, per_stream, out);
    return hipGetLastError();
}

hipError_t launch_bulk_gaussian(int kind, void *state, uint64_t S, uint64_t per_stream, float *out, hipStream_t st) {
    if (S == 0 || per_stream == 0) return hipSuccess;
    if (kind == RNGLD_LCG)
        u32_gaussian_kernel<Lcg32><<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S, per_stream,
                                                                      out);
    else if (kind == RNGLD_HYBRID_TAUS)
        u32_gaussian_kernel<HybridTaus><<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<uint32_t *>(state), S,
                                                                           per_stream, out);
    else
        ran2_gaussian_kernel<<<grid_for(S), kBulkBlock, 0, st>>>(static_cast<int32_t *>(state), S, per_stream, out);
    return hipGetLastError();
}

hipError_t launch_box_muller_inplace(uint32_t *buf, uint64_t n_pairs, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    box_muller_inplace_kernel<<<grid_for(n_pairs), kBulkBlock, 0, st>>>(buf, n_pairs);
    return hipGetLastError();
}

hipError_t launch_box_muller(const uint32_t *words, uint64_t n_pairs, float *out, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    box_muller_kernel<<<grid_for(n_pairs), kBulkBlock, 0, st>>>(words, n_pairs, out);
    return hipGetLastError();
}

}  // namespace rngld
