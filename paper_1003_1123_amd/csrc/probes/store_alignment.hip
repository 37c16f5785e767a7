// Alignment probe for device-scope (agent) wave accesses: each wave streams 1024-word slices (16
// loads and/or 16 stores of 64 consecutive words) over a 32 MB region, with the loads and the
// stores shifted by a given number of words from 256-byte alignment.  All accesses stay inside the
// buffer and every loop is bounded.
// Build and run: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//   paper_1003_1123_amd/csrc/probes/store_alignment.hip -o store_alignment && ./store_alignment
// Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__device__ __forceinline__ uint32_t ald(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void ast(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// mode 0: loads + stores; 1: loads only; 2: stores only; 3: two loads per store (two source slices)
__global__ __launch_bounds__(1024) void slices(uint32_t *buf, uint32_t nchunks, uint32_t iters, uint32_t mis_ld,
                                               uint32_t mis_st, int mode, uint32_t *sink) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gw = blockIdx.x * 16u + (threadIdx.x >> 6), nw = gridDim.x * 16u;
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t c = (gw + it * nw) % nchunks;
        const uint32_t c2 = (c + nchunks / 2) % nchunks;
        const uint32_t *src = buf + c * 1024u + mis_ld;
        uint32_t *dst = buf + c2 * 1024u + mis_st;
        uint32_t v[16];
        if (mode == 3) {
            const uint32_t *src2 = buf + ((c + nchunks / 4) % nchunks) * 1024u + mis_ld;
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = ald(src + lane + 64 * r) + ald(src2 + lane + 64 * r);
        } else if (mode != 2) {
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = ald(src + lane + 64 * r);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = it + r;
        }
        if (mode != 1) {
#pragma unroll
            for (int r = 0; r < 16; ++r) ast(dst + lane + 64 * r, v[r] + 1u);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) acc += v[r];
        }
    }
    if (acc == 0x12345678u) sink[0] = acc;
}

int main() {
    const uint64_t words = 8ull << 20;  // 32 MB
    const uint32_t nchunks = static_cast<uint32_t>((words - 2048) / 1024);
    uint32_t *buf, *sink;
    CHK(hipMalloc(&buf, words * 4));
    CHK(hipMalloc(&sink, 256));
    CHK(hipMemset(buf, 0, words * 4));
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    const uint32_t iters = 400;
    const int blocks = 256;
    const uint32_t mis[][2] = {{0, 0}, {13, 0}, {0, 13}, {13, 13}, {1, 26}, {16, 16}, {32, 32}};
    for (int mode = 0; mode < 4; ++mode)
        for (auto &m : mis) {
            slices<<<blocks, 1024>>>(buf, nchunks, 20, m[0], m[1], mode, sink);  // warm
            CHK(hipEventRecord(e0));
            slices<<<blocks, 1024>>>(buf, nchunks, iters, m[0], m[1], mode, sink);
            CHK(hipEventRecord(e1));
            CHK(hipEventSynchronize(e1));
            float ms;
            CHK(hipEventElapsedTime(&ms, e0, e1));
            const double bytes = (double)blocks * 16 * iters * 1024 * 4 * (mode == 0 ? 2 : (mode == 3 ? 3 : 1));
            printf("mode %d (%s) mis ld %2u st %2u: %.3f ms, %.2f TB/s\n", mode,
                   mode == 0 ? "ld+st" : (mode == 1 ? "ld" : (mode == 2 ? "st" : "2ld+st")), m[0], m[1], ms,
                   bytes / ms / 1e9);
        }
    return 0;
}
