// Wide-access probe for the lagged-Fibonacci run's traffic: each wave moves 1024-word slices of a
// 32 MB region with two loads per store (two source slices, one destination slice), either as 4-byte
// device-scope (agent) accesses, 16 loads and 16 stores of 64 consecutive words (mode 3, as in
// store_alignment.hip), or as 16-byte buffer loads and stores with the sc1 cache policy, each lane
// moving four consecutive words (mode 4); loads and stores shifted by the given number of words from
// 256-byte alignment.  All accesses stay inside the buffer (buffer accesses are also range-checked)
// and every loop is bounded.
// Build and run: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//   paper_1003_1123_amd/csrc/probes/wide_access.hip -o wide_access && ./wide_access
// Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t ald(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void ast(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// mode 3: 4-byte agent-scope accesses; mode 4: 16-byte sc1 buffer accesses
__global__ __launch_bounds__(1024) void slices(uint32_t *buf, uint32_t bytes, uint32_t nchunks, uint32_t iters,
                                               uint32_t mis_ld, uint32_t mis_st, int mode, uint32_t *sink) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gw = blockIdx.x * 16u + (threadIdx.x >> 6), nw = gridDim.x * 16u;
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(buf, 0, bytes, 0x00020000);
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t c = (gw + it * nw) % nchunks;
        const uint32_t c2 = (c + nchunks / 2) % nchunks;
        const uint32_t c3 = (c + nchunks / 4) % nchunks;
        if (mode == 3) {
            const uint32_t *src = buf + c * 1024u + mis_ld, *src2 = buf + c3 * 1024u + mis_ld;
            uint32_t *dst = buf + c2 * 1024u + mis_st;
            uint32_t v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = ald(src + lane + 64 * r) + ald(src2 + lane + 64 * r);
#pragma unroll
            for (int r = 0; r < 16; ++r) ast(dst + lane + 64 * r, v[r] + 1u);
        } else {
            const uint32_t s1 = (c * 1024u + mis_ld) * 4u, s2 = (c3 * 1024u + mis_ld) * 4u, d = (c2 * 1024u + mis_st) * 4u;
            v4u v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[r] = __builtin_amdgcn_raw_buffer_load_b128(rs, s1 + 16u * lane + 1024u * r, 0, 16) +
                       __builtin_amdgcn_raw_buffer_load_b128(rs, s2 + 16u * lane + 1024u * r, 0, 16);
#pragma unroll
            for (int r = 0; r < 4; ++r) __builtin_amdgcn_raw_buffer_store_b128(v[r] + 1u, rs, d + 16u * lane + 1024u * r, 0, 16);
        }
    }
    if (sink[0] == 0x12345678u) sink[1] = 1;
}

int main() {
    const uint64_t words = 8ull << 20;  // 32 MB
    const uint32_t nchunks = static_cast<uint32_t>((words - 2048) / 1024);
    uint32_t *buf, *sink;
    CHK(hipMalloc(&buf, words * 4));
    CHK(hipMalloc(&sink, 256));
    CHK(hipMemset(buf, 0, words * 4));
    CHK(hipMemset(sink, 0, 256));
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    const uint32_t iters = 400;
    const int blocks = 256;
    const uint32_t mis[][2] = {{0, 0}, {13, 0}, {2, 0}, {13, 13}};
    for (int mode = 3; mode < 5; ++mode)
        for (auto &m : mis) {
            slices<<<blocks, 1024>>>(buf, (uint32_t)(words * 4), nchunks, 20, m[0], m[1], mode, sink);  // warm
            CHK(hipEventRecord(e0));
            slices<<<blocks, 1024>>>(buf, (uint32_t)(words * 4), nchunks, iters, m[0], m[1], mode, sink);
            CHK(hipEventRecord(e1));
            CHK(hipEventSynchronize(e1));
            float ms;
            CHK(hipEventElapsedTime(&ms, e0, e1));
            const double bytes = (double)blocks * 16 * iters * 1024 * 4 * 3;
            printf("mode %d (%s) mis ld %2u st %2u: %.3f ms, %.2f TB/s\n", mode, mode == 3 ? "2ld+st dword" : "2ld+st dwordx4",
                   m[0], m[1], ms, bytes / ms / 1e9);
        }
    return 0;
}
