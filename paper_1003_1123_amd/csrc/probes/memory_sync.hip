// Latency/bandwidth probe for device-scope (agent) accesses. Every loop is bounded.
// Build and run: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//   paper_1003_1123_amd/csrc/probes/memory_sync.hip -o memory_sync && ./memory_sync
// Measures the dependent latency of device-scope loads, store + completion, a cross-CU flag
// ping-pong, and streaming bandwidth with plain and device-scope accesses over a 32 MB and a 2 GB
// region.  Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>
#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__device__ __forceinline__ uint32_t ald(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void ast(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// 1. pointer chase with agent loads: next = buf[cur]; buf holds a permutation cycle (stride 4099 words)
__global__ void chase(const uint32_t *buf, uint32_t steps, uint64_t *out) {
    if (threadIdx.x != 0) return;
    uint32_t cur = 0;
    const uint64_t t0 = wall_clock64();
    for (uint32_t i = 0; i < steps; ++i) cur = ald(buf + cur);
    const uint64_t t1 = wall_clock64();
    out[0] = t1 - t0;
    out[1] = cur;
}
// 2. store + ack
__global__ void store_ack(uint32_t *buf, uint32_t steps, uint64_t *out) {
    if (threadIdx.x != 0) return;
    const uint64_t t0 = wall_clock64();
    for (uint32_t i = 0; i < steps; ++i) {
        ast(buf + (i * 4099u) % (1u << 22), i);
        __builtin_amdgcn_s_waitcnt(0);
    }
    out[2] = wall_clock64() - t0;
}
// 3. ping-pong between block 0 and block 1 (launched on different CUs), bounded
__global__ void pingpong(uint32_t *flags, uint32_t rounds, uint64_t *out) {
    if (threadIdx.x != 0) return;
    const uint32_t me = blockIdx.x;  // 0 or 1
    uint32_t *mine = flags + 64 * me, *other = flags + 64 * (1 - me);
    const uint64_t t0 = wall_clock64();
    uint32_t fails = 0;
    for (uint32_t r = 1; r <= rounds; ++r) {
        if (me == 0) {
            ast(mine, r);
            uint32_t spins = 0;
            while (ald(other) < r && ++spins < (1u << 22)) {}
            if (spins >= (1u << 22)) { ++fails; break; }
        } else {
            uint32_t spins = 0;
            while (ald(other) < r && ++spins < (1u << 22)) {}
            if (spins >= (1u << 22)) { ++fails; break; }
            ast(mine, r);
        }
    }
    if (me == 0) { out[3] = wall_clock64() - t0; out[4] = fails; }
}
// 4. streaming: each thread reads one word and writes one word per iteration over a region of `words`
__global__ void stream(uint32_t *buf, uint64_t words, uint32_t iters, int agent) {
    const uint64_t gid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, nth = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it)
        for (uint64_t i = gid; i < words / 2; i += nth) {
            const uint32_t v = agent ? ald(buf + i) : buf[i];
            acc += v;
            if (agent) ast(buf + words / 2 + i, v + it); else buf[words / 2 + i] = v + it;
        }
    if (acc == 0x12345678u) buf[0] = acc;
}

int main() {
    const uint64_t W = 1ull << 22;  // 16 MB of words for chase/store
    uint32_t *buf; uint64_t *out;
    CHK(hipMalloc(&buf, W * 4));
    CHK(hipMalloc(&out, 64));
    std::vector<uint32_t> h(W);
    for (uint64_t i = 0; i < W; ++i) h[i] = (uint32_t)((i + 4099u) % W);
    CHK(hipMemcpy(buf, h.data(), W * 4, hipMemcpyHostToDevice));
    CHK(hipMemset(out, 0, 64));
    const uint32_t steps = 20000;
    chase<<<1, 64>>>(buf, steps, out); CHK(hipGetLastError()); CHK(hipDeviceSynchronize());
    store_ack<<<1, 64>>>(buf, steps, out); CHK(hipGetLastError()); CHK(hipDeviceSynchronize());
    uint32_t *flags; CHK(hipMalloc(&flags, 4096)); CHK(hipMemset(flags, 0, 4096));
    pingpong<<<2, 64>>>(flags, steps, out); CHK(hipGetLastError()); CHK(hipDeviceSynchronize());
    uint64_t o[5]; CHK(hipMemcpy(o, out, 40, hipMemcpyDeviceToHost));
    printf("agent load latency (dependent)   : %.0f ns\n", o[0] * 10.0 / steps);
    printf("agent store + waitcnt            : %.0f ns\n", o[2] * 10.0 / steps);
    printf("flag ping-pong round (2 hops)    : %.0f ns (fails %llu)\n", o[3] * 10.0 / steps, (unsigned long long)o[4]);
    fflush(stdout);
    // streaming
    for (uint64_t mb : {32ull, 2048ull}) {
        const uint64_t words = mb << 18;
        uint32_t *b2; CHK(hipMalloc(&b2, words * 4)); CHK(hipMemset(b2, 0, words * 4));
        for (int agent : {0, 1}) {
            const uint32_t iters = mb == 32 ? 64 : 2;
            hipEvent_t e0, e1; CHK(hipEventCreate(&e0)); CHK(hipEventCreate(&e1));
            stream<<<2048, 256>>>(b2, words, 1, agent); CHK(hipGetLastError()); CHK(hipDeviceSynchronize());
            CHK(hipEventRecord(e0));
            stream<<<2048, 256>>>(b2, words, iters, agent);
            CHK(hipEventRecord(e1)); CHK(hipEventSynchronize(e1));
            float ms; CHK(hipEventElapsedTime(&ms, e0, e1));
            printf("stream %4llu MB %-6s: %.2f TB/s (read+write)\n", (unsigned long long)mb, agent ? "agent" : "plain",
                   (double)words * 4 * iters / (ms * 1e-3) / 1e12);
            fflush(stdout);
        }
        CHK(hipFree(b2));
    }
    printf("probe done\n");
    return 0;
}
