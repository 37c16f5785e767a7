// VALU issue-rate probe: 8 independent chains per lane, one instruction kind per kernel.
// Build and run: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//   paper_1003_1123_amd/csrc/probes/valu_rates.hip -o valu_rates && ./valu_rates
// Prints lane-instructions per second for each instruction kind, relative to 256 CUs x 64 lanes x
// 2.4 GHz.  Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <vector>

#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

template <int OP>
__global__ __launch_bounds__(256) void probe(uint32_t *out, int iters) {
    uint32_t a[8];
    float f[8];
    const uint32_t gid = blockIdx.x * 256 + threadIdx.x;
    for (int i = 0; i < 8; ++i) { a[i] = gid * 2654435761u + i * 97u + 1u; f[i] = 0.25f + 1e-7f * (gid & 1023) + 0.01f * i; }
    const uint32_t k = gid | 1u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (OP == 0) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(k));
            if (OP == 1) asm volatile("v_log_f32 %0, %0" : "+v"(f[i]));
            if (OP == 2) asm volatile("v_sqrt_f32 %0, %0" : "+v"(f[i]));
            if (OP == 3) asm volatile("v_cos_f32 %0, %0" : "+v"(f[i]));
            if (OP == 4) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
            if (OP == 5) asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(f[i]) : "v"(a[i]));
            if (OP == 6) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(f[i]) : "v"(f[(i + 1) & 7]));
            if (OP == 7) {  // one transcendental and three full-rate ops
                asm volatile("v_log_f32 %0, %0" : "+v"(f[i]));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(k));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[(i + 1) & 7]) : "v"(k));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[(i + 2) & 7]) : "v"(k));
            }
            if (OP == 8) {  // one mul_lo and three full-rate ops
                asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[i]) : "v"(k));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[(i + 1) & 7]) : "v"(k));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[(i + 2) & 7]) : "v"(k));
                asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[(i + 3) & 7]) : "v"(k));
            }
            if (OP == 9) asm volatile("v_and_or_b32 %0, %0, %1, %1" : "+v"(a[i]) : "v"(k));
            if (OP == 10) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a[i]) : "v"(k));
        }
    }
    uint32_t s = 0;
    for (int i = 0; i < 8; ++i) s += a[i] ^ __float_as_uint(f[i]);
    out[gid] = s;
}

template <int OP>
int run(const char *name, int per_iter, uint32_t *d, int blocks, int iters) {
    hipEvent_t e0, e1;
    CHK(hipEventCreate(&e0));
    CHK(hipEventCreate(&e1));
    probe<OP><<<blocks, 256>>>(d, iters);  // warm-up
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) probe<OP><<<blocks, 256>>>(d, iters);
    CHK(hipEventRecord(e1));
    CHK(hipEventSynchronize(e1));
    float ms;
    CHK(hipEventElapsedTime(&ms, e0, e1));
    const double lane_instr = 5.0 * blocks * 256.0 * iters * 8.0 * per_iter;
    const double rate = lane_instr / (ms * 1e-3);
    // one full-rate wave64 instruction per SIMD every 4 cycles: 256 CU x 64 lanes x clock
    printf("%-28s %8.3f ms  %.3e lane-instr/s  = %.3f x (256 CU * 64 lanes * 2.4 GHz)\n", name, ms / 5, rate,
           rate / (256.0 * 64 * 2.4e9));
    fflush(stdout);
    return 0;
}

int main() {
    const int blocks = 256 * 4 * 8 / 4 * 2;  // 4096 blocks of 4 waves: 16 waves per CU
    const int iters = 2048;
    uint32_t *d;
    CHK(hipMalloc(&d, sizeof(uint32_t) * blocks * 256));
    int rc = 0;
    rc |= run<0>("v_xor_b32", 1, d, blocks, iters);
    rc |= run<9>("v_and_or_b32", 1, d, blocks, iters);
    rc |= run<10>("v_cndmask_b32", 1, d, blocks, iters);
    rc |= run<6>("v_fma_f32", 1, d, blocks, iters);
    rc |= run<5>("v_cvt_f32_u32", 1, d, blocks, iters);
    rc |= run<4>("v_mul_lo_u32", 1, d, blocks, iters);
    rc |= run<1>("v_log_f32", 1, d, blocks, iters);
    rc |= run<2>("v_sqrt_f32", 1, d, blocks, iters);
    rc |= run<3>("v_cos_f32", 1, d, blocks, iters);
    rc |= run<7>("1 log + 3 xor (per 4)", 4, d, blocks, iters);
    rc |= run<8>("1 mul_lo + 3 xor (per 4)", 4, d, blocks, iters);
    CHK(hipFree(d));
    printf("probe done rc=%d\n", rc);
    return rc;
}
