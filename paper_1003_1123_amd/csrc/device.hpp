// device.hpp -- device-side generators, uniform mapping, Box-Muller and the LD update for gfx950.
//
// Hybrid Taus: Sec. II.D (Eq. 2 in L'Ecuyer's shift form) and Appendix A Alg. 1.
// Ran2: Sec. II.C and Alg. 2, with a*x mod m for m = 2^31 - C evaluated from the 64-bit product
//       reduced with 2^31 = C (mod m) (gen_int.hpp); the state stays in 32-bit integers.
// Lagged Fibonacci: Sec. II.E Eq. 3 with addition mod 2^32 (the ring kernels live in k_lf.hip).
// Box-Muller: Sec. I; four uniforms give one oscillator-step's three force components
//       (Table II caption).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_int.hpp"

namespace rngld {

// ---- per-stream seeding: SplitMix64 (Steele, Lea & Flood 2014) in counter form -----------------
constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix_finalize(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// word i (0..3) of global stream j
__device__ __forceinline__ uint32_t stream_seed_word(uint64_t seed, uint64_t j, uint32_t i) {
    return static_cast<uint32_t>(splitmix_finalize(seed + (4ull * j + i + 1ull) * kGoldenGamma) >> 32);
}

// a ^ b ^ c ^ d in two instructions: gfx950's three-input bitwise op (truth table 0x96 is the
// three-way xor), which the compiler does not form from a chain of xors by itself
__device__ __forceinline__ uint32_t xor4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96) ^ d;
}

// The uniform mapping uses a word's top 24 bits only (below): kTop24 keeps them in place.
constexpr uint32_t kTop24 = 0xFFFFFF00u;

// (a ^ b ^ c ^ d) & kTop24 in two three-input bitwise ops: 0x96 is the three-way xor and 0x28 the
// truth table of (x ^ y) & z
__device__ __forceinline__ uint32_t xor4_top24(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    return __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_bitop3_b32(a, b, c, 0x96), d, kTop24, 0x28);
}

struct HybridTaus {
    uint32_t t1, t2, t3, lcg;
    static constexpr int kRows = 4;
    static constexpr float kTopScale = 0x1p-32f;  // next_top24() is the word with its low 8 bits clear

    __device__ __forceinline__ void step() {
        t1 = tausworthe<13, 12, 31>(t1);
        t2 = tausworthe<2, 4, 29>(t2);
        t3 = tausworthe<3, 17, 28>(t3);
        lcg = lcg_next(lcg);
    }
    __device__ __forceinline__ uint32_t next() {
        step();
        return xor4(t1, t2, t3, lcg);
    }
    // the next word with its low 8 bits cleared (what the uniform mapping reads)
    __device__ __forceinline__ uint32_t next_top24() {
        step();
        return xor4_top24(t1, t2, t3, lcg);
    }
    // state rows: uint32 [4][S]
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t S, uint64_t j) {
        t1 = st[j];
        t2 = st[S + j];
        t3 = st[2 * S + j];
        lcg = st[3 * S + j];
    }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t S, uint64_t j) const {
        st[j] = t1;
        st[S + j] = t2;
        st[2 * S + j] = t3;
        st[3 * S + j] = lcg;
    }
    __device__ __forceinline__ void seed(uint64_t seed, uint64_t stream) {
        t1 = tausworthe_lift<31>(stream_seed_word(seed, stream, 0));
        t2 = tausworthe_lift<29>(stream_seed_word(seed, stream, 1));
        t3 = tausworthe_lift<28>(stream_seed_word(seed, stream, 2));
        lcg = stream_seed_word(seed, stream, 3);
    }
};

// ---- Quick-and-Dirty LCG (Eq. 1 with m = 2^32) ------------------------------------------------------
// One 32-bit word per stream; the output is the updated word.  Seeding: with leap = 0 stream j
// starts from its own seed word; with leap > 0 the streams divide one sequence (the cycle division
// of Sec. III): stream j starts at position j * leap of the sequence from seed word (0, 0).
struct Lcg32 {
    uint32_t x;
    static constexpr int kRows = 1;
    static constexpr float kTopScale = 0x1p-32f;

    __device__ __forceinline__ uint32_t next() {
        x = lcg_next(x);
        return x;
    }
    __device__ __forceinline__ uint32_t next_top24() { return next() & kTop24; }
    __device__ __forceinline__ void load(const uint32_t *st, uint64_t, uint64_t j) { x = st[j]; }
    __device__ __forceinline__ void store(uint32_t *st, uint64_t, uint64_t j) const { st[j] = x; }
    __device__ __forceinline__ void seed(uint64_t seed, uint64_t stream, uint64_t leap) {
        x = leap ? lcg_skip(stream_seed_word(seed, 0, 0), stream * leap) : stream_seed_word(seed, stream, 0);
    }
};

// ---- no random force ----------------------------------------------------------------------------------
// The deterministic part of the LD step alone (Fig. 6's timing of the dynamics with no random forces): no
// state, no draws; the kernels use a zero force in place of the Box-Muller output.
struct NoNoise {
    static constexpr int kRows = 0;
    __device__ __forceinline__ void load(const uint32_t *, uint64_t, uint64_t) {}
    __device__ __forceinline__ void store(uint32_t *, uint64_t, uint64_t) const {}
};

// ---- Ran2 -------------------------------------------------------------------------------------------
// Ran2's two generators x -> A x mod M with M = 2^31 - C (Numerical Recipes' constants)
constexpr int32_t kR2M1 = 2147483563, kR2A1 = 40014;
constexpr int32_t kR2M2 = 2147483399, kR2A2 = 40692;
constexpr uint32_t kR2C1 = 85, kR2C2 = 249;
static_assert(kR2M1 == 2147483648ll - kR2C1 && kR2M2 == 2147483648ll - kR2C2, "M = 2^31 - C");
constexpr int kR2Tab = 32;
constexpr int32_t kR2Imm1 = kR2M1 - 1;
constexpr uint32_t kR2Ndiv = 1u + static_cast<uint32_t>(kR2Imm1) / kR2Tab;

__device__ __forceinline__ int32_t ran2_lcg1(int32_t x) {
    return static_cast<int32_t>(mulmod_2p31m<kR2A1, kR2C1>(static_cast<uint32_t>(x)));
}
__device__ __forceinline__ int32_t ran2_lcg2(int32_t x) {
    return static_cast<int32_t>(mulmod_2p31m<kR2A2, kR2C2>(static_cast<uint32_t>(x)));
}

// iy / Ndiv for 1 <= iy < 2^31 as (iy m) >> 57 with m = 2^31 + 65: m Ndiv - 2^57 = 2^26 - 130, so
// the product overshoots iy / Ndiv by less than iy 2^26 / (Ndiv 2^57) < 1 / Ndiv, never enough to
// reach the next integer.
constexpr uint32_t kR2SlotMul = 0x80000041u;
static_assert(static_cast<unsigned __int128>(kR2SlotMul) * kR2Ndiv - (static_cast<unsigned __int128>(1) << 57) ==
                  (1u << 26) - 130u,
              "slot multiplier");

// Ran2 stream with its shuffle table in LDS: tab[t * tstride] is entry t of this thread's table.
// The last output is kept as iym1 = iy - 1, which is also what the uniform mapping reads.
struct Ran2 {
    int32_t idum, idum2;
    uint32_t iym1;
    int32_t *tab;
    uint64_t tstride;
    static constexpr int kRows = 35;
    // next_top24() returns (iy - 1) with its low 7 bits clear, half of the top-24 word of next()
    static constexpr float kTopScale = 0x1p-31f;

    // bits 25..29 of the product's high word: one bit-field extract (written out, since the compiler
    // otherwise folds the extract into the address arithmetic as a shift and a mask)
    __device__ __forceinline__ static uint32_t slot_of(uint32_t hi) {
        uint32_t slot;
        asm("v_bfe_u32 %0, %1, 25, 5" : "=v"(slot) : "v"(hi));
        return slot;
    }
    // one step of Alg. 2; returns iy - 1 in [0, M1 - 2]
    __device__ __forceinline__ uint32_t next_iym1() {
        idum = ran2_lcg1(idum);
        idum2 = ran2_lcg2(idum2);
        // entry iy / Ndiv, from the 64-bit (iym1 + 1) m (one multiply-add)
        const uint64_t prod = static_cast<uint64_t>(iym1) * kR2SlotMul + kR2SlotMul;
        int32_t *cell = tab + slot_of(static_cast<uint32_t>(prod >> 32)) * tstride;
        // iy - 1 = entry - idum2 - 1, plus Imm1 when that is negative: as unsigned words the
        // smaller of e and e + Imm1 (e + Imm1 wraps exactly when e is negative)
        const uint32_t e = static_cast<uint32_t>(*cell) + ~static_cast<uint32_t>(idum2);
        *cell = idum;
        const uint32_t f = e + static_cast<uint32_t>(kR2Imm1);
        iym1 = e < f ? e : f;
        return iym1;
    }
    // word fed to the uniform mapping: iy - 1 spans [0, 2^31), doubled
    __device__ __forceinline__ uint32_t next() { return next_iym1() << 1; }
    __device__ __forceinline__ uint32_t next_top24() { return next_iym1() & (kTop24 >> 1); }

    // state rows: int32 [35][S]: idum, idum2, iy, iv[0..31]
    __device__ __forceinline__ void load(const int32_t *st, uint64_t S, uint64_t j) {
        idum = st[j];
        idum2 = st[S + j];
        iym1 = static_cast<uint32_t>(st[2 * S + j]) - 1u;
        for (int t = 0; t < kR2Tab; ++t) tab[t * tstride] = st[(3 + t) * S + j];
    }
    __device__ __forceinline__ void store(int32_t *st, uint64_t S, uint64_t j) const {
        st[j] = idum;
        st[S + j] = idum2;
        st[2 * S + j] = static_cast<int32_t>(iym1 + 1u);
        for (int t = 0; t < kR2Tab; ++t) st[(3 + t) * S + j] = tab[t * tstride];
    }
    // Alg. 2 initialisation: idum2 = idum; 8 discarded LCG1 steps, then 32 filling iv[31]..iv[0]
    __device__ __forceinline__ void seed(uint64_t seed, uint64_t stream) {
        const uint32_t w = stream_seed_word(seed, stream, 0);
        int32_t x = 1 + static_cast<int32_t>(w % static_cast<uint32_t>(kR2M1 - 1));
        idum2 = x;
        for (int t = 0; t < 8; ++t) x = ran2_lcg1(x);
        for (int t = kR2Tab - 1; t >= 0; --t) {
            x = ran2_lcg1(x);
            tab[t * tstride] = x;
        }
        idum = x;
        iym1 = static_cast<uint32_t>(tab[0]) - 1u;
    }
};

// ---- uniform mapping and Box-Muller ----------------------------------------------------------------
// u_open = ((w >> 8) + 1) 2^-24 in (0, 1]; u_half = (w >> 8) 2^-24 in [0, 1); both exact in FP32.
// They are evaluated on m = w & kTop24, whose conversion to FP32 is exact (24 significant bits):
// u_half = float(m) 2^-32 and u_open = float(m) 2^-32 + 2^-24 as one FMA, exact because the result
// is representable.  A generator that clears the low bits in its last instruction (Hybrid Taus:
// one three-input bitwise op) so saves the shift and the add of the plain form.
// The transform uses the hardware transcendentals: -2 ln u = -2 ln(2) log2(u) with v_log_f32 and
// v_sqrt_f32, and v_cos_f32 / v_sin_f32, whose argument is in revolutions (sin(2 pi x)), so the
// angle needs no multiply.  Checked over every one of the 2^24 possible inputs of each factor
// against double precision: radius error < 5e-7, cosine/sine error < 1.3e-7, so every Gaussian is
// within 2e-6 of its exact value (r <= sqrt(48 ln 2)).
constexpr float kMinusTwoLn2 = -1.38629436f;

// `scale` is the weight of the word's lowest bit: 2^-32 for a word with its low 8 bits clear, 2^-31
// for the same bits one place lower (Ran2's iy - 1); either way float(m) scale is exact.
__device__ __forceinline__ float u_open_top24(uint32_t m, float scale = 0x1p-32f) {
    return __builtin_fmaf(static_cast<float>(m), scale, 0x1p-24f);
}
__device__ __forceinline__ float u_half_top24(uint32_t m, float scale = 0x1p-32f) {
    return static_cast<float>(m) * scale;
}

__device__ __forceinline__ float box_muller_radius_top24(uint32_t m, float scale = 0x1p-32f) {
    return __builtin_amdgcn_sqrtf(kMinusTwoLn2 * __builtin_amdgcn_logf(u_open_top24(m, scale)));
}
__device__ __forceinline__ float box_muller_radius(uint32_t w) { return box_muller_radius_top24(w & kTop24); }
__device__ __forceinline__ void box_muller_angle(uint32_t w, float &c, float &s) {
    const float u = u_half_top24(w & kTop24);
    c = __builtin_amdgcn_cosf(u);
    s = __builtin_amdgcn_sinf(u);
}

// three force components from one oscillator-step's four words, given with their low 8 bits clear
// (or, with scale 2^-31, the same 24 bits one place lower)
__device__ __forceinline__ void gaussian_forces_top24(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3, float &gx,
                                                      float &gy, float &gz, float scale = 0x1p-32f) {
    const float r0 = box_muller_radius_top24(m0, scale);
    const float u1 = u_half_top24(m1, scale);
    gx = r0 * __builtin_amdgcn_cosf(u1);
    gy = r0 * __builtin_amdgcn_sinf(u1);
    gz = box_muller_radius_top24(m2, scale) * __builtin_amdgcn_cosf(u_half_top24(m3, scale));
}
// the same from whole words
__device__ __forceinline__ void gaussian_forces(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, float &gx,
                                                float &gy, float &gz) {
    gaussian_forces_top24(w0 & kTop24, w1 & kTop24, w2 & kTop24, w3 & kTop24, gx, gy, gz);
}

// ---- LD update ----------------------------------------------------------------------------------------
// underdamped semi-implicit Euler-Maruyama (scheme 0) or overdamped Eq. 5 (scheme 1), per component
struct LdCoef {
    float c, kap, sig, h;  // scheme 0: c = 1 - gamma h, kap = k h / m, sig = sqrt(2 gamma kT h / m)
    float odc, ods;        // scheme 1: odc = k h / xi, ods = sqrt(2 kT h / xi), xi = m gamma
    int32_t scheme;
    int32_t pad;
};

template <int SCHEME>
__device__ __forceinline__ void ld_update_s(const LdCoef &q, float &x, float &v, float g) {
    if constexpr (SCHEME == 0) {
        v = q.c * v - q.kap * x + q.sig * g;
        x = x + q.h * v;
    } else {
        x = x - q.odc * x + q.ods * g;
    }
}
// runtime-selected scheme (one uniform branch; hot loops dispatch once outside the loop instead)
__device__ __forceinline__ void ld_update(const LdCoef &q, float &x, float &v, float g) {
    if (q.scheme == 0)
        ld_update_s<0>(q, x, v, g);
    else
        ld_update_s<1>(q, x, v, g);
}

// ---- reductions -----------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m, 64);
    return a;
}

// Six per-thread FP64 sums -> one fixed-order block total written by threads 0..5 to dst.
// Every thread of the block must call it (it synchronises the block twice).
template <int BLOCK>
__device__ __forceinline__ void block_sum6(const double (&q)[6], double (*red)[6], double *dst) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double s = wave_sum(q[i]);
        if (lane == 0) red[wave][i] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) s += red[w][threadIdx.x];
        dst[threadIdx.x] = s;
    }
    __syncthreads();
}

// the six observables of one oscillator's three coordinates, FP64 products of FP32 values
__device__ __forceinline__ void add_observables(double (&q)[6], const float (&x)[3], const float (&v)[3],
                                                const float (&x0)[3], const float (&v0)[3], bool after_t0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xd = x[d], vd = v[d];
        q[0] += xd * xd;
        q[1] += vd * vd;
        q[2] += xd * vd;
        q[3] += xd;
        if (after_t0) {
            q[4] += xd * static_cast<double>(x0[d]);
            q[5] += vd * static_cast<double>(v0[d]);
        }
    }
}

}  // namespace rngld
