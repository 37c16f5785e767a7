// gen_int.hpp -- the integer steps of the per-thread generators.
//
// LCG of Eq. 1 with m = 2^32 (Sec. II.B), and the Tausworthe components of Hybrid Taus (Sec. II.D,
// Eq. 2 in L'Ecuyer's shift form; Appendix A Alg. 1).
//
// Plain C++, so that a CPU test can use it as well as the kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define RNGLD_HDI __host__ __device__ __forceinline__
#else
#define RNGLD_HDI inline
#endif

namespace rngld {

// ---- LCG of Eq. 1, m = 2^32 -------------------------------------------------------------------------
constexpr uint32_t kLcgMul = 1664525u;
constexpr uint32_t kLcgAdd = 1013904223u;

// On the device the multiply and the add are one v_mad_u64_u32 (the low word of a x + c) where
// the compiler would emit a 32-bit multiply and an add.
RNGLD_HDI uint32_t lcg_next(uint32_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t r;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(x), "s"(kLcgMul), "v"(static_cast<uint64_t>(kLcgAdd)) : "vcc");
    return static_cast<uint32_t>(r);
#else
    return kLcgMul * x + kLcgAdd;
#endif
}

// x advanced by n steps: the affine map x -> a x + c composed with itself by binary powering
// (a - 1 is even, so the geometric-sum closed form cannot use a modular inverse).
RNGLD_HDI uint32_t lcg_skip(uint32_t x, uint64_t n) {
    uint32_t mul = 1u, add = 0u;            // accumulated map
    uint32_t pm = kLcgMul, pa = kLcgAdd;    // map for 2^bit steps
    while (n) {
        if (n & 1u) {
            mul = pm * mul;
            add = pm * add + pa;
        }
        pa = pm * pa + pa;
        pm = pm * pm;
        n >>= 1;
    }
    return mul * x + add;
}

// low 32 bits of the 64-bit concatenation hi : lo shifted right by s, 0 < s < 32 (v_alignbit_b32)
RNGLD_HDI uint32_t funnel_shift_right(uint32_t hi, uint32_t lo, uint32_t s) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, s);
#else
    return static_cast<uint32_t>(((static_cast<uint64_t>(hi) << 32) | lo) >> s);
#endif
}

// ---- Tausworthe component for the trinomial x^K + x^Q + 1 with step S (Eq. 2) ---------------------
// The state occupies the top K bits; the low 32-K bits are dropped before the left shift.
//
// In terms of the component's bit sequence y (y_m = y_{m-K+Q} xor y_{m-K}), a word produced by
// this step holds 32 consecutive sequence bits, oldest in bit 31: its top K bits are the state
// and the low 32-K bits the next bits of the same sequence (the feedback computes them from state
// bits only, since S + 32 + Q <= 2K for the three components).  A seeded word is such a window
// only in its top K bits.
//
// The step is ((z & top K bits) << S) xor (((z << Q) xor z) >> (K - S)).  The two terms occupy
// disjoint bits: the first the top K - S bits, the second the 32 - K + S bits below them.  So the
// new word is the low half of the 64-bit concatenation (z >> (32 - K)) : ((z << Q) xor z) shifted
// right by K - S, one funnel shift (v_alignbit_b32) in place of a shift and a masked merge.
template <int Q, int S, int K>
RNGLD_HDI uint32_t tausworthe(uint32_t z) {
    static_assert(0 < S && S < K && K < 32 && 0 < Q, "component parameters");
    return funnel_shift_right(z >> (32 - K), (z << Q) ^ z, K - S);
}

// A x mod M for M = 2^31 - C and 0 <= x < M (the multiplicative steps of Ran2's two generators):
// the product p = A x, below 2^47, is H 2^31 + L, and 2^31 = C (mod M), so p = C H + L (mod M), where
// C H + L < 2 M takes one conditional subtraction.  One 32 x 32 -> 64-bit multiply and one
// multiply-add, against four multiplies for Schrage's method; the same exact residue.  On the
// device the multiply-add is one v_mad_u64_u32 on the whole product: the low word of
// p + H (C + 2^31) is L + C H, since the low word of p is L + (H mod 2) 2^31 and H 2^31 adds the
// same bit again (mod 2^32), so no mask is needed.
template <uint32_t A, uint32_t C>
RNGLD_HDI uint32_t mulmod_2p31m(uint32_t x) {
    static_assert(A < (1u << 16) && C < (1u << 14), "C H + L < 2 M");
    const uint64_t p = static_cast<uint64_t>(A) * x;
    const uint32_t H = static_cast<uint32_t>(p >> 31);
#if defined(__HIP_DEVICE_COMPILE__)
    uint64_t q;
    asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(q) : "v"(H), "s"(C + 0x80000000u), "v"(p) : "vcc");
    const uint32_t r = static_cast<uint32_t>(q);
#else
    const uint32_t r = (static_cast<uint32_t>(p) & 0x7fffffffu) + C * H;
#endif
    constexpr uint32_t m = 0x80000000u - C;
    return r >= m ? r - m : r;
}

// smallest word whose top K bits are not all zero
template <int K>
RNGLD_HDI uint32_t tausworthe_lift(uint32_t z) {
    constexpr uint32_t kFloor = 1u << (32 - K);
    return z < kFloor ? z + kFloor : z;
}

}  // namespace rngld
