// CPU check of the integer generator steps in paper_1003_1123_amd/csrc/gen_int.hpp: the Tausworthe
// step's funnel-shift form against the masked shift-and-xor of Eq. 2 on arbitrary words; the words
// it produces from random seeds against the component's bit recurrence y_m = y_{m-K+Q} xor y_{m-K}
// (consecutive words are windows of one bit sequence, S bits apart); the LCG's n-step map (the
// generator jump of the segment-parallel runs) against n single steps; and the modular product
// A x mod (2^31 - C) of Ran2's two generators (mulmod_2p31m) against the plain 64-bit remainder,
// at random and at the ends of its range, with the device's mask-free form of its reduction.
// Prints "ok" on success.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "../../paper_1003_1123_amd/csrc/gen_int.hpp"

using namespace rngld;

static uint64_t sm_state = 0x1234567887654321ull;
static uint32_t rnd() {
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return static_cast<uint32_t>((z ^ (z >> 31)) >> 32);
}

template <int Q, int S, int K>
static int check_component(int n_seeds, int n_steps) {
    int bad = 0;
    // the funnel-shift form of the step equals Eq. 2's masked shift-and-xor on arbitrary words
    for (int t = 0; t < 1 << 16; ++t) {
        const uint32_t z = t < 64 ? (t < 32 ? 1u << t : ~(1u << (t - 32))) : rnd();
        const uint32_t plain = ((z & ~((1u << (32 - K)) - 1u)) << S) ^ (((z << Q) ^ z) >> (K - S));
        if (tausworthe<Q, S, K>(z) != plain) ++bad;
    }
    for (int t = 0; t < n_seeds; ++t) {
        const uint32_t z0 = tausworthe_lift<K>(rnd());
        std::vector<uint32_t> w(n_steps + 1);
        w[0] = z0;
        for (int n = 1; n <= n_steps; ++n) w[n] = tausworthe<Q, S, K>(w[n - 1]);
        // produced words are 32-bit windows of the bit sequence, S bits apart
        for (int n = 1; n < n_steps && bad < 10; ++n) {
            // bit i of the sequence window of word n (i = 0 oldest) is bit 31 - i
            auto bit = [&](int word, int i) { return (w[word] >> (31 - i)) & 1u; };
            for (int i = 0; i + S < 32; ++i)
                if (bit(n, i + S) != bit(n + 1, i)) ++bad;  // overlap of consecutive windows
            for (int i = K; i < 32; ++i)
                if (bit(n, i) != (bit(n, i - K + Q) ^ bit(n, i - K))) ++bad;  // recurrence inside one word
        }
    }
    if (bad) std::printf("component (%d,%d,%d): %d mismatches\n", Q, S, K, bad);
    return bad;
}

template <uint32_t A, uint32_t C>
static int check_mulmod() {
    const uint64_t m = (1ull << 31) - C;
    int bad = 0;
    auto one = [&](uint32_t x) {
        if (mulmod_2p31m<A, C>(x) != static_cast<uint32_t>(static_cast<uint64_t>(A) * x % m)) ++bad;
        // the device's form of the reduction: the low word of p + H (C + 2^31) equals L + C H
        const uint64_t p = static_cast<uint64_t>(A) * x;
        const uint32_t H = static_cast<uint32_t>(p >> 31);
        const uint32_t dev = static_cast<uint32_t>(p + static_cast<uint64_t>(H) * (C + 0x80000000u));
        if (dev != (static_cast<uint32_t>(p) & 0x7fffffffu) + C * H) ++bad;
    };
    for (uint32_t x : {0u, 1u, 2u, 3u, static_cast<uint32_t>(m - 1), static_cast<uint32_t>(m - 2),
                       static_cast<uint32_t>(m / A), static_cast<uint32_t>(m / A + 1), 0x40000000u})
        one(x);
    // every x whose product's high part H = floor(A x / 2^31) changes (the carries into C H)
    for (uint64_t h = 1; h < A; ++h) {
        const uint64_t x0 = (h << 31) / A;
        for (uint64_t x = x0 > 2 ? x0 - 2 : 0; x <= x0 + 2 && x < m; ++x) one(static_cast<uint32_t>(x));
    }
    for (int t = 0; t < 1000000; ++t) one(static_cast<uint32_t>(rnd() % m));
    return bad;
}

int main() {
    int bad = 0;
    bad += check_component<13, 12, 31>(2000, 60);
    bad += check_component<2, 4, 29>(2000, 60);
    bad += check_component<3, 17, 28>(2000, 60);
    // the LCG's n-step map against n single steps, for every n up to 4096 and at random seeds
    for (int t = 0; t < 16; ++t) {
        const uint32_t x0 = rnd();
        uint32_t x = x0;
        for (uint64_t n = 0; n <= 4096; ++n) {
            if (lcg_skip(x0, n) != x) ++bad;
            x = lcg_next(x);
        }
    }
    // and composed: n = 2^40 + 12345 as 2^40 then 12345 steps
    {
        const uint32_t x0 = rnd();
        if (lcg_skip(lcg_skip(x0, 1ull << 40), 12345) != lcg_skip(x0, (1ull << 40) + 12345)) ++bad;
    }
    bad += check_mulmod<40014, 85>();
    bad += check_mulmod<40692, 249>();
    if (bad) {
        std::printf("FAILED: %d\n", bad);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
