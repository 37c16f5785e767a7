/*
 * rngld_oracle.c -- plain, slow CPU reference for the on-the-fly RNG + Langevin-dynamics path of
 * Zhmurov, Rybnikov, Kholodov & Barsegov, "Efficient pseudo-random number generators for
 * biomolecular simulations on graphics processors" (arXiv:1003.1123).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  The product library (paper_1003_1123_amd) never links, loads or
 * calls it, and the two share no source: every generator, transform and integrator below is
 * written out again from its definition.
 *
 * Rules followed here: sequential loops in the order the paper states them, integer generators
 * computed from their plain definitions (e.g. a*x mod m with a 64-bit product, not Schrage's
 * trick), every floating-point quantity in double precision with the C library's log, sqrt, cos
 * and sin.  No blocking, fusion or reordering.
 *
 * Parity status per function is recorded next to it ("pinned by" = which non-circular check in the
 * test-suite fixes it).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------------------------- */
/* Per-stream seeding.  The paper (Sec. III.B) only asks that per-thread seeds come from an
 * independent sequence or a different generator.  Reading taken: SplitMix64 (Steele, Lea & Flood,
 * OOPSLA 2014) in counter form; word i of stream j is the high half of
 * mix(seed + (4j + i + 1) * golden_gamma).
 * Pinned by: bijectivity of mix (explicit inverse) and avalanche statistics in the tests; the
 * exact constants have no printed vector to check against, so beyond that it is parity unpinned. */
static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64_mix(uint64_t z) { return sm64_mix(z); }

uint32_t orc_seed_word(uint64_t seed, uint64_t stream, uint32_t i)
{
    uint64_t counter = 4ULL * stream + (uint64_t)i + 1ULL;
    return (uint32_t)(sm64_mix(seed + counter * 0x9E3779B97F4A7C15ULL) >> 32);
}

/* ------------------------------------------------------------------------------------------- */
/* Linear congruential generator, Eq. (1) of Sec. II.B, with m = 2^32 ("Quick and Dirty").
 * Pinned by: Hull-Dobell full period 2^32 (brute force) and the jump-ahead closed form
 * x_n = a^n x_0 + c (a^n - 1)/(a - 1) mod 2^32 evaluated with exact integers in the tests. */
#define LCG_A 1664525u
#define LCG_C 1013904223u

uint32_t orc_lcg_next(uint32_t x) { return (uint32_t)((uint64_t)LCG_A * x + LCG_C); }

/* n steps of the LCG, one at a time. */
uint32_t orc_lcg_advance(uint32_t x, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) x = orc_lcg_next(x);
    return x;
}

/* Number of steps until the LCG returns to x0 (stops after limit steps, returning 0). */
uint64_t orc_lcg_period(uint32_t x0, uint64_t limit)
{
    uint32_t x = x0;
    for (uint64_t n = 1; n <= limit; ++n) {
        x = orc_lcg_next(x);
        if (x == x0) return n;
    }
    return 0;
}

/* One LCG per stream (Sec. II.B used as a per-thread generator, Sec. III).  Stream j's state is
 * one 32-bit word x; each draw returns the next x_n of Eq. (1).  Seeding reading:
 *   leap = 0: x = the stream's SplitMix64 seed word (independent offsets in the 2^32 cycle);
 *   leap > 0: x = the stream-0 seed word advanced j * leap steps, i.e. the streams are windows
 *             of one sequence that start leap values apart (the correlated seeding that the
 *             Fig. 4b discussion blames for the repeating pattern).
 * The advance is reduced modulo the full period 2^32, which the tests confirm by brute force. */
void orc_lcg_seed(uint64_t seed, uint64_t stream, uint64_t leap, uint32_t *state)
{
    if (leap == 0) {
        *state = orc_seed_word(seed, stream, 0);
        return;
    }
    uint64_t n = (stream * leap) & 0xFFFFFFFFULL;
    *state = orc_lcg_advance(orc_seed_word(seed, 0, 0), n);
}

/* ------------------------------------------------------------------------------------------- */
/* Tausworthe (taus88) component, Eq. (2) of Sec. II.D in L'Ecuyer's fast form, for a
 * characteristic trinomial x^k + x^q + 1 and step size s.  The component keeps its state in the
 * top k bits of the word; the low 32-k bits are masked away before the left shift.
 * Parameters (Appendix A, read as triples (q, k-s, s) with masks of width k = 31, 29, 28):
 *   (q, s, k) = (13, 12, 31), (2, 4, 29), (3, 17, 28).
 * Pinned by: the bit-level recurrence y_m = y_{m-k+q} xor y_{m-k} (Eq. 2) in the tests, and the
 * component periods 2^k - 1 (brute force). */
static const int TAUS_Q[3] = {13, 2, 3};
static const int TAUS_S[3] = {12, 4, 17};
static const int TAUS_K[3] = {31, 29, 28};

uint32_t orc_taus_component(uint32_t z, int which)
{
    int q = TAUS_Q[which], s = TAUS_S[which], k = TAUS_K[which];
    uint32_t keep_mask = (uint32_t)(0xFFFFFFFFu << (32 - k)); /* top k bits */
    uint32_t feedback = ((z << q) ^ z) >> (k - s);
    return ((z & keep_mask) << s) ^ feedback;
}

/* Brute-force period of one component from state z0 (0 if not found within limit). */
uint64_t orc_taus_component_period(uint32_t z0, int which, uint64_t limit)
{
    uint32_t z = orc_taus_component(z0, which); /* first post-step state */
    uint32_t first = z;
    for (uint64_t n = 1; n <= limit; ++n) {
        z = orc_taus_component(z, which);
        if (z == first) return n;
    }
    return 0;
}

/* Hybrid Taus state: three Tausworthe components and one LCG word (Alg. 1). */
typedef struct { uint32_t z[4]; } orc_taus_t;

/* Seeding reading: z_i = seed word i of the stream; a Tausworthe component whose k significant
 * bits are all zero is stuck at zero, so such a word is lifted by 2^(32-k). */
void orc_taus_lift(uint32_t *z)
{
    for (int c = 0; c < 3; ++c) {
        uint32_t floor_val = 1u << (32 - TAUS_K[c]);
        if (z[c] < floor_val) z[c] += floor_val;
    }
}

void orc_taus_seed(uint64_t seed, uint64_t stream, uint32_t *z)
{
    for (int i = 0; i < 4; ++i) z[i] = orc_seed_word(seed, stream, (uint32_t)i);
    orc_taus_lift(z);
}

/* First stream index >= start whose seed word i is below floor_val (search helper for tests that
 * must exercise the lift); returns UINT64_MAX if none below start + limit. */
uint64_t orc_find_small_seed_word(uint64_t seed, uint32_t i, uint32_t floor_val, uint64_t start, uint64_t limit)
{
    for (uint64_t j = start; j < start + limit; ++j)
        if (orc_seed_word(seed, j, i) < floor_val) return j;
    return UINT64_MAX;
}

/* One Hybrid Taus output: advance each of the three components and the LCG once, then combine
 * by exclusive-or (Sec. II.D; Alg. 1 updates before it outputs). */
uint32_t orc_taus_next(uint32_t *z)
{
    z[0] = orc_taus_component(z[0], 0);
    z[1] = orc_taus_component(z[1], 1);
    z[2] = orc_taus_component(z[2], 2);
    z[3] = orc_lcg_next(z[3]);
    return z[0] ^ z[1] ^ z[2] ^ z[3];
}

/* ------------------------------------------------------------------------------------------- */
/* Ran2 (Sec. II.C; Alg. 2): L'Ecuyer's two multiplicative LCGs combined through a Bays-Durham
 * shuffle table of NTAB = 32 entries.  Constants are the Numerical-Recipes values the paper
 * refers to.  The oracle evaluates a*x mod m with an exact 64-bit product (the plain definition);
 * the paper's Schrage decomposition is an implementation detail that must give the same bits.
 * State layout (35 int32): [0] idum, [1] idum2, [2] iy, [3..34] iv[0..31].
 * Pinned by: multiplicative order of a1 mod m1 and a2 mod m2 (primitive-root check against the
 * factorisations of m-1), and the shuffle's conservation invariant (every value placed in the
 * table is emitted exactly once) in the tests.  The table index rule itself has no closed form:
 * beyond the invariant it is parity unpinned. */
#define R2_M1 2147483563LL
#define R2_M2 2147483399LL
#define R2_A1 40014LL
#define R2_A2 40692LL
#define R2_NTAB 32
#define R2_IMM1 (R2_M1 - 1)
#define R2_NDIV (1 + R2_IMM1 / R2_NTAB)

int32_t orc_ran2_lcg1(int32_t x) { return (int32_t)((R2_A1 * (int64_t)x) % R2_M1); }
int32_t orc_ran2_lcg2(int32_t x) { return (int32_t)((R2_A2 * (int64_t)x) % R2_M2); }

/* Seeding reading: idum = 1 + (seed word 0 mod (m1 - 1)) so that idum lies in [1, m1-1];
 * then Alg. 2's initialisation: idum2 = idum, eight discarded steps of the first LCG followed by
 * 32 steps whose values fill iv[31] .. iv[0]; the first shuffle output register is iy = iv[0]. */
void orc_ran2_seed(uint64_t seed, uint64_t stream, int32_t *st)
{
    uint32_t w = orc_seed_word(seed, stream, 0);
    int32_t idum = (int32_t)(1 + (int64_t)(w % (uint32_t)(R2_M1 - 1)));
    int32_t *iv = st + 3;
    st[1] = idum;
    for (int j = R2_NTAB + 7; j >= 0; --j) {
        idum = orc_ran2_lcg1(idum);
        if (j < R2_NTAB) iv[j] = idum;
    }
    st[0] = idum;
    st[2] = iv[0];
}

/* One Ran2 output iy in [1, m1-1]. */
int32_t orc_ran2_next(int32_t *st)
{
    int32_t *iv = st + 3;
    st[0] = orc_ran2_lcg1(st[0]);
    st[1] = orc_ran2_lcg2(st[1]);
    int32_t j = (int32_t)(st[2] / R2_NDIV);
    int32_t iy = iv[j] - st[1];
    iv[j] = st[0];
    if (iy < 1) iy += (int32_t)R2_IMM1;
    st[2] = iy;
    return iy;
}

/* 32-bit word fed to the uniform mapping: (iy - 1) spans [0, m1-2] < 2^31, doubled. */
static uint32_t ran2_word(int32_t iy) { return (uint32_t)(iy - 1) << 1; }

/* ------------------------------------------------------------------------------------------- */
/* Additive lagged Fibonacci mod 2^32, Eq. (3) of Sec. II.E with f = addition:
 *   y_n = y_{n-ll} + y_{n-sl} mod 2^32  (reading of Alg. 3's short-lag index: lag sl, as in Eq. 3).
 * The generator state is the window of the last ll values, stored here in logical order
 * win[i] = y_{n-ll+i}.  Seeding reading: win[i] = i+1 LCG steps from the stream-0 seed word.
 * Pinned by: the period of the low b bits for small primitive trinomials (brute force) and the
 * primitivity checker below, in the tests. */
void orc_lf_seed(uint64_t seed, uint32_t ll, uint32_t *win)
{
    uint32_t x = orc_seed_word(seed, 0, 0);
    for (uint32_t i = 0; i < ll; ++i) {
        x = orc_lcg_next(x);
        win[i] = x;
    }
}

/* The window after a warm-up discard: seeded as above, then the first `discard` values of the
 * sequence generated from it (Eq. 3) and dropped, so that win[i] = y_{discard-ll+i}.
 * Pinned by: equality of the continued sequence with the undiscarded one shifted by `discard`,
 * and the recurrence across the window, in the tests. */
int orc_lf_generate(uint32_t ll, uint32_t sl, uint32_t *win, uint64_t count, uint32_t *out);

int orc_lf_seed_discard(uint64_t seed, uint32_t ll, uint32_t sl, uint64_t discard, uint32_t *win)
{
    orc_lf_seed(seed, ll, win);
    return orc_lf_generate(ll, sl, win, discard, NULL);
}

/* Generate count values of the sequence continuing from win; out may be NULL. */
int orc_lf_generate(uint32_t ll, uint32_t sl, uint32_t *win, uint64_t count, uint32_t *out)
{
    if (sl == 0 || sl >= ll) return -1;
    /* circular copy: buf[(head + i) % ll] = y_{n-ll+i} */
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ll);
    if (!buf) return -2;
    memcpy(buf, win, sizeof(uint32_t) * ll);
    uint64_t head = 0;
    for (uint64_t n = 0; n < count; ++n) {
        uint32_t y_ll = buf[head];                         /* y_{n-ll} */
        uint32_t y_sl = buf[(head + (ll - sl)) % ll];      /* y_{n-sl} */
        uint32_t y = y_ll + y_sl;
        if (out) out[n] = y;
        buf[head] = y;                                     /* y_n replaces y_{n-ll} */
        head = (head + 1) % ll;
    }
    for (uint32_t i = 0; i < ll; ++i) win[i] = buf[(head + i) % ll];
    free(buf);
    return 0;
}

/* Irreducibility of x^ll + x^sl + 1 over GF(2) for prime ll by Rabin's test:
 * irreducible  <=>  x^(2^ll) == x (mod P)  (P has no roots, since P(0) = P(1) = 1).
 * When 2^ll - 1 is a Mersenne prime, irreducible implies primitive (Sec. II.E asks for a
 * Mersenne-exponent ll and a primitive trinomial).  Polynomials are bit arrays (bit i = the
 * coefficient of x^i), 64 coefficients a word; ll squarings, each reduced mod P.
 * Pinned by: agreement with brute-force LFSR periods for every trinomial of small prime degree. */
/* dst ^= (src >> shift) restricted to coefficients below nbits_src - shift */
static void poly_xor_shr(uint64_t *dst, const uint64_t *src, size_t nw_src, uint64_t shift)
{
    size_t ws = (size_t)(shift >> 6);
    unsigned bs = (unsigned)(shift & 63);
    for (size_t w = 0; w + ws < nw_src; ++w) {
        uint64_t lo = src[w + ws] >> bs;
        uint64_t hi = (bs && w + ws + 1 < nw_src) ? (src[w + ws + 1] << (64 - bs)) : 0;
        dst[w] ^= lo | hi;
    }
}

/* dst ^= (src << shift), dst has nw_dst words */
static void poly_xor_shl(uint64_t *dst, size_t nw_dst, const uint64_t *src, size_t nw_src, uint64_t shift)
{
    size_t ws = (size_t)(shift >> 6);
    unsigned bs = (unsigned)(shift & 63);
    for (size_t w = 0; w < nw_src; ++w) {
        if (w + ws < nw_dst) dst[w + ws] ^= src[w] << bs;
        if (bs && w + ws + 1 < nw_dst) dst[w + ws + 1] ^= src[w] >> (64 - bs);
    }
}

/* spread the 32 bits of v to the even bit positions of a 64-bit word */
static uint64_t spread32(uint64_t v)
{
    v &= 0xFFFFFFFFULL;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFULL;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFULL;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0FULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

int orc_trinomial_irreducible(uint32_t ll, uint32_t sl)
{
    if (sl == 0 || sl >= ll) return -1;
    size_t nw = ((size_t)2 * ll + 63) / 64 + 2;  /* room for a square before reduction */
    size_t nlow = ((size_t)ll + 63) / 64;         /* words holding degrees < ll */
    uint64_t *a = (uint64_t *)calloc(nw, sizeof(uint64_t));
    uint64_t *high = (uint64_t *)calloc(nw, sizeof(uint64_t));
    if (!a || !high) { free(a); free(high); return -2; }
    a[0] = 2ULL; /* the polynomial x */
    for (uint32_t it = 0; it < ll; ++it) {
        /* square: coefficient i moves to 2i (cross terms vanish in characteristic 2) */
        for (size_t w = nlow; w-- > 0;) {
            uint64_t v = a[w];
            a[2 * w] = spread32(v);
            a[2 * w + 1] = spread32(v >> 32);
        }
        for (size_t w = 2 * nlow; w < nw; ++w) a[w] = 0;
        /* reduce: with H = a >> ll, a = (a mod x^ll) + H + H x^sl, until deg a < ll */
        for (int pass = 0;; ++pass) {
            if (pass > 64) { free(a); free(high); return -3; } /* degree must fall every pass */
            /* any coefficient of degree >= ll left? */
            int any = (a[ll >> 6] >> (ll & 63)) != 0;
            for (size_t w = (ll >> 6) + 1; w < nw && !any; ++w) any = (a[w] != 0);
            if (!any) break;
            memset(high, 0, nw * sizeof(uint64_t));
            poly_xor_shr(high, a, nw, ll);
            /* clear the coefficients of degree >= ll */
            a[ll >> 6] &= (ll & 63) ? ((1ULL << (ll & 63)) - 1ULL) : 0ULL;
            for (size_t w = (ll >> 6) + 1; w < nw; ++w) a[w] = 0;
            for (size_t w = 0; w < nw; ++w) a[w] ^= high[w];
            poly_xor_shl(a, nw, high, nw, sl);
        }
    }
    int is_x = (a[0] == 2ULL);
    for (size_t w = 1; w < nw && is_x; ++w) is_x = (a[w] == 0);
    free(a);
    free(high);
    return is_x;
}

/* Period of the one-bit LFSR y_n = y_{n-ll} xor y_{n-sl} from the state y_{-ll..-1} = 0..01
 * (brute force, small ll only; 0 if not found within limit). */
uint64_t orc_lfsr_period(uint32_t ll, uint32_t sl, uint64_t limit)
{
    if (ll > 62 || sl == 0 || sl >= ll) return 0;
    uint8_t *buf = (uint8_t *)calloc(ll, 1);
    uint8_t *first = (uint8_t *)calloc(ll, 1);
    if (!buf || !first) { free(buf); free(first); return 0; }
    buf[ll - 1] = 1;
    memcpy(first, buf, ll);
    uint64_t head = 0, found = 0;
    for (uint64_t n = 1; n <= limit; ++n) {
        uint8_t y = buf[head] ^ buf[(head + (ll - sl)) % ll];
        buf[head] = y;
        head = (head + 1) % ll;
        int same = 1;
        for (uint32_t i = 0; i < ll && same; ++i) same = (buf[(head + i) % ll] == first[i]);
        if (same) { found = n; break; }
    }
    free(buf);
    free(first);
    return found;
}

/* ------------------------------------------------------------------------------------------- */
/* Uniform mapping and Box-Muller transform (Sec. I; Table II: four uniforms give the three
 * Gaussian force components).  Reading: the top 24 bits of a word give u_open in (0, 1] and
 * u_half in [0, 1), both exact in single and double precision; r = sqrt(-2 ln u_open(w0)),
 * theta = 2 pi u_half(w1), (g0, g1) = (r cos theta, r sin theta).
 * Pinned by: g0^2 + g1^2 = -2 ln u, closed-form special angles and the N(0,1) moments, in the
 * tests. */
double orc_u_open(uint32_t w) { return (double)((w >> 8) + 1u) * (1.0 / 16777216.0); }
double orc_u_half(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

double orc_bm_radius(uint32_t w) { return sqrt(-2.0 * log(orc_u_open(w))); }

void orc_box_muller(uint32_t w0, uint32_t w1, double *g0, double *g1)
{
    double r = orc_bm_radius(w0);
    double theta = 2.0 * ORC_PI * orc_u_half(w1);
    *g0 = r * cos(theta);
    *g1 = r * sin(theta);
}

/* Box-Muller of n word pairs: out[2i], out[2i+1] from words[2i], words[2i+1]. */
void orc_box_muller_many(const uint32_t *words, uint64_t n_pairs, double *out)
{
    for (uint64_t i = 0; i < n_pairs; ++i) orc_box_muller(words[2 * i], words[2 * i + 1], &out[2 * i], &out[2 * i + 1]);
}

/* ------------------------------------------------------------------------------------------- */
/* Bulk streams.  kind: 0 = Hybrid Taus, 1 = Ran2, 3 = LCG (per-stream states), 2 = lagged
 * Fibonacci (one shared window).  Per-stream output layout out[t*S + j] = value t of stream j.
 * Ran2 streams yield iy itself as the integer output. */
enum { ORC_TAUS = 0, ORC_RAN2 = 1, ORC_LF = 2, ORC_LCG = 3 };

static uint32_t lcg_stream_next(uint32_t *x)
{
    *x = orc_lcg_next(*x);
    return *x;
}

static uint32_t next_word_stream(int kind, void *states, uint64_t j)
{
    if (kind == ORC_TAUS) return orc_taus_next((uint32_t *)states + 4 * j);
    if (kind == ORC_LCG) return lcg_stream_next((uint32_t *)states + j);
    return ran2_word(orc_ran2_next((int32_t *)states + 35 * j));
}

int orc_uniform_streams(int kind, void *states, uint64_t S, uint64_t per_stream, uint32_t *out)
{
    for (uint64_t j = 0; j < S; ++j)
        for (uint64_t t = 0; t < per_stream; ++t) {
            uint32_t v;
            if (kind == ORC_TAUS) v = orc_taus_next((uint32_t *)states + 4 * j);
            else if (kind == ORC_RAN2) v = (uint32_t)orc_ran2_next((int32_t *)states + 35 * j);
            else if (kind == ORC_LCG) v = lcg_stream_next((uint32_t *)states + j);
            else return -1;
            out[t * S + j] = v;
        }
    return 0;
}

/* Gaussian streams: values 2i and 2i+1 of a stream are the cosine and sine branches of the
 * Box-Muller pair built from that stream's uniforms 2i and 2i+1. */
int orc_gaussian_streams(int kind, void *states, uint64_t S, uint64_t per_stream, double *out)
{
    if (per_stream % 2) return -1;
    for (uint64_t j = 0; j < S; ++j)
        for (uint64_t t = 0; t < per_stream; t += 2) {
            uint32_t w0 = next_word_stream(kind, states, j);
            uint32_t w1 = next_word_stream(kind, states, j);
            double g0, g1;
            orc_box_muller(w0, w1, &g0, &g1);
            out[t * S + j] = g0;
            out[(t + 1) * S + j] = g1;
        }
    return 0;
}

int orc_lf_gaussian(uint32_t ll, uint32_t sl, uint32_t *win, uint64_t count, double *out)
{
    if (count % 2) return -1;
    uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (count ? count : 1));
    if (!w) return -2;
    int rc = orc_lf_generate(ll, sl, win, count, w);
    for (uint64_t i = 0; rc == 0 && i < count; i += 2) orc_box_muller(w[i], w[i + 1], &out[i], &out[i + 1]);
    free(w);
    return rc;
}

/* ------------------------------------------------------------------------------------------- */
/* Langevin dynamics of independent 3-D harmonic oscillators (force -k x per component).
 * scheme 0, underdamped: m dv/dt = -xi v - k x + G, <G G> = 2 kT xi delta (Sec. I, with the sign
 * of the friction term read as -xi v), integrated by the first-order semi-implicit
 * Euler-Maruyama step (reading; the paper gives no underdamped scheme):
 *     v' = (1 - gamma h) v - (k h / m) x + sqrt(2 gamma kT h / m) g,   x' = x + h v',
 *   with xi = m gamma, which is G = g sqrt(2 kT xi h) divided by m.
 * scheme 1, overdamped, Eq. (5) of Sec. IV with the random displacement read as
 *   sqrt(2 kT h / xi) g (the printed sqrt(2 kT xi h) is the random impulse, divided by xi):
 *     x' = x - (k h / xi) x + sqrt(2 kT h / xi) g ;  v is left untouched.
 * Per oscillator-step four uniforms w0..w3 are drawn; (g_x, g_y) = BoxMuller(w0, w1) and g_z is
 * the cosine branch of BoxMuller(w2, w3) (Table II caption: four numbers per three components).
 * Pinned by: the exact linear-Gaussian solution z_n = A^n z_0 + sum A^(n-1-i) B g_i and the
 * stationary moments of the scheme, in the tests. */
typedef struct { double c, kap, sig, h, odc, ods; int scheme; } orc_coef;

static orc_coef make_coef(double m, double k, double gamma, double kT, double dt, int scheme)
{
    orc_coef q;
    q.scheme = scheme;
    q.h = dt;
    q.c = 1.0 - gamma * dt;
    q.kap = k * dt / m;
    q.sig = sqrt(2.0 * gamma * kT * dt / m);
    double xi = m * gamma;
    q.odc = k * dt / xi;
    q.ods = sqrt(2.0 * kT * dt / xi);
    return q;
}

static void forces_from_words(const uint32_t w[4], double g[3])
{
    double unused;
    orc_box_muller(w[0], w[1], &g[0], &g[1]);
    orc_box_muller(w[2], w[3], &g[2], &unused);
}

static void ld_update(const orc_coef *q, double *x, double *v, const double g[3])
{
    for (int d = 0; d < 3; ++d) {
        if (q->scheme == 0) {
            v[d] = q->c * v[d] - q->kap * x[d] + q->sig * g[d];
            x[d] = x[d] + q->h * v[d];
        } else {
            x[d] = x[d] - q->odc * x[d] + q->ods * g[d];
        }
    }
}

/* Observables recorded after t steps for t = 0, stride, 2 stride, ... <= n_steps, each a mean
 * over the 3N coordinates: <x^2>, <v^2>, <x v>, <x>, <x(t) x(t0)>, <v(t) v(t0)> (the last two are
 * zero before t0). */
#define ORC_NOBS 6

static void record_obs(uint64_t N, const double *x, const double *v, const double *x0, const double *v0,
                       int have_t0, double *dst)
{
    double s[ORC_NOBS] = {0, 0, 0, 0, 0, 0};
    for (uint64_t i = 0; i < 3 * N; ++i) {
        s[0] += x[i] * x[i];
        s[1] += v[i] * v[i];
        s[2] += x[i] * v[i];
        s[3] += x[i];
        if (have_t0) {
            s[4] += x[i] * x0[i];
            s[5] += v[i] * v0[i];
        }
    }
    for (int q = 0; q < ORC_NOBS; ++q) dst[q] = (N > 0) ? s[q] / (double)(3 * N) : 0.0;
}

/*
 * Run n_steps for N oscillators.  x, v are [3][N] component-major.  Generator:
 *   per-stream kinds: states holds N states (oscillator i uses state i);
 *   LF: states is the window of ll values; oscillator i at step s consumes y_{P + 4i + r},
 *       r = 0..3, with P the sequence position at the start of the step (Alg. 3's thread offset).
 * obs (may be NULL, stride 0 = none): [n_points][6].
 */
int orc_ld_run(int kind, void *states, uint32_t ll, uint32_t sl, uint64_t N, uint32_t n_steps,
               double m, double k, double gamma, double kT, double dt, int scheme,
               double *x, double *v, uint32_t stride, uint32_t t0, double *obs)
{
    orc_coef q = make_coef(m, k, gamma, kT, dt, scheme);
    double *x0 = (double *)calloc(3 * N + 1, sizeof(double));
    double *v0 = (double *)calloc(3 * N + 1, sizeof(double));
    uint32_t *words = (uint32_t *)malloc(sizeof(uint32_t) * (4 * N + 1));
    if (!x0 || !v0 || !words) { free(x0); free(v0); free(words); return -2; }
    int rc = 0;
    for (uint32_t s = 0; s <= n_steps && rc == 0; ++s) {
        if (s == t0) {
            memcpy(x0, x, sizeof(double) * 3 * N);
            memcpy(v0, v, sizeof(double) * 3 * N);
        }
        if (obs && stride && s % stride == 0)
            record_obs(N, x, v, x0, v0, s >= t0, obs + (uint64_t)(s / stride) * ORC_NOBS);
        if (s == n_steps) break;
        /* draw the step's words */
        if (kind == ORC_LF) {
            rc = orc_lf_generate(ll, sl, (uint32_t *)states, 4 * N, words);
        } else {
            for (uint64_t i = 0; i < N; ++i)
                for (int r = 0; r < 4; ++r) words[4 * i + r] = next_word_stream(kind, states, i);
        }
        for (uint64_t i = 0; i < N; ++i) {
            double g[3], xi[3], vi[3];
            forces_from_words(words + 4 * i, g);
            for (int d = 0; d < 3; ++d) { xi[d] = x[d * N + i]; vi[d] = v[d * N + i]; }
            ld_update(&q, xi, vi, g);
            for (int d = 0; d < 3; ++d) { x[d * N + i] = xi[d]; v[d * N + i] = vi[d]; }
        }
    }
    free(x0);
    free(v0);
    free(words);
    return rc;
}

/*
 * The lagged-Fibonacci LD run of orc_ld_run restricted to a few oscillators: the one sequence is
 * generated in full, in order (Eq. 3), but only the words of the n_sample oscillators ids[]
 * (ascending, each < N) are kept, and only those oscillators are integrated.  Oscillator i at step
 * s consumes y_{P + 4i + r}, r = 0..3, P the position at the start of the step, as in orc_ld_run.
 * x, v are [3][n_sample]; win (the last ll values) advances by 4 N n_steps positions.  Lets a test
 * follow a few oscillators of a run whose full state would not fit the oracle's time.
 * Pinned by: equality with orc_ld_run on the same oscillators, in the tests.
 */
int orc_ld_run_lf_sampled(uint32_t ll, uint32_t sl, uint32_t *win, uint64_t N, uint32_t n_steps, double m,
                          double k, double gamma, double kT, double dt, int scheme, const uint64_t *ids,
                          uint64_t n_sample, double *x, double *v)
{
    if (sl == 0 || sl >= ll) return -1;
    for (uint64_t q = 0; q < n_sample; ++q)
        if (ids[q] >= N || (q > 0 && ids[q] <= ids[q - 1])) return -1;
    orc_coef co = make_coef(m, k, gamma, kT, dt, scheme);
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * ll);
    uint32_t *words = (uint32_t *)malloc(sizeof(uint32_t) * (4 * n_sample + 1));
    if (!buf || !words) { free(buf); free(words); return -2; }
    memcpy(buf, win, sizeof(uint32_t) * ll);
    /* buf[head] = y_{n-ll}; buf[tail] = y_{n-sl}, tail = head + ll - sl (mod ll) */
    uint32_t head = 0, tail = ll - sl;
    for (uint32_t s = 0; s < n_steps; ++s) {
        uint64_t q = 0;
        for (uint64_t i = 0; i < N; ++i) {
            int keep = q < n_sample && ids[q] == i;
            for (int r = 0; r < 4; ++r) {
                uint32_t y = buf[head] + buf[tail];
                buf[head] = y;
                if (++head == ll) head = 0;
                if (++tail == ll) tail = 0;
                if (keep) words[4 * q + r] = y;
            }
            if (keep) ++q;
        }
        for (q = 0; q < n_sample; ++q) {
            double g[3], xi[3], vi[3];
            forces_from_words(words + 4 * q, g);
            for (int d = 0; d < 3; ++d) { xi[d] = x[d * n_sample + q]; vi[d] = v[d * n_sample + q]; }
            ld_update(&co, xi, vi, g);
            for (int d = 0; d < 3; ++d) { x[d * n_sample + q] = xi[d]; v[d * n_sample + q] = vi[d]; }
        }
    }
    for (uint32_t i = 0; i < ll; ++i) win[i] = buf[(head + i) % ll];
    free(buf);
    free(words);
    return 0;
}

/* The Gaussian forces g[s][d][i] an LD run would use (for the exact-solution pin). */
int orc_ld_forces(int kind, void *states, uint32_t ll, uint32_t sl, uint64_t N, uint32_t n_steps, double *g)
{
    uint32_t *words = (uint32_t *)malloc(sizeof(uint32_t) * (4 * N + 1));
    if (!words) return -2;
    int rc = 0;
    for (uint32_t s = 0; s < n_steps && rc == 0; ++s) {
        if (kind == ORC_LF) {
            rc = orc_lf_generate(ll, sl, (uint32_t *)states, 4 * N, words);
        } else {
            for (uint64_t i = 0; i < N; ++i)
                for (int r = 0; r < 4; ++r) words[4 * i + r] = next_word_stream(kind, states, i);
        }
        for (uint64_t i = 0; i < N; ++i) {
            double gi[3];
            forces_from_words(words + 4 * i, gi);
            for (int d = 0; d < 3; ++d) g[((uint64_t)s * 3 + d) * N + i] = gi[d];
        }
    }
    free(words);
    return rc;
}

/* ------------------------------------------------------------------------------------------- */
/* Loss and its reverse-mode (adjoint) gradient for the underdamped scheme, per-stream kinds only.
 *   L = (1 / (t_end - t_begin + 1)) * sum_{t = t_begin}^{t_end} (1 / 3N) sum_{i,d} x_{t,i,d}^2,
 * where x_t is the position after t steps (1 <= t_begin <= t_end <= n_steps).
 * With mu = lam_v' + h lam_x' (adjoints of the step's outputs), one reverse step is
 *   lam_x = lam_x' - kap mu + dL/dx,   lam_v = c mu,
 *   dL/dtheta += mu (dc/dtheta v - dkap/dtheta x + dsig/dtheta g),
 * with dc/dgamma = -h, dkap/dk = h/m, dsig/dgamma = sig/(2 gamma), dsig/dkT = sig/(2 kT).
 * Each oscillator is independent, so it is run forward (storing its path and noise) and then
 * swept backward before moving to the next one.  grad = [dL/dk, dL/dgamma, dL/dkT].
 * Pinned by: central finite differences under common random numbers and the exact identity
 * dL/dkT = L/kT for x0 = v0 = 0, in the tests. */
/* The same with the step's coefficients given directly: cq = {c, kap, sig, h} and their partials
 * dq = {dkap/dk, dc/dgamma, dsig/dgamma, dsig/dkT} (e.g. a parameter block held at another
 * precision, whose rounded coefficients define the map actually iterated). */
int orc_ld_adjoint_coef(int kind, void *states, uint64_t N, uint32_t n_steps, const double *cq, const double *dq,
                        const double *x_init, const double *v_init, uint32_t t_begin, uint32_t t_end,
                        double *loss, double *grad)
{
    if (kind == ORC_LF || t_begin < 1 || t_end < t_begin || t_end > n_steps) return -1;
    orc_coef q;
    memset(&q, 0, sizeof(q));
    q.scheme = 0;
    q.c = cq[0];
    q.kap = cq[1];
    q.sig = cq[2];
    q.h = cq[3];
    double h = q.h;
    double dkap_dk = dq[0], dc_dgamma = dq[1];
    double dsig_dgamma = dq[2], dsig_dkT = dq[3];
    double scale = 1.0 / ((double)(t_end - t_begin + 1) * 3.0 * (double)N);
    /* path[s] = (x_s, v_s) for s = 0..n_steps; noise[s] = g used in step s -> s+1 */
    double *path = (double *)malloc(sizeof(double) * 6 * ((size_t)n_steps + 1));
    double *noise = (double *)malloc(sizeof(double) * 3 * ((size_t)n_steps + 1));
    if (!path || !noise) { free(path); free(noise); return -2; }
    double L = 0.0, gk = 0.0, gg = 0.0, gT = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        double x[3], v[3];
        for (int d = 0; d < 3; ++d) { x[d] = x_init[d * N + i]; v[d] = v_init[d * N + i]; }
        for (int d = 0; d < 3; ++d) { path[d] = x[d]; path[3 + d] = v[d]; }
        for (uint32_t s = 0; s < n_steps; ++s) {
            uint32_t w[4];
            for (int r = 0; r < 4; ++r) w[r] = next_word_stream(kind, states, i);
            double g[3];
            forces_from_words(w, g);
            for (int d = 0; d < 3; ++d) noise[3 * (size_t)s + d] = g[d];
            ld_update(&q, x, v, g);
            for (int d = 0; d < 3; ++d) {
                path[6 * ((size_t)s + 1) + d] = x[d];
                path[6 * ((size_t)s + 1) + 3 + d] = v[d];
            }
            if (s + 1 >= t_begin && s + 1 <= t_end)
                for (int d = 0; d < 3; ++d) L += scale * x[d] * x[d];
        }
        /* reverse sweep; lam holds the adjoints of (x_{s+1}, v_{s+1}) */
        double lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
        for (uint32_t s = n_steps; s-- > 0;) {
            /* direct dependence of L on x_{s+1} */
            if (s + 1 >= t_begin && s + 1 <= t_end)
                for (int d = 0; d < 3; ++d) lx[d] += 2.0 * scale * path[6 * ((size_t)s + 1) + d];
            for (int d = 0; d < 3; ++d) {
                double xs = path[6 * (size_t)s + d], vs = path[6 * (size_t)s + 3 + d];
                double g = noise[3 * (size_t)s + d];
                double mu = lv[d] + h * lx[d];
                gk += mu * (-dkap_dk * xs);
                gg += mu * (dc_dgamma * vs + dsig_dgamma * g);
                gT += mu * (dsig_dkT * g);
                lx[d] = lx[d] - q.kap * mu;
                lv[d] = q.c * mu;
            }
        }
    }
    free(path);
    free(noise);
    *loss = L;
    grad[0] = gk;
    grad[1] = gg;
    grad[2] = gT;
    return 0;
}

int orc_ld_adjoint(int kind, void *states, uint64_t N, uint32_t n_steps, double m, double k, double gamma,
                   double kT, double dt, const double *x_init, const double *v_init, uint32_t t_begin,
                   uint32_t t_end, double *loss, double *grad)
{
    orc_coef q = make_coef(m, k, gamma, kT, dt, 0);
    double cq[4] = {q.c, q.kap, q.sig, q.h};
    double dq[4] = {dt / m, -dt, q.sig / (2.0 * gamma), q.sig / (2.0 * kT)};
    return orc_ld_adjoint_coef(kind, states, N, n_steps, cq, dq, x_init, v_init, t_begin, t_end, loss, grad);
}

/* Loss only (forward), for finite differences under common random numbers. */
int orc_ld_loss(int kind, void *states, uint64_t N, uint32_t n_steps, double m, double k, double gamma,
                double kT, double dt, const double *x_init, const double *v_init, uint32_t t_begin,
                uint32_t t_end, double *loss)
{
    if (kind == ORC_LF || t_begin < 1 || t_end < t_begin || t_end > n_steps) return -1;
    orc_coef q = make_coef(m, k, gamma, kT, dt, 0);
    double scale = 1.0 / ((double)(t_end - t_begin + 1) * 3.0 * (double)N);
    double L = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        double x[3], v[3];
        for (int d = 0; d < 3; ++d) { x[d] = x_init[d * N + i]; v[d] = v_init[d * N + i]; }
        for (uint32_t s = 0; s < n_steps; ++s) {
            uint32_t w[4];
            for (int r = 0; r < 4; ++r) w[r] = next_word_stream(kind, states, i);
            double g[3];
            forces_from_words(w, g);
            ld_update(&q, x, v, g);
            if (s + 1 >= t_begin && s + 1 <= t_end)
                for (int d = 0; d < 3; ++d) L += scale * x[d] * x[d];
        }
    }
    *loss = L;
    return 0;
}
