"""Pins for the oracle's integer generators, seeding and Box-Muller transform.

Every test here checks the oracle against something other than itself: a closed form, a
brute-force property, a bit-level definition or a library routine.  No GPU is used.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _constants():
    out = {}
    for line in open(os.path.join(GOLDEN, "paper_constants.txt")):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        vals = []
        for p in parts[1:]:
            try:
                vals.append(float(p) if ("." in p or "e" in p) else int(p))
            except ValueError:
                break
        out[parts[0]] = vals
    return out


CONST = _constants()
M32 = 2**32


# ---------------------------------------------------------------------------------------------
# LCG, Eq. (1)

def test_lcg_constants_match_paper():
    a, c = CONST["lcg_a"][0], CONST["lcg_c"][0]
    for x in (0, 1, 12345, M32 - 1):
        assert orc.lcg_next(x) == (a * x + c) % M32


def test_lcg_jump_closed_form_exact_integers():
    """x_n = a^n x0 + c (a^n - 1)/(a - 1) mod 2^32, evaluated with Python's exact integers
    (the division is exact over the integers; it is not a modular inverse)."""
    a, c = CONST["lcg_a"][0], CONST["lcg_c"][0]
    for x0 in (0, 1, 0xDEADBEEF):
        for n in (0, 1, 2, 7, 1000, 123457, 1_000_003):
            an = a**n if n < 2000 else pow(a, n, M32 * (a - 1))
            geo = (an - 1) // (a - 1) if n < 2000 else ((pow(a, n, M32 * (a - 1)) - 1) // (a - 1))
            expect = (an * x0 + c * geo) % M32
            assert orc.lcg_advance(x0, n) == expect, (x0, n)


def test_lcg_hull_dobell_full_period():
    """c odd and a = 1 mod 4 give the full period 2^32 (brute force, a few seconds)."""
    a, c = CONST["lcg_a"][0], CONST["lcg_c"][0]
    assert c % 2 == 1 and a % 4 == 1
    assert orc.lcg_period(12345, M32 + 1) == M32


def _lcg_jump(x0, n):
    """Closed-form jump of Eq. (1) with exact integers: a^n x0 + c (a^n - 1)/(a - 1) mod 2^32."""
    a, c = CONST["lcg_a"][0], CONST["lcg_c"][0]
    mod = M32 * (a - 1)
    an = pow(a, n, mod)
    return (an * x0 + c * ((an - 1) // (a - 1))) % M32


def test_lcg_stream_seeding_independent_and_leaped():
    """Per-stream LCG states: leap 0 takes each stream's own seed word; leap L puts stream j at
    j*L steps past the stream-0 seed word (checked by the closed-form jump, also past 2^32)."""
    ids = np.array([0, 1, 2, 17, 2**20 - 1, 2**33 + 5], dtype=np.uint64)
    st0 = orc.seed_states("lcg", 77, ids)
    assert st0.shape == (len(ids), 1) and st0.dtype == np.uint32
    assert [int(v) for v in st0[:, 0]] == [orc.seed_word(77, int(j), 0) for j in ids]
    x0 = orc.seed_word(77, 0, 0)
    for leap in (1, 4, 1000):
        st = orc.seed_states("lcg", 77, ids[:5], leap=leap)
        assert [int(v) for v in st[:, 0]] == [_lcg_jump(x0, int(j) * leap) for j in ids[:5]]
    # the reduction of the advance by the period 2^32
    big = orc.seed_states("lcg", 77, [2**32 + 3], leap=1)
    assert int(big[0, 0]) == _lcg_jump(x0, 3)


def test_lcg_streams_follow_eq1_and_leaped_streams_are_shifted_windows():
    S, per, leap = 9, 40, 4
    st = orc.seed_states("lcg", 5, np.arange(S))
    first = st[:, 0].copy()
    out = orc.uniform_streams("lcg", st, per)
    for j in range(S):
        assert [int(v) for v in out[:, j]] == [_lcg_jump(int(first[j]), t + 1) for t in range(per)]
    assert np.array_equal(st[:, 0], out[-1])
    # leap 4: stream j+1 is stream j four values later -- the neighbour-shift that correlates
    # oscillators driven by such streams
    out = orc.uniform_streams("lcg", orc.seed_states("lcg", 5, np.arange(S), leap=leap), per)
    assert np.array_equal(out[:-leap, 1:], out[leap:, :-1])


# ---------------------------------------------------------------------------------------------
# Tausworthe components, Eq. (2): bit-level definition

TAUS_QSK = [(13, 12, 31), (2, 4, 29), (3, 17, 28)]  # (q, s, k) from the printed triples


def test_taus_printed_triples_are_consistent():
    """The printed triples (c1j, c2j, c3j) read in order satisfy c2j + c3j = mask width k."""
    for j, (q, s, k) in enumerate(TAUS_QSK):
        c1, c2, c3 = CONST["taus_c%d" % (j + 1)]
        mask = CONST["taus_mask%d" % (j + 1)][0]
        width = 32 - (bin(mask ^ (M32 - 1)).count("1"))
        assert (c1, c3) == (q, s)
        assert width == k and c2 + c3 == k
        # the fast-form conditions of Sec. II.D: 0 < 2q < k, 0 < s <= k - q
        assert 0 < 2 * q < k and 0 < s <= k - q


def _bits_msb_first(z, nbits):
    return [(z >> (31 - i)) & 1 for i in range(nbits)]


def _taus_by_bit_recurrence(z0, q, s, k, n_steps):
    """Eq. (2) with characteristic trinomial x^k + x^q + 1: y_m = y_{m-k+q} xor y_{m-k}.
    y_0..y_{k-1} are the top k bits of z0 (MSB first); after n steps the word is the block of
    32 bits y_{ns} .. y_{ns+31} (MSB first)."""
    need = n_steps * s + 32
    y = _bits_msb_first(z0, k)
    while len(y) < need:
        m = len(y)
        y.append(y[m - k + q] ^ y[m - k])
    words = []
    for n in range(1, n_steps + 1):
        blk = y[n * s:n * s + 32]
        words.append(int("".join(map(str, blk)), 2))
    return words


@pytest.mark.parametrize("which", [0, 1, 2])
def test_taus_component_matches_bitwise_definition(which):
    q, s, k = TAUS_QSK[which]
    rng = np.random.default_rng(2024 + which)
    for z0 in rng.integers(0, M32, size=40, dtype=np.uint64):
        z0 = int(z0)
        ref = _taus_by_bit_recurrence(z0, q, s, k, 30)
        z = z0
        for n in range(30):
            z = orc.taus_component(z, which)
            assert z == ref[n], (which, z0, n)


@pytest.mark.parametrize("which,k", [(0, 31), (1, 29), (2, 28)])
def test_taus_component_period_is_2k_minus_1(which, k):
    """Maximal period 2^k - 1 (brute force).  The paper's text gives 2^30 - 1 for the second
    component; its 29-bit mask makes it 2^29 - 1."""
    assert orc.taus_component_period(0x9E3779B9, which, 2**k) == 2**k - 1


def test_taus_degenerate_seeds_and_lift():
    # a component whose k significant bits are zero stays at zero
    assert orc.taus_component(1, 0) == 0 and orc.taus_component(7, 1) == 0 and orc.taus_component(15, 2) == 0
    # seeding never produces such a component
    st = orc.taus_seed(99, np.arange(20000))
    assert (st[:, 0] >= 2).all() and (st[:, 1] >= 8).all() and (st[:, 2] >= 16).all()


def test_taus_lift_values():
    """A word whose k significant bits are zero is lifted by 2^(32-k); the LCG word is untouched."""
    assert list(orc.taus_lift([0, 0, 0, 0])) == [2, 8, 16, 0]
    assert list(orc.taus_lift([1, 7, 15, 1])) == [3, 15, 31, 1]
    assert list(orc.taus_lift([2, 8, 16, 5])) == [2, 8, 16, 5]


def _lift_streams():
    rows = []
    for line in open(os.path.join(GOLDEN, "taus_lift_streams.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append(tuple(int(v) for v in line.split()))
    return rows


def test_taus_lift_streams_fixture():
    for seed, comp, stream, raw in _lift_streams():
        assert orc.seed_word(seed, stream, comp) == raw < (1 << (32 - (31, 29, 28)[comp]))
        z = orc.taus_seed(seed, [stream])[0]
        assert z[comp] == raw + (1 << (32 - (31, 29, 28)[comp]))


def test_hybrid_taus_is_xor_of_independent_components():
    z = orc.taus_seed(1234, [5])[0].copy()
    comps = [int(z[0]), int(z[1]), int(z[2])]
    lcg = int(z[3])
    st = z.copy().reshape(1, 4)
    out = orc.uniform_streams("taus", st, 200)[:, 0]
    for n in range(200):
        comps = [orc.taus_component(comps[i], i) for i in range(3)]
        lcg = orc.lcg_next(lcg)
        assert int(out[n]) == comps[0] ^ comps[1] ^ comps[2] ^ lcg


def test_hybrid_taus_uniformity():
    st = orc.taus_seed(1234, np.arange(256))
    w = orc.uniform_streams("taus", st, 4096).ravel()
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-4
    bits = np.unpackbits(w.view(np.uint8)).reshape(-1, 32).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.005)


# ---------------------------------------------------------------------------------------------
# Seeding: SplitMix64 (the paper leaves the seed source open)

def _unxorshift(y, s):
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x & (2**64 - 1)


def _splitmix_inverse(z):
    z = _unxorshift(z, 31)
    z = (z * pow(0x94D049BB133111EB, -1, 2**64)) % 2**64
    z = _unxorshift(z, 27)
    z = (z * pow(0xBF58476D1CE4E5B9, -1, 2**64)) % 2**64
    return _unxorshift(z, 30)


def test_splitmix_mix_is_a_bijection():
    rng = np.random.default_rng(5)
    for z in rng.integers(0, 2**63, size=200, dtype=np.uint64):
        z = int(z) * 2 + 1
        assert _splitmix_inverse(orc.splitmix64_mix(z)) == z % 2**64


def test_seed_words_avalanche():
    flips = []
    for j in range(500):
        a = orc.seed_word(1234, j, 0)
        b = orc.seed_word(1235, j, 0)
        flips.append(bin(a ^ b).count("1"))
    assert abs(np.mean(flips) - 16.0) < 0.6


# ---------------------------------------------------------------------------------------------
# Ran2, Sec. II.C / Alg. 2 with the Numerical-Recipes constants

R2 = dict(m1=2147483563, m2=2147483399, a1=40014, a2=40692)
R2_FACTORS = {2147483563 - 1: [2, 3, 7, 631, 81031], 2147483399 - 1: [2, 19, 31, 1019, 1789]}


def _is_prime(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def test_ran2_component_lcgs_have_full_period():
    """Both moduli are prime and both multipliers are primitive roots, so each LCG has period
    m - 1, and the combined period lcm(m1-1, m2-1) exceeds 2e18 (Sec. II.B)."""
    for m, a in ((R2["m1"], R2["a1"]), (R2["m2"], R2["a2"])):
        assert _is_prime(m)
        fs = R2_FACTORS[m - 1]
        assert math.prod(fs) == m - 1 and all(_is_prime(p) for p in fs)
        for p in fs:
            assert pow(a, (m - 1) // p, m) != 1
    assert math.lcm(R2["m1"] - 1, R2["m2"] - 1) > 2e18


def test_ran2_lcgs_are_multiplications_mod_m():
    x1 = x2 = 987654321
    for n in range(1, 2001):
        x1 = orc.ran2_lcg1(x1)
        x2 = orc.ran2_lcg2(x2)
        if n in (1, 2, 10, 1000, 2000):
            assert x1 == pow(R2["a1"], n, R2["m1"]) * 987654321 % R2["m1"]
            assert x2 == pow(R2["a2"], n, R2["m2"]) * 987654321 % R2["m2"]


def test_ran2_shuffle_conserves_values_and_tracks_both_lcgs():
    """Bays-Durham conservation: every LCG1 value placed in the table leaves it exactly once, as
    output + idum2 (mod the wrap by m1 - 1), and idum2 follows the second LCG's orbit."""
    m1, m2, a1, a2 = R2["m1"], R2["m2"], R2["a1"], R2["a2"]
    imm1 = m1 - 1
    st = orc.ran2_seed(777, [3])
    st0 = st[0].copy()
    table0 = sorted(int(v) for v in st0[3:])
    idum0, idum2_0 = int(st0[0]), int(st0[1])
    M = 5000
    read_values, inserted = [], []
    for n in range(1, M + 1):
        iy = int(orc.lib().orc_ran2_next(orc._p(st[0])))
        idum, idum2 = int(st[0][0]), int(st[0][1])
        assert idum == pow(a1, n, m1) * idum0 % m1
        assert idum2 == pow(a2, n, m2) * idum2_0 % m2
        assert 1 <= iy <= imm1
        r = iy + idum2
        if r > m1 - 1:
            r -= imm1
        read_values.append(r)
        inserted.append(idum)
    final = [int(v) for v in st[0][3:]]
    assert sorted(read_values + final) == sorted(table0 + inserted)


def test_ran2_output_range_boundary():
    """Crafted state where the table entry equals the new idum2: the difference is 0, which lies
    outside the output range [1, m1-1] and wraps to m1 - 1 (Alg. 2: iy < 1 -> iy + IMM1)."""
    m1, m2, a2 = R2["m1"], R2["m2"], R2["a2"]
    ndiv = 1 + (m1 - 1) // 32
    st = orc.ran2_seed(5, [0])
    idum2 = 123456
    j = 5
    st[0][1] = idum2
    st[0][2] = j * ndiv + 17                     # selects table slot j
    st[0][3 + j] = a2 * idum2 % m2               # = idum2 after the step
    iy = int(orc.lib().orc_ran2_next(orc._p(st[0])))
    assert iy == m1 - 1


def test_ran2_seeding_follows_alg2_initialisation():
    m1, a1 = R2["m1"], R2["a1"]
    for stream in (0, 1, 2**20 - 1):
        st = orc.ran2_seed(1234, [stream])[0]
        w = orc.seed_word(1234, stream, 0)
        idum_seed = 1 + w % (m1 - 1)
        assert st[1] == idum_seed                      # idum2 = seed
        for j in range(32):                            # iv[j] = LCG1^(40 - j)(seed)
            assert st[3 + j] == pow(a1, 40 - j, m1) * idum_seed % m1
        assert st[0] == st[3] and st[2] == st[3]       # idum = last value, iy = iv[0]


# ---------------------------------------------------------------------------------------------
# Additive lagged Fibonacci, Eq. (3), Table I

def _table1():
    rows = []
    for line in open(os.path.join(GOLDEN, "table1_lf_lags.txt")):
        if line.startswith("#") or not line.strip():
            continue
        nb, sl, ll = map(int, line.split())
        rows.append((nb, sl, ll))
    return rows


def _primitivity_fixture():
    out = {}
    for line in open(os.path.join(GOLDEN, "lf_primitivity.txt")):
        if line.startswith("#") or not line.strip():
            continue
        ll, sl, flag = line.split()
        out[(int(ll), int(sl))] = flag == "primitive"
    return out


@pytest.mark.parametrize("ll", [2, 3, 5, 7, 13, 17, 19])
def test_trinomial_checker_matches_brute_force_lfsr_period(ll):
    """For a Mersenne-prime degree, x^ll + x^sl + 1 is irreducible iff the one-bit LFSR it drives
    has the maximal period 2^ll - 1 (brute force over every sl)."""
    for sl in range(1, ll):
        maximal = orc.lfsr_period(ll, sl, 2**ll) == 2**ll - 1
        assert orc.trinomial_irreducible(ll, sl) == maximal, (ll, sl)


def test_table1_small_rows_primitive_and_typo_row():
    for nb, sl, ll in _table1():
        if ll > 44497:
            continue
        if (ll, sl) == (23209, 12470):
            assert not orc.trinomial_irreducible(ll, sl)
            assert orc.trinomial_irreducible(ll, 13470)
        else:
            assert orc.trinomial_irreducible(ll, sl), (ll, sl)
        # sl ~ 0.618 ll is recommended (Sec. II.E); every row is a reciprocal-pair member
        assert 0.25 < sl / ll < 0.75 or (ll, sl) == (859433, 288477)


def test_table1_large_rows_from_fixture():
    """Large rows are checked by tests/golden/make_lf_primitivity.py (oracle only, minutes)."""
    if not os.path.exists(os.path.join(GOLDEN, "lf_primitivity.txt")):
        pytest.skip("fixture not yet written by tests/golden/make_lf_primitivity.py")
    fx = _primitivity_fixture()
    for nb, sl, ll in _table1():
        if (ll, sl) == (23209, 12470):
            assert fx[(ll, sl)] is False
            continue
        assert fx[(ll, sl)] is True, (ll, sl)
    assert fx[(23209, 13470)] is True


@pytest.mark.slow
def test_table1_large_rows_recomputed():
    fx = _primitivity_fixture()
    for (ll, sl), prim in fx.items():
        assert orc.trinomial_irreducible(ll, sl) == prim


def test_lf_output_satisfies_recurrence():
    ll, sl = 2281, 1252
    win = orc.lf_seed(1234, ll)
    hist = win.astype(np.uint64).copy()
    out = orc.lf_generate(ll, sl, win, 20000).astype(np.uint64)
    y = np.concatenate([hist, out])              # y[ll + n] = y_n
    n = np.arange(ll, len(y))
    assert np.array_equal(y[n], (y[n - ll] + y[n - sl]) % M32)
    # the window now holds the last ll values
    assert np.array_equal(win.astype(np.uint64), y[-ll:])


@pytest.mark.parametrize("discard", [1, 1251, 1252, 2281, 22810, 100_003])
def test_lf_discard_shifts_the_sequence(discard):
    """Seeding with a discard D gives the sequence from position D on: its window is y_{D-ll..D-1}
    of the undiscarded sequence (which satisfies Eq. 3 across the seeded window), and what it
    generates next is y_{D}, y_{D+1}, ..."""
    ll, sl = 2281, 1252
    win0 = orc.lf_seed(77, ll)
    hist = win0.astype(np.uint64).copy()
    y = np.concatenate([hist, orc.lf_generate(ll, sl, win0, discard + 5000).astype(np.uint64)])
    n = np.arange(ll, len(y))
    assert np.array_equal(y[n], (y[n - ll] + y[n - sl]) % M32)
    wd = orc.lf_seed(77, ll, sl, discard)
    assert np.array_equal(wd.astype(np.uint64), y[discard:discard + ll])  # y[ll + m] = y_m
    assert np.array_equal(orc.lf_generate(ll, sl, wd, 5000).astype(np.uint64), y[ll + discard:])


def test_lf_seed_is_lcg_orbit_of_the_seed_word():
    a, c = CONST["lcg_a"][0], CONST["lcg_c"][0]
    win = orc.lf_seed(1234, 5000)
    x0 = orc.seed_word(1234, 0, 0)
    for i in (0, 1, 2, 4999):
        n = i + 1
        expect = (pow(a, n, M32 * (a - 1)) * x0 + c * ((pow(a, n, M32 * (a - 1)) - 1) // (a - 1))) % M32
        assert int(win[i]) == expect


@pytest.mark.parametrize("ll,sl,bits", [(7, 3, 1), (7, 3, 3), (5, 2, 4), (17, 5, 1)])
def test_lf_low_bit_periods(ll, sl, bits):
    """With a primitive trinomial and an odd value in the seed window, the low b bits of the
    additive generator have period (2^ll - 1) 2^(b-1) (Brent)."""
    assert orc.trinomial_irreducible(ll, sl)
    win = orc.lf_seed(99, ll)
    assert (win & 1).any()
    expect = (2**ll - 1) * 2 ** (bits - 1)
    seq = orc.lf_generate(ll, sl, win, 3 * expect + ll) & np.uint32(2**bits - 1)
    first = seq[:ll]
    period = None
    for p in range(1, 2 * expect + 1):
        if np.array_equal(seq[p:p + ll], first):
            period = p
            break
    assert period == expect


# ---------------------------------------------------------------------------------------------
# Uniform mapping and Box-Muller

def test_uniform_mapping_edges():
    assert orc.u_open(0) == 2.0**-24 and orc.u_open(M32 - 1) == 1.0
    assert orc.u_half(0) == 0.0 and orc.u_half(M32 - 1) == 1.0 - 2.0**-24
    assert orc.bm_radius(M32 - 1) == 0.0
    assert abs(orc.bm_radius(0) - math.sqrt(48.0 * math.log(2.0))) < 1e-14


def test_box_muller_identity_and_special_angles():
    rng = np.random.default_rng(11)
    for w0, w1 in rng.integers(0, M32, size=(500, 2), dtype=np.uint64):
        g0, g1 = orc.box_muller(int(w0), int(w1))
        u = ((int(w0) >> 8) + 1) / 2.0**24
        assert abs(g0 * g0 + g1 * g1 - (-2.0 * math.log(u))) < 1e-12
    r = orc.bm_radius(0x12345678)
    quarter = 1 << 30  # u_half = 1/4
    for w1, (c, s) in ((0, (1, 0)), (quarter, (0, 1)), (2 * quarter, (-1, 0)), (3 * quarter, (0, -1))):
        g0, g1 = orc.box_muller(0x12345678, w1)
        assert abs(g0 - c * r) < 1e-14 and abs(g1 - s * r) < 1e-14


def test_box_muller_gaussian_moments_and_ks():
    st = orc.taus_seed(4321, np.arange(128))
    g = orc.gaussian_streams("taus", st, 8192).ravel()
    n = g.size
    assert abs(g.mean()) < 5 / math.sqrt(n)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(stats.kurtosis(g, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / n)
    assert stats.kstest(g, "norm").pvalue > 1e-4


def test_gaussian_stream_pairs_come_from_uniform_pairs():
    st_u = orc.taus_seed(1, np.arange(4))
    st_g = st_u.copy()
    w = orc.uniform_streams("taus", st_u, 10)
    g = orc.gaussian_streams("taus", st_g, 10)
    for j in range(4):
        for i in range(0, 10, 2):
            g0, g1 = orc.box_muller(int(w[i, j]), int(w[i + 1, j]))
            assert g[i, j] == g0 and g[i + 1, j] == g1
