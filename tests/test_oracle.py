"""Pins for the CPU oracle: facts the paper and the mathematics fix.

Every check here is independent of the oracle function it pins: exact
rationals from the EGFs, Glaisher's binomial congruence brute-forced, the
paper's printed residues and prime lists, exact interval costs, textbook
prime counts, and agreement between independently derived congruences.
"""
import functools
import random
from fractions import Fraction
from math import comb

import pytest

import oracle
from oracle import congruences as C
from oracle import exact
from conftest import read_golden


def small_primes(lo, hi):
    """Primes in [lo, hi) by trial division (independent of the oracle's sieve)."""
    out = []
    for n in range(max(lo, 2), hi):
        if all(n % d for d in range(2, int(n ** 0.5) + 1)):
            out.append(n)
    return out


PRIMES_5_2000 = small_primes(5, 2000)


@functools.lru_cache(maxsize=None)
def b_rec(p):
    return oracle.bernoulli_rec(p)


@functools.lru_cache(maxsize=None)
def e_rec(p):
    return oracle.euler_rec(p)


def want_rec(kind, p):
    return b_rec(p) if kind == "B" else e_rec(p)

# ---------------------------------------------------------------------------
# Section 1: Bernoulli and Euler numbers
# ---------------------------------------------------------------------------


def test_bernoulli_egf_matches_recurrence_and_textbook():
    egf = exact.bernoulli_egf(40)
    rec = exact.bernoulli_recurrence(40)
    assert egf == rec
    # textbook values of z/(e^z-1)
    assert egf[1] == Fraction(-1, 2)
    assert egf[2] == Fraction(1, 6)
    assert egf[4] == Fraction(-1, 30)
    assert egf[12] == Fraction(-691, 2730)
    assert all(egf[k] == 0 for k in range(3, 41, 2))


def test_euler_egf_secant_convention():
    egf = exact.euler_egf(30)
    rec = exact.euler_recurrence(30)
    assert [int(x) for x in egf] == rec
    # sec z = 1 + z^2/2! + 5 z^4/4! + 61 z^6/6! + 1385 z^8/8! + ... (all positive)
    assert rec[:9] == [1, 0, 1, 0, 5, 0, 61, 0, 1385]
    assert all(rec[k] == 0 for k in range(1, 31, 2))


def test_recurrence_mod_p_matches_exact_rationals():
    ps = small_primes(5, 260)
    B = exact.bernoulli_recurrence(ps[-1] - 3)
    E = exact.euler_recurrence(ps[-1] - 3)
    for p in ps:
        assert oracle.bernoulli_rec(p) == exact.rational_mod_p(B[p - 3], p), p
        assert oracle.euler_rec(p) == E[p - 3] % p, p


@pytest.mark.parametrize("h", [2, 3, 5])
def test_glaisher_binomial_bruteforce(h):
    """eqnGlaisher: binom(hp-1, p-1) == 1 - h(h-1)/3 p^3 B_{p-3} (mod p^4)."""
    for p in small_primes(5, 400):
        if h % p == 0 or (h - 1) % p == 0:
            continue
        assert exact.glaisher_b_mod_p(p, h) == b_rec(p), (p, h)


def test_wolstenholme_invariants_and_harmonic_form():
    """Section 1, first display: sum k^-2 == 0 (p), sum k^-1 == 0 (p^2), binom == 1 (p^3);
    and sum k^-2 == (2/3) p B_{p-3} (p^2), which gives eqnWolst's criterion."""
    for p in small_primes(5, 700) + small_primes(1400, 1500):
        H2 = oracle.harmonic2_mod_p2(p)
        assert H2 % p == 0
        assert oracle.harmonic1_mod_p2(p) == 0
        assert (comb(2 * p - 1, p - 1) - 1) % p ** 3 == 0
        assert oracle.b_from_harmonic(p) == b_rec(p), p
    # the first Wolstenholme prime: sum k^-2 == 0 mod p^2 (eqnWolst)
    assert oracle.harmonic2_mod_p2(16843) == 0


# ---------------------------------------------------------------------------
# Section 2: the sums S_l(x, y)
# ---------------------------------------------------------------------------


def test_interval_endpoints_bruteforce():
    """lo/hi of x*p < s < y*p against exact rational comparison: every s for
    tiny p, and the defining neighbourhood (lo-1 <= xp < lo, hi < yp <= hi+1)
    for larger p."""
    fracs = set()
    for cong in list(C.ALL_TABLES.values()) + list(C.ROOT_FORMS.values()):
        for _, x, y in cong.terms:
            fracs.add(x)
            fracs.add(y)
    fracs |= {Fraction(1, 2), Fraction(1, 3), Fraction(0)}
    fr = sorted(fracs)
    pairs = [(x, y) for x in fr for y in fr if x < y]
    for p in [5, 7, 11, 13, 97]:
        for x, y in pairs:
            lo, hi = oracle.interval(p, x, y)
            inside = [s for s in range(0, p + 1) if x * p < s < y * p]
            if inside:
                assert (lo, hi) == (inside[0], inside[-1]), (p, x, y)
            else:
                assert lo > hi
    for p in [1009, 2161, 6481, 10007, 999999937, 99999999977]:
        for x, y in pairs[::7]:
            lo, hi = oracle.interval(p, x, y)
            assert lo - 1 <= x * p < lo, (p, x)
            assert hi < y * p <= hi + 1, (p, y)
    # an integer endpoint is excluded (open interval): p=12 is not prime, but
    # the formula is the same; x=1/4 * 12 = 3, y = 1/2 * 12 = 6 -> s in {4, 5}
    assert oracle.interval(12, Fraction(1, 4), Fraction(1, 2)) == (4, 5)


def test_sum_direct_equals_polynomial_method():
    """eqnComputeS (c1/c0 of prod(z + s^l)) equals the sum of inverses."""
    rng = random.Random(7)
    for p in [11, 101, 10007, 1000003, 998244353]:
        for _ in range(6):
            a = rng.randrange(1, p)
            b = min(p - 1, a + rng.randrange(0, 3000))
            for ell in (2, 3):
                for alt in (False, True):
                    d = oracle.sum_direct(p, a, b, ell, alt)
                    c0, c1 = oracle.sum_poly_pair(p, a, b, ell, alt)
                    assert c1 * pow(c0, -1, p) % p == d
                    assert oracle.sum_poly(p, a, b, ell, alt, nthreads=4) == d


def test_sum_poly_pair_definition_tiny():
    """c0 = prod s^3, c1 = sum_s prod_{s' != s} s'^3, written out."""
    p = 101
    lo, hi = 7, 19
    c0, c1 = oracle.sum_poly_pair(p, lo, hi, 3, False)
    us = [pow(s, 3, p) for s in range(lo, hi + 1)]
    e0 = 1
    for u in us:
        e0 = e0 * u % p
    e1 = 0
    for i in range(len(us)):
        t = 1
        for j, u in enumerate(us):
            if j != i:
                t = t * u % p
        e1 = (e1 + t) % p
    assert (c0, c1) == (e0, e1)


# ---------------------------------------------------------------------------
# Sections 2-5: the congruences
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("name", sorted(C.ALL_TABLES) + sorted(C.ROOT_FORMS))
def test_printed_cost(name):
    cong = C.table(name)
    assert cong.exact_cost() == cong.cost
    # intervals lie in [0, 1/2] or [0, 1], disjoint and ordered
    prev = Fraction(-1)
    for _, x, y in cong.terms:
        assert 0 <= x < y <= 1
        assert x >= prev
        prev = y


def test_tanner_wagstaff_family_costs():
    for b in range(2, 14):
        t = C.tanner_wagstaff(b)
        assert t.exact_cost() == t.cost


@pytest.mark.parametrize("name", sorted(C.ALL_TABLES))
def test_table_matches_recurrence_small_p(name):
    """Each specialised table reproduces B_{p-3} / E_{p-3} mod p for 11 <= p < 2000."""
    cong = C.table(name)
    ps = [p for p in PRIMES_5_2000 if p >= 11]
    got = oracle.congruence_residues(ps, cong)
    for p, r in zip(ps, got):
        assert r == want_rec(cong.kind, p), (name, p)


@pytest.mark.parametrize("name", ["SV", "V12", "Vandiver", "V10", "E1", "MacE"])
def test_root_forms_match_recurrence(name):
    cong = C.table(name)
    ps = [p for p in PRIMES_5_2000 if p >= cong.min_p]
    got = oracle.congruence_residues(ps, cong)
    for p, r in zip(ps, got):
        if cong.lhs % p == 0:
            assert r is None       # left side vanishes: not usable at this p
        else:
            assert r == want_rec(cong.kind, p), (name, p)


def test_tanner_wagstaff_family_matches_recurrence():
    for b in range(2, 14):
        t = C.tanner_wagstaff(b)
        ps = [p for p in PRIMES_5_2000 if p > b + 1 and p >= 11][:60]
        for p, r in zip(ps, oracle.congruence_residues(ps, t)):
            if t.lhs % p == 0:
                assert r is None        # C_k(2,b,b+1) vanishes mod p
            else:
                assert r == b_rec(p), (b, p)


def test_e1_sign_reading():
    """eqnE1 as printed carries (-1)^((p-1)/2-k); at k=1 that is -1 for p == 1 mod 4
    and +1 for p == 3 mod 4, while eqnE3 and eqnEE3 (derived from it) carry (-1)^k,
    i.e. -1 always.  The oracle reads the sign as (-1)^k: the printed factor
    disagrees with the recurrence at every p == 3 mod 4 here, (-1)^k at none."""
    for p in PRIMES_5_2000[:120]:
        S = oracle.sum_direct(p, 1, (p - 1) // 4, 2)
        e = e_rec(p)
        printed = (-1) ** (((p - 1) // 2 - 1) % 2)
        lhs_k = (-4 * e) % p           # (-1)^1 4^1 E
        lhs_printed = (printed * 4 * e) % p
        assert lhs_k == S
        if p % 4 == 3 and e != 0:
            assert lhs_printed != S
        if p % 4 == 1:
            assert lhs_printed == S


def test_tables_agree_beyond_recurrence_range():
    """All B tables and all E tables give one residue each on primes far above
    the recurrence range (independent intervals and coefficients)."""
    rng = random.Random(11)
    ps = oracle.primes(10 ** 6, 10 ** 6 + 20000)
    ps = rng.sample(ps, 12) + [16843, 2124679]
    for kind, names in (("B", sorted(C.TABLES_B) + ["SV", "V12", "Vandiver", "V10"]),
                        ("E", sorted(C.TABLES_E) + ["E1", "MacE"])):
        cols = [oracle.congruence_residues(ps, C.table(n)) for n in names]
        for i, p in enumerate(ps):
            vals = {col[i] for col in cols}
            assert len(vals) == 1, (kind, p, dict(zip(names, [c[i] for c in cols])))
    # and the harmonic form of eqnWolst on the B side
    for p in ps[:4]:
        assert oracle.b_from_harmonic(p) == oracle.congruence_residue(p, C.SV)


def test_planted_coefficient_mistakes_are_caught():
    """Flip the sign of, or perturb, one coefficient or endpoint of eqnBB30 / eqnEE33
    (a copy, on the CPU): the agreement check above must notice every mutation."""
    ps = [p for p in PRIMES_5_2000 if p >= 600][:25] + oracle.primes(10 ** 5, 10 ** 5 + 400)
    for base in (C.BB30, C.EE33):
        want = oracle.congruence_residues(ps, base)
        for i in range(len(base.terms)):
            c, x, y = base.terms[i]
            muts = [(-c, x, y), (c + 1, x, y), (c, x, y + Fraction(1, 2 * y.denominator))]
            for m in muts:
                terms = list(base.terms)
                terms[i] = m
                bad = C.Congruence("mut", base.kind, base.ell, base.lhs, terms, 0, "")
                got = oracle.congruence_residues(ps, bad)
                assert got != want, (base.name, i, m)


# ---------------------------------------------------------------------------
# Printed facts: Theorem 1.1, Tables 2 and 3
# ---------------------------------------------------------------------------


def test_known_wolstenholme_and_vandiver_primes():
    rows = read_golden("known_primes.txt")
    for kind, p in rows:
        p = int(p)
        if kind == "wolstenholme":
            assert oracle.congruence_residue(p, C.SV) == 0, p
            assert oracle.congruence_residue(p, C.BB30) == 0, p
        elif kind == "vandiver":
            assert oracle.congruence_residue(p, C.EE33, nthreads=8) == 0, p
            if p < 10 ** 8:
                assert oracle.congruence_residue(p, C.E1, nthreads=8) == 0, p
        elif kind == "not_vandiver":
            assert oracle.congruence_residue(p, C.E1) != 0
            assert oracle.congruence_residue(p, C.EE33) != 0
    # below 1e5: exactly these hits (brute force over every prime)
    ps = oracle.primes(5, 100000)
    res = oracle.residues(ps)
    assert [p for p, (b, _) in zip(ps, res) if b == 0] == [16843]
    assert [p for p, (_, e) in zip(ps, res) if e == 0] == [149, 241]


def _near_miss(name, cong, limit, slow, ends_only=False):
    rows = [(int(p), int(r)) for p, r in read_golden(name)]
    rows = sorted((p, r) for p, r in rows if (p >= limit) == slow)
    if ends_only:
        rows = [rows[0], rows[-1]]
    for p, r in rows:
        got = oracle.congruence_residue(p, cong, nthreads=oracle.max_threads())
        assert exact.symmetric(got, p) == r, (p, r, got)


def test_table2_near_misses():
    _near_miss("near_miss_B.txt", C.BB30, 1.6e10, slow=False)


def test_table3_near_misses():
    _near_miss("near_miss_E.txt", C.EE33, 1.2e10, slow=False)


def test_tables_2_and_3_largest_printed_primes():
    """The smallest and the largest printed prime of each table above the
    default range (up to 7.76e10, Tables 2 and 3): the oracle's plain
    eqnBB30 / eqnEE33 gives the printed symmetric residues; the slow tests
    below check every printed prime up there."""
    _near_miss("near_miss_B.txt", C.BB30, 1.6e10, slow=True, ends_only=True)
    _near_miss("near_miss_E.txt", C.EE33, 1.2e10, slow=True, ends_only=True)


@pytest.mark.slow
def test_table2_near_misses_large():
    _near_miss("near_miss_B.txt", C.BB30, 1.6e10, slow=True)


@pytest.mark.slow
def test_table3_near_misses_large():
    _near_miss("near_miss_E.txt", C.EE33, 1.2e10, slow=True)


def test_table2_root_form_cross_check():
    """Two Table 2 and Table 3 entries once more by the root forms (eqnBB1, eqnE1)."""
    assert exact.symmetric(oracle.congruence_residue(1029113299, C.SV, nthreads=8), 1029113299) == -7
    assert exact.symmetric(oracle.congruence_residue(1348936931, C.E1, nthreads=8), 1348936931) == -17


# ---------------------------------------------------------------------------
# Sieve
# ---------------------------------------------------------------------------


def test_sieve_textbook_counts():
    # pi(10^k) for k = 1..7
    for k, pi in zip(range(1, 8), [4, 25, 168, 1229, 9592, 78498, 664579]):
        assert len(oracle.primes(0, 10 ** k + 1)) == pi
    assert oracle.primes(0, 60) == small_primes(0, 60)
    assert oracle.primes(10 ** 6, 10 ** 6 + 5000) == small_primes(10 ** 6, 10 ** 6 + 5000)
    # Section 3 counts its primes from 5 on: [5, 1e5) has pi(1e5) - 2 primes
    assert len(oracle.primes(5, 10 ** 5)) == 9590


def test_residues_dispatch_small_and_large_agree():
    ps = [p for p in PRIMES_5_2000 if p >= 11][-20:]
    small = oracle.residues(ps)
    via_root = list(zip(oracle.congruence_residues(ps, C.SV), oracle.congruence_residues(ps, C.E1)))
    via_table = oracle.residues([p + 0 for p in ps], method="table")
    assert small == via_root
    # method="table" still uses the recurrence below 2000, so check above it
    big = oracle.primes(2000, 2400)
    assert oracle.residues(big, "root") == oracle.residues(big, "table")
    assert via_table == small
    assert oracle.residues([5, 7]) == [(1, 1), (3, 5)]


# ---------------------------------------------------------------------------
# residue statistics (histograms of Sections 3 and 5, Tables 2 and 3)
# ---------------------------------------------------------------------------

def test_residue_stats_bins_equal_p_is_a_bijection():
    """With bins = p, floor((s/p + 1/2) p) = s + (p-1)/2: every residue has its
    own bin, in order, so an offset, sign or scaling slip moves some bin."""
    for p in (11, 13, 101, 997):
        rows = [(p, r, (p - r) % p) for r in range(p)]
        hb, he, _ = oracle.residue_stats(rows, bins=p, bound=0)
        assert hb == [1] * p and he == [1] * p
        for r in range(p):
            s = exact.symmetric(r, p)
            one, _, _ = oracle.residue_stats([(p, r, 0)], bins=p, bound=0)
            assert one.index(1) == s + (p - 1) // 2


def test_residue_stats_small_bin_counts():
    """bins = 1 puts everything in bin 0; bins = 2 splits at <r> < 0; the
    extremes +-(p-1)/2 land in the first and last bins."""
    p = 1000003
    rows = [(p, 0, 1), (p, p - 1, (p - 1) // 2), (p, (p + 1) // 2, 5)]
    hb, he, near = oracle.residue_stats(rows, bins=1, bound=0)
    assert hb == [3] and he == [3] and near == []
    hb, he, _ = oracle.residue_stats(rows, bins=2, bound=0)
    assert hb == [2, 1] and he == [0, 3]
    hb, he, _ = oracle.residue_stats(rows, bins=2000, bound=0)
    assert hb[0] == 1 and he[1999] == 1 and hb[1000] == 1


def test_residue_stats_near_misses_from_table_2_and_3():
    """The printed near misses come back with their printed signed values."""
    rows_b = [(int(p), int(r)) for p, r in read_golden("near_miss_B.txt")]
    rows_e = [(int(p), int(r)) for p, r in read_golden("near_miss_E.txt")]
    for rows, which in ((rows_b, 1), (rows_e, 2)):
        data = []
        for p, r in rows[:4]:
            far = (p - 1) // 2                      # the other residue: far from 0
            data.append((p, r % p, far) if which == 1 else (p, far, r % p))
        _, _, near = oracle.residue_stats(data, bins=2000, bound=50)
        assert near == sorted(((p, r, which) for p, r in rows[:4]), key=lambda t: (t[0], t[2]))
        cut = sorted(abs(r) for _, r in rows[:4])[2]
        _, _, near = oracle.residue_stats(data, bins=2000, bound=cut)
        assert near == sorted(((p, r, which) for p, r in rows[:4] if abs(r) < cut), key=lambda t: (t[0], t[2]))


# ---------------------------------------------------------------------------
# Every index: irregular and E-irregular pairs (Section 1)
# ---------------------------------------------------------------------------


def test_all_index_recurrences_match_exact_rationals():
    """B_{2k}, E_{2k} mod p for every 2k <= p - 3 equal the exact EGF
    coefficients reduced mod p (textbook values, independent of the oracle)."""
    ps = small_primes(5, 200)
    B = exact.bernoulli_egf(ps[-1] - 3)
    E = [int(x) for x in exact.euler_egf(ps[-1] - 3)]
    for p in ps:
        want_b = [exact.rational_mod_p(B[2 * k], p) for k in range(1, (p - 3) // 2 + 1)]
        want_e = [E[2 * k] % p for k in range(1, (p - 3) // 2 + 1)]
        assert oracle.bernoulli_all(p) == want_b, p
        assert oracle.euler_all(p) == want_e, p


def test_all_index_last_entry_is_the_p_minus_3_residue():
    for p in small_primes(7, 400):
        assert oracle.bernoulli_all(p)[-1] == b_rec(p)
        assert oracle.euler_all(p)[-1] == e_rec(p)


def test_smallest_irregular_and_e_irregular_primes():
    """Section 1: 37 is the smallest irregular prime, 19 the smallest
    E-irregular one (19 | E_10)."""
    first_b = next(p for p in small_primes(5, 100) if any(x[2] == 1 for x in oracle.irregular_pairs(p)))
    first_e = next(p for p in small_primes(5, 100) if any(x[2] == 2 for x in oracle.irregular_pairs(p)))
    assert first_b == 37 and first_e == 19
    assert (19, 10, 2) in oracle.irregular_pairs(19)


def test_wolstenholme_and_vandiver_primes_are_extremal_pairs():
    """Section 1: (p, p-3) is an irregular pair at a Wolstenholme prime and an
    E-irregular pair at a Vandiver prime."""
    assert (16843, 16840, 1) in oracle.irregular_pairs(16843)
    for p in (149, 241):
        assert (p, p - 3, 2) in oracle.irregular_pairs(p)


def test_e_index_of_5783_is_five():
    """Section 1: p = 5783 has index of E-irregularity 5."""
    assert sum(1 for x in oracle.irregular_pairs(5783) if x[2] == 2) == 5


@pytest.mark.slow
def test_e_irregularity_census_below_10_4():
    """Section 1: below 10^4 the largest index of E-irregularity is 5,
    attained by 5783 alone."""
    from concurrent.futures import ThreadPoolExecutor
    ps = small_primes(5, 10 ** 4)
    with ThreadPoolExecutor(8) as ex:
        idx = dict(zip(ps, ex.map(lambda p: sum(1 for x in oracle.irregular_pairs(p) if x[2] == 2), ps)))
    top = max(idx.values())
    assert top == 5 and [p for p, v in idx.items() if v == top] == [5783]
