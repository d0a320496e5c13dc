"""Congruences of the paper, transcribed for the oracle (test infrastructure only).

This module is part of the oracle: plain data typed in from the paper, used by
the oracle's CPU evaluators and by the tests.  Nothing in the product package
imports it; the product keeps its own, separately typed copy of the tables.

Notation (Booker, Hathi, Mossinghoff, Trudgian, "Wolstenholme and Vandiver
primes", arXiv:2101.11157):

* S_l(x, y) = sum over integers s with x*p < s < y*p of s^l, taken mod p
  (Section 2, definition of S_l, eqnDefnS).  The interval is open.
* At the index used by the searches, S_{p-4} == sum s^-3 (Bernoulli side,
  Section 3, the remark after eqnBB30) and S_{p-3} == sum s^-2 (Euler side,
  Section 5, opening paragraph).
* Each specialised congruence reads  L * X_{p-3} == sum_i c_i S(x_i, y_i)
  (mod p) with X = B (Bernoulli) or E (Euler, secant convention, footnote to
  the Euler EGF in Section 1).

Every table carries the cost p*sum(y_i - x_i) that the paper prints for it;
the tests recompute that sum exactly and compare (a transcription pin).
"""
from fractions import Fraction as F

__all__ = ["Congruence", "TABLES_B", "TABLES_E", "ROOT_FORMS", "ALL_TABLES", "table", "tanner_wagstaff"]


class Congruence:
    """One congruence  lhs * X_{p-3} == sum c_i * S_ell(x_i, y_i)  (mod p).

    kind   'B' or 'E'
    ell    exponent of s in each summand: -3 for B_{p-3}, -2 for E_{p-3}
    alt    True when the summand carries the sign (-1)^s (McIntosh's S-tilde,
           Section 4, eqnMacE)
    lhs    integer multiplier of X_{p-3}
    terms  list of (c_i, x_i, y_i) with integer c_i and Fraction endpoints
    cost   Fraction printed by the paper for p*sum(y_i - x_i), divided by p
    min_p  smallest prime for which the congruence is used by the oracle
    cite   where the paper states it
    """

    def __init__(self, name, kind, ell, lhs, terms, cost, cite, min_p=11, alt=False):
        self.name = name
        self.kind = kind
        self.ell = ell
        self.lhs = lhs
        self.terms = [(int(c), F(x), F(y)) for c, x, y in terms]
        self.cost = F(cost)
        self.cite = cite
        self.min_p = min_p
        self.alt = alt

    def exact_cost(self):
        return sum((y - x for _, x, y in self.terms), F(0))

    def __repr__(self):
        return f"Congruence({self.name}, {len(self.terms)} sums, cost {self.cost})"


def _f(s):
    """'a/b' -> Fraction; '0' -> 0."""
    return F(s)


def _t(*rows):
    return [(c, _f(x), _f(y)) for c, x, y in rows]


# ---------------------------------------------------------------------------
# Root congruences at the search index (used as independent oracle forms).
# ---------------------------------------------------------------------------

# Stafford-Vandiver, Section 2 eqnSV; at k=(p-3)/2 the factor C_k(3,4,6)
# becomes (6^3-3^3-4^3+1)/6 = 21 (Section 3, first display), which is eqnBB1.
SV = Congruence("SV", "B", -3, 21, _t((1, "1/6", "1/4")), "1/12",
                "Section 2 eqnSV; Section 3 eqnBB1", min_p=5)

# Voronoi form, Section 2 eqnV12: C_k(2,3,4) B_2k == S(1/4,1/3); at
# k=(p-3)/2, C_k(2,3,4) = (4^3-2^3-3^3+1)/6 = 5.
V12 = Congruence("V12", "B", -3, 5, _t((1, "1/4", "1/3")), "1/12",
                 "Section 2 eqnV12 with the specialisation of C_k in Section 3", min_p=5)

# Vandiver, Section 2 eqnVandiver; C_k(2,5,6) -> (6^3-2^3-5^3+1)/6 = 14.
VANDIVER = Congruence("Vandiver", "B", -3, 14,
                      _t((1, "1/6", "1/5"), (1, "1/3", "2/5")), "1/10",
                      "Section 2 eqnVandiver", min_p=7)

# Section 2 eqnV10; C_k(4,5,8) -> (8^3-4^3-5^3+1)/6 = 54.
V10 = Congruence("V10", "B", -3, 54,
                 _t((1, "1/8", "1/5"), (1, "3/8", "2/5")), "1/10",
                 "Section 2 eqnV10", min_p=7)


def tanner_wagstaff(b):
    """Section 2 eqnTW1 at k=(p-3)/2: C_k(2,b,b+1) -> ((b+1)^3-8-b^3+1)/6.

    Valid for p > b+1 (the paper's hypothesis), cost floor(b/2)(floor(b/2)+1)/(2b(b+1)).
    """
    lhs = ((b + 1) ** 3 - 8 - b ** 3 + 1) // 6
    beta = b // 2
    terms = [(1, F(m, b + 1), F(m, b)) for m in range(1, beta + 1)]
    cost = F(beta * (beta + 1), 2 * b * (b + 1))
    return Congruence(f"TW1(b={b})", "B", -3, lhs, terms, cost,
                      "Section 2 eqnTW1", min_p=max(b + 2, 5))


# Glaisher, Section 4 eqnE1, read with the sign (-1)^k (the printed factor
# (-1)^((p-1)/2-k) contradicts eqnE3 and eqnEE3; see the oracle notes).
# At k=1: -4 E_{p-3} == S_{p-3}(0,1/4) == sum s^-2.
E1 = Congruence("E1", "E", -2, -4, _t((1, "0", "1/4")), "1/4",
                "Section 4 eqnE1 (sign read as (-1)^k)", min_p=5)

# McIntosh, Section 4 eqnMacE at k=1: -(9+1) E_{p-3} == S-tilde(0,1/6),
# valid for p not dividing 10.
MACE = Congruence("MacE", "E", -2, -10, _t((1, "0", "1/6")), "1/6",
                  "Section 4 eqnMacE at k=1", min_p=7, alt=True)

ROOT_FORMS = {c.name: c for c in (SV, V12, VANDIVER, V10, E1, MACE)}

# ---------------------------------------------------------------------------
# Specialised Bernoulli tables, Section 3 (eqnBB2, eqnBB1, eqnBB6, eqnBB9,
# eqnBB16, eqnBB22, eqnBB30).  S = S_{p-4} = sum s^-3.
# ---------------------------------------------------------------------------

BB1 = Congruence("BB1", "B", -3, 21, _t((1, "1/6", "1/4")), "1/12",
                 "Section 3 eqnBB1")

BB2 = Congruence("BB2", "B", -3, 112, _t(
    (9, "1/6", "1/5"),
    (-1, "3/10", "1/3"),
), "1/15", "Section 3 eqnBB2")

BB6 = Congruence("BB6", "B", -3, 458752, _t(
    (-512, "3/20", "13/80"),
    (-520, "13/80", "1/6"),
    (36929, "1/6", "27/160"),
    (36928, "27/160", "7/40"),
    (36864, "7/40", "1/5"),
    (-1, "53/160", "1/3"),
), "5/96", "Section 3 eqnBB6")

BB9 = Congruence("BB9", "B", -3, 336000, _t(
    (1000, "1/18", "11/180"),
    (976, "11/180", "1/15"),
    (-101, "2/15", "5/36"),
    (125, "7/36", "1/5"),
    (-24, "47/180", "4/15"),
    (-3125, "3/10", "11/36"),
    (24, "1/3", "61/180"),
    (125, "13/36", "11/30"),
    (-24, "83/180", "7/15"),
), "1/20", "Section 3 eqnBB9")

BB16 = Congruence("BB16", "B", -3, 72576000, _t(
    (216000, "1/18", "11/180"),
    (210816, "11/180", "7/108"),
    (211816, "7/108", "47/720"),
    (211735, "47/720", "1/15"),
    (-25000, "1/10", "11/108"),
    (-21816, "2/15", "5/36"),
    (-648, "83/360", "25/108"),
    (24352, "25/108", "7/30"),
    (-352, "4/15", "29/108"),
    (648, "29/108", "97/360"),
    (5184, "1/3", "61/180"),
    (27000, "13/36", "11/30"),
    (648, "11/30", "133/360"),
    (1000, "43/108", "2/5"),
    (-24919, "13/30", "313/720"),
    (-25000, "313/720", "47/108"),
), "1/24", "Section 3 eqnBB16")

BB22 = Congruence("BB22", "B", -3, 72576000, _t(
    (216024, "1/18", "61/1080"),
    (216000, "61/1080", "11/180"),
    (210816, "11/180", "7/108"),
    (211816, "7/108", "47/720"),
    (211735, "47/720", "1/15"),
    (-25000, "1/10", "11/108"),
    (-21860, "2/15", "29/216"),
    (-21735, "29/216", "97/720"),
    (-21816, "97/720", "5/36"),
    (-192, "119/540", "479/2160"),
    (-195, "479/2160", "2/9"),
    (-648, "83/360", "25/108"),
    (24352, "25/108", "7/30"),
    (3, "5/18", "601/2160"),
    (27000, "13/36", "263/720"),
    (26919, "263/720", "79/216"),
    (27044, "79/216", "11/30"),
    (648, "11/30", "133/360"),
    (1000, "43/108", "2/5"),
    (-24919, "13/30", "313/720"),
    (-25000, "313/720", "47/108"),
    (192, "4/9", "241/540"),
), "3/80", "Section 3 eqnBB22")

BB30 = Congruence("BB30", "B", -3, 15676416000, _t(
    (46661184, "1/18", "61/1080"),
    (46656000, "61/1080", "11/180"),
    (45536256, "11/180", "7/108"),
    (45752256, "7/108", "47/720"),
    (45734760, "47/720", "43/648"),
    (45735760, "43/648", "1/15"),
    (-5401000, "1/10", "65/648"),
    (-5400000, "65/648", "11/108"),
    (-4721885, "2/15", "173/1296"),
    (-4721760, "173/1296", "29/216"),
    (-4694760, "29/216", "97/720"),
    (-4712256, "97/720", "299/2160"),
    (-4712904, "299/2160", "5/36"),
    (-41472, "119/540", "479/2160"),
    (-42120, "479/2160", "2/9"),
    (5184, "2/9", "241/1080"),
    (-139968, "83/360", "25/108"),
    (5260032, "25/108", "151/648"),
    (5261032, "151/648", "7/30"),
    (648, "5/18", "601/2160"),
    (5832648, "13/36", "781/2160"),
    (5832000, "781/2160", "263/720"),
    (5814504, "263/720", "79/216"),
    (5841504, "79/216", "475/1296"),
    (5841629, "475/1296", "11/30"),
    (139968, "11/30", "133/360"),
    (1000, "259/648", "2/5"),
    (-5383504, "13/30", "281/648"),
    (-5382504, "281/648", "313/720"),
    (-5400000, "313/720", "47/108"),
), "227/6480", "Section 3 eqnBB30")

# ---------------------------------------------------------------------------
# Specialised Euler tables, Section 5 (eqnEE3 ... eqnEE33).  S = sum s^-2.
# ---------------------------------------------------------------------------

EE3 = Congruence("EE3", "E", -2, -64, _t(
    (1, "0", "1/16"),
    (4, "3/8", "7/16"),
    (5, "7/16", "1/2"),
), "3/16", "Section 5 eqnEE3")

EE5 = Congruence("EE5", "E", -2, -1024, _t(
    (1, "0", "1/64"),
    (64, "3/8", "7/16"),
    (80, "7/16", "15/32"),
    (84, "15/32", "31/64"),
    (85, "31/64", "1/2"),
), "9/64", "Section 5 eqnEE5")

EE9 = Congruence("EE9", "E", -2, -36864, _t(
    (9, "0", "1/128"),
    (256, "1/8", "7/48"),
    (256, "3/16", "5/24"),
    (2880, "7/16", "11/24"),
    (3136, "11/24", "15/32"),
    (3280, "15/32", "23/48"),
    (3024, "23/48", "31/64"),
    (3060, "31/64", "63/128"),
    (3069, "63/128", "1/2"),
), "43/384", "Section 5 eqnEE9")

EE16 = Congruence("EE16", "E", -2, -1327104, _t(
    (81, "0", "1/256"),
    (3328, "1/16", "5/72"),
    (2304, "5/72", "7/96"),
    (11520, "7/48", "11/72"),
    (11520, "13/72", "3/16"),
    (28224, "11/48", "15/64"),
    (1024, "19/72", "17/64"),
    (29248, "17/64", "13/48"),
    (1024, "19/48", "29/72"),
    (2304, "41/96", "7/16"),
    (118080, "15/32", "23/48"),
    (120384, "23/48", "31/64"),
    (121680, "31/64", "35/72"),
    (110160, "35/72", "63/128"),
    (110484, "63/128", "127/256"),
    (110565, "127/256", "1/2"),
), "205/2304", "Section 5 eqnEE16")

EE24 = Congruence("EE24", "E", -2, -5308416, _t(
    (81, "0", "1/512"),
    (832, "1/64", "5/288"),
    (9216, "5/72", "41/576"),
    (9472, "41/576", "7/96"),
    (46080, "7/48", "11/72"),
    (46080, "13/72", "3/16"),
    (1024, "3/16", "55/288"),
    (112896, "11/48", "67/288"),
    (113728, "67/288", "15/64"),
    (118080, "15/64", "137/576"),
    (118080, "151/576", "19/72"),
    (122176, "19/72", "17/64"),
    (117824, "17/64", "77/288"),
    (116992, "77/288", "13/48"),
    (4096, "19/48", "29/72"),
    (256, "41/96", "247/576"),
    (473344, "137/288", "23/48"),
    (481536, "23/48", "139/288"),
    (482368, "139/288", "31/64"),
    (486720, "31/64", "35/72"),
    (440640, "35/72", "63/128"),
    (441936, "63/128", "127/256"),
    (442260, "127/256", "255/512"),
    (442341, "255/512", "1/2"),
), "115/1536", "Section 5 eqnEE24")

EE33 = Congruence("EE33", "E", -2, 477757440, _t(
    (-729, "0", "1/1536"),
    (82944, "5/144", "11/288"),
    (36864, "61/432", "31/216"),
    (995328, "11/72", "133/864"),
    (1004544, "133/864", "67/432"),
    (995328, "67/432", "17/108"),
    (1142784, "17/108", "205/1296"),
    (1146880, "205/1296", "103/648"),
    (1142784, "103/648", "23/144"),
    (1059840, "23/144", "35/216"),
    (1059840, "37/216", "25/144"),
    (1142784, "25/144", "113/648"),
    (1146880, "113/648", "227/1296"),
    (1142784, "227/1296", "19/108"),
    (995328, "19/108", "77/432"),
    (1004544, "77/432", "155/864"),
    (995328, "155/864", "13/72"),
    (1327104, "13/72", "41/216"),
    (1363968, "41/216", "83/432"),
    (1327104, "83/432", "7/36"),
    (9206784, "35/72", "421/864"),
    (9216000, "421/864", "211/432"),
    (9206784, "211/432", "47/96"),
    (9020160, "47/96", "53/108"),
    (9167616, "53/108", "637/1296"),
    (9171712, "637/1296", "319/648"),
    (9167616, "319/648", "71/144"),
    (9084672, "71/144", "95/192"),
    (9038016, "95/192", "107/216"),
    (7978176, "107/216", "191/384"),
    (7966512, "191/384", "383/768"),
    (7963596, "383/768", "767/1536"),
    (7962867, "767/1536", "1/2"),
), "27/512", "Section 5 eqnEE33")

TABLES_B = {c.name: c for c in (BB1, BB2, BB6, BB9, BB16, BB22, BB30)}
TABLES_E = {c.name: c for c in (EE3, EE5, EE9, EE16, EE24, EE33)}
ALL_TABLES = {**TABLES_B, **TABLES_E}


def table(name):
    if name in ALL_TABLES:
        return ALL_TABLES[name]
    if name in ROOT_FORMS:
        return ROOT_FORMS[name]
    raise KeyError(name)
