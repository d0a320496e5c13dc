"""Derivation of congruences for B_{p-3} and E_{p-3} mod p.

Host-side generator of the tables the term-sum kernels evaluate (the step
before the hot path).  Implements, in exact rational arithmetic:

* the three transformations of Proposition propTW (Section 2): separation,
  reflection S_l(x, y) == (-1)^l S_l(1-y, 1-x), and subdivision
  S_l(x, y) == d^l sum_{i<d} S_l((x+i)/d, (y+i)/d) for p not dividing d;
* the exhaustive search of Section 2.1 (every sequence of at most L
  subdivisions, the i-th with 2 <= d <= d_i) and the greedy search of
  Section 2.2 (lambda subdivisions with d <= D per round, keep a cheapest
  result, repeat);
* the starting congruences of Sections 2 and 4, specialised to the index the
  searches need: for B_{p-3}, k = (p-3)/2 and l = p - 4 == -3 (mod p - 1), so
  d^l == d^-3 and C_k(a, b, c) == (c^3 - a^3 - b^3 + 1)/6 (Section 3); for
  E_{p-3}, k = 1 and l = p - 3 == -2, so d^l == d^-2 and reflection keeps the
  sign.

A congruence is held as  lhs * X == sum_i c_i S(x_i, y_i)  with X = B_{p-3} or
E_{p-3}, the right side as a piecewise-constant coefficient function on
[0, 1/2] (every interval reflected below 1/2, which the reflection property
allows; p/2 is never an integer, so splitting at 1/2 is a valid separation).
Each maximal interval of constant nonzero coefficient is one sum; the cost is
p times their total length (Section 2).

The congruences derived here hold for every prime p >= 11 that divides no
subdivision factor (factors are at most 8 here, so every p >= 11), as long as
the starting congruence holds and p does not divide lhs.
"""
from bisect import bisect_left, bisect_right
from fractions import Fraction as Q
from math import gcd
import itertools
import json

HALF = Q(1, 2)

# (name, side, lhs, [(coef, x, y)]) at the index p-3, Sections 2-4
#   Vandiver:  C_k(2,5,6) = (216 - 8 - 125 + 1)/6 = 14
#   SV:        C_k(3,4,6) = (216 - 27 - 64 + 1)/6 = 21
#   V12:       C_k(2,3,4) = (64 - 8 - 27 + 1)/6 = 5
#   V10:       C_k(4,5,8) = (512 - 64 - 125 + 1)/6 = 54
#   E1:        (-1)^k 4^(2k-1) with k = 1: -4
#   EMac2:     (-1)^k 4^(k-1) (9^k + 1) with k = 1: -10, right side 2^t (...) = (1/4)(...)
STARTS = {
    "Vandiver": ("B", 14, [(1, Q(1, 6), Q(1, 5)), (1, Q(1, 3), Q(2, 5))]),
    "SV": ("B", 21, [(1, Q(1, 6), Q(1, 4))]),
    "V12": ("B", 5, [(1, Q(1, 4), Q(1, 3))]),
    "V10": ("B", 54, [(1, Q(1, 8), Q(1, 5)), (1, Q(3, 8), Q(2, 5))]),
    "E1": ("E", -4, [(1, Q(0), Q(1, 4))]),
    "EMac2": ("E", -10, [(Q(1, 4), Q(0), Q(1, 12)), (Q(-1, 4), Q(5, 12), HALF)]),
}

SIDES = {"B": (3, -1), "E": (2, 1)}   # side -> (power k in d^-k, reflection sign)


def tw1(b):
    """eqnTW1 at the index p-3: C_k(2, b, b+1) = ((b+1)^3 - 8 - b^3 + 1)/6, right
    side sum_{m=1}^{floor(b/2)} S(m/(b+1), m/b)."""
    lhs = Q((b + 1) ** 3 - 8 - b ** 3 + 1, 6)
    return ("B", lhs, [(1, Q(m, b + 1), Q(m, b)) for m in range(1, b // 2 + 1)])


class Poly:
    """A coefficient of a general-index congruence: sum_n m_n n^t for the
    exponent t of the sums (t = 2k - 1 for B_{2k}, t = p - 1 - 2k for E_t),
    held as {n: m_n} with rational m_n.  Subdivision by d multiplies by d^t
    (n -> n d); reflection multiplies by (-1)^t, a constant sign per side."""

    __slots__ = ("m",)

    def __init__(self, m=None):
        self.m = {n: Q(v) for n, v in (m or {}).items() if v != 0}

    @staticmethod
    def of(v):
        return v if isinstance(v, Poly) else Poly({1: Q(v)} if v != 0 else {})

    def __add__(self, o):
        o = Poly.of(o)
        r = dict(self.m)
        for n, v in o.m.items():
            r[n] = r.get(n, Q(0)) + v
        return Poly(r)

    __radd__ = __add__

    def __neg__(self):
        return Poly({n: -v for n, v in self.m.items()})

    def __sub__(self, o):
        return self + (-Poly.of(o))

    def __mul__(self, k):
        if isinstance(k, Poly):
            raise TypeError("coefficients multiply only by constants")
        return Poly({n: v * k for n, v in self.m.items()})

    __rmul__ = __mul__

    def times_power(self, d):
        """self * d^t."""
        return Poly({n * d: v for n, v in self.m.items()})

    def __eq__(self, o):
        if isinstance(o, (int, Q)):
            return (not self.m) if o == 0 else self.m == {1: Q(o)}
        return isinstance(o, Poly) and self.m == o.m

    def __ne__(self, o):
        return not self.__eq__(o)

    def __hash__(self):
        return hash(tuple(sorted(self.m.items())))

    def __repr__(self):
        return " + ".join(f"{v}*{n}^t" for n, v in sorted(self.m.items())) or "0"

    def at(self, t, p):
        """Value mod p at the exponent t (any integer; p prime to every base)."""
        acc = 0
        for n, v in self.m.items():
            acc += v.numerator * pow(v.denominator, -1, p) * pow(n, t, p)
        return acc % p

    def specialise(self, e):
        """Rational value at the exponent t = e (e <= 0 allowed)."""
        return sum((v * Q(n) ** e for n, v in self.m.items()), Q(0))


# General-index starting congruences (Sections 2 and 4), coefficients as
# polynomials in the powers n^t; the left sides are named, not evaluated:
#   C256 = C_k(2,5,6) (Vandiver, and every congruence derived from it),
#   C346 = C_k(3,4,6) (SV), C234 = C_k(2,3,4) (V12),
#   E1 = (-1)^k 4^(2k-1) (eqnE1, sign read as (-1)^k; exponent t = p - 1 - 2k),
#   MacE = (-1)^k 4^(k-1) (9^k + 1) (eqnMacE / eqnEMac2).
GENERAL_STARTS = {
    "Vandiver": ("B", "C256", [(Poly({1: 1}), Q(1, 6), Q(1, 5)), (Poly({1: 1}), Q(1, 3), Q(2, 5))]),
    "SV": ("B", "C346", [(Poly({1: 1}), Q(1, 6), Q(1, 4))]),
    "V12": ("B", "C234", [(Poly({1: 1}), Q(1, 4), Q(1, 3))]),
    "E1": ("E", "E1", [(Poly({1: 1}), Q(0), Q(1, 4))]),
    "EMac2": ("E", "MacE", [(Poly({2: 1}), Q(0), Q(1, 12)), (Poly({2: -1}), Q(5, 12), HALF)]),
}


class Congruence:
    """lhs * X == sum over pieces c * S(x, y), pieces disjoint in [0, 1/2]."""

    def __init__(self, side, lhs, terms=(), general=False):
        if side not in SIDES:
            raise ValueError("side is 'B' or 'E'")
        self.side = side
        self.power, self.refl = SIDES[side]
        # general: coefficients are Poly (any index), lhs a name; otherwise
        # rationals at the index p - 3 and a rational lhs
        self.general = general
        self.lhs = lhs if general else Q(lhs)
        self.bp = []   # breakpoints, ascending
        self.cf = []   # cf[j]: coefficient on (bp[j], bp[j+1]); len(cf) == len(bp) - 1 (or both empty)
        for c, x, y in terms:
            self.add(Q(x), Q(y), Poly.of(c) if general else Q(c))

    @classmethod
    def start(cls, name, general=False):
        if general:
            side, lhs, terms = GENERAL_STARTS[name]
            return cls(side, lhs, terms, general=True)
        side, lhs, terms = tw1(int(name[3:])) if name.startswith("TW1") else STARTS[name]
        return cls(side, lhs, terms)

    def copy(self):
        o = Congruence.__new__(Congruence)
        o.side, o.power, o.refl, o.lhs, o.general = self.side, self.power, self.refl, self.lhs, self.general
        o.bp, o.cf = list(self.bp), list(self.cf)
        return o

    def _zero(self):
        return Poly() if self.general else Q(0)

    def _images_weight(self, c, d):
        """Coefficient of each of the d images of a sum with coefficient c."""
        return c.times_power(d) if self.general else c / Q(d) ** self.power

    def specialise(self):
        """The index p - 3 form of a general congruence (n^t -> n^-3 for B,
        n^-2 for E); the left side stays named."""
        o = Congruence(self.side, 1)
        o.lhs = self.lhs
        for c, x, y in self.pieces():
            o.add(x, y, c.specialise(-self.power))
        return o

    # ---- the coefficient function ----------------------------------------
    def _cut(self, t):
        """Make t a breakpoint (inside or at the ends of the support)."""
        if not self.bp:
            self.bp = [t]
            return
        if t < self.bp[0]:
            self.bp.insert(0, t)
            self.cf.insert(0, self._zero())
            return
        if t > self.bp[-1]:
            self.bp.append(t)
            self.cf.append(self._zero())
            return
        j = bisect_left(self.bp, t)
        if self.bp[j] != t:
            self.bp.insert(j, t)
            self.cf.insert(j, self.cf[j - 1])

    def _raw_add(self, x, y, c):
        if not (0 <= x < y <= HALF):
            raise ValueError("interval outside [0, 1/2]")
        self._cut(x)
        self._cut(y)
        i, j = bisect_left(self.bp, x), bisect_left(self.bp, y)
        for k in range(i, j):
            self.cf[k] += c
        self._tidy(max(i - 1, 0), min(j + 1, len(self.bp)))

    def _tidy(self, lo, hi):
        """Drop breakpoints in bp[lo:hi] that separate equal coefficients, and
        zero-coefficient ends."""
        k = max(lo, 1)
        while k < min(hi, len(self.bp) - 1):
            if self.cf[k - 1] == self.cf[k]:
                del self.bp[k]
                del self.cf[k]
                hi -= 1
            else:
                k += 1
        while self.cf and self.cf[0] == 0:
            del self.bp[0]
            del self.cf[0]
        while self.cf and self.cf[-1] == 0:
            del self.bp[-1]
            del self.cf[-1]
        if not self.cf:
            self.bp = []

    def add(self, x, y, c):
        """c * S(x, y) for any 0 <= x < y <= 1, reflected into [0, 1/2]."""
        if c == 0 or x == y:
            return
        if y <= HALF:
            self._raw_add(x, y, c)
        elif x >= HALF:
            self._raw_add(1 - y, 1 - x, self.refl * c)
        else:
            self._raw_add(x, HALF, c)
            self._raw_add(1 - y, HALF, self.refl * c)

    # ---- transformations ------------------------------------------------
    def pieces(self):
        """[(c, x, y)]: the sums, ascending."""
        return [(c, self.bp[j], self.bp[j + 1]) for j, c in enumerate(self.cf) if c != 0]

    def subdivide(self, x, y, d):
        """Replace the sum on (x, y) (an existing piece) by d^-k times its d images."""
        c = self._coef_of(x, y)
        self.add(x, y, -c)
        w = self._images_weight(c, d)
        for i in range(d):
            self.add((x + i) / d, (y + i) / d, w)
        return self

    def _coef_of(self, x, y):
        j = bisect_left(self.bp, x)
        if j >= len(self.cf) or self.bp[j] != x or self.bp[j + 1] != y or self.cf[j] == 0:
            raise KeyError(f"({x}, {y}) is not a sum of this congruence")
        return self.cf[j]

    # ---- measures -------------------------------------------------------
    def cost(self):
        """Total length of the sums (cost / p)."""
        return sum((self.bp[j + 1] - self.bp[j] for j, c in enumerate(self.cf) if c != 0), Q(0))

    def n_sums(self):
        return sum(1 for c in self.cf if c != 0)

    def value_at(self, t):
        """Coefficient at a point t in (0, 1/2) that is not a breakpoint."""
        j = bisect_right(self.bp, t) - 1
        return self.cf[j] if 0 <= j < len(self.cf) else self._zero()

    def cost_after(self, x, y, d):
        """cost() after subdivide(x, y, d), without changing the congruence."""
        return self.cost() + self.cost_delta(x, y, d)

    def cost_delta(self, x, y, d):
        """Change of cost() that subdivide(x, y, d) would make."""
        c = self._coef_of(x, y)
        w = self._images_weight(c, d)
        delta = [(x, y, -c)]
        for i in range(d):
            a, b = (x + i) / d, (y + i) / d
            if b <= HALF:
                delta.append((a, b, w))
            elif a >= HALF:
                delta.append((1 - b, 1 - a, self.refl * w))
            else:
                delta.append((a, HALF, w))
                delta.append((1 - b, HALF, self.refl * w))
        pts = set()
        for a, b, _ in delta:
            pts.add(a)
            pts.add(b)
            lo, hi = bisect_right(self.bp, a), bisect_left(self.bp, b)
            pts.update(self.bp[lo:hi])
        pts = sorted(pts)
        change = Q(0)
        for a, b in zip(pts, pts[1:]):
            mid = (a + b) / 2
            dv = sum((c2 for a2, b2, c2 in delta if a2 <= a and b <= b2), self._zero())
            if dv == 0:
                continue
            old = self.value_at(mid)
            change += (b - a) * ((old + dv != 0) - (old != 0))
        return change

    # ---- output ---------------------------------------------------------
    def integer_form(self):
        """(L, [(N_i, x_i, y_i)]) with L * X == sum N_i S(x_i, y_i), all integers,
        the common content divided out and L > 0."""
        ps = self.pieces()
        den = self.lhs.denominator
        for c, _, _ in ps:
            den = den * c.denominator // gcd(den, c.denominator)
        L = self.lhs * den
        Ns = [c * den for c, _, _ in ps]
        g = abs(int(L))
        for n in Ns:
            g = gcd(g, abs(int(n)))
        sgn = -1 if L < 0 else 1
        L = int(L) // g * sgn
        return L, [(int(n) // g * sgn, x, y) for n, (_, x, y) in zip(Ns, ps)]

    def to_json(self, name):
        L, terms = self.integer_form()
        return {"name": name, "side": self.side, "lhs": str(L), "n": len(terms),
                "cost": [self.cost().numerator, self.cost().denominator],
                "terms": [[str(n), x.numerator, x.denominator, y.numerator, y.denominator] for n, x, y in terms]}


# Subdivision steps (x, y, d) of the congruences the paper derives for every
# index, replayed on the general-index starts above.  Section 2.1 gives eqnB6
# from eqnB2 and eqnB9 ... eqnB30 in sequence; Section 4 gives eqnE3 ...
# eqnE24 from eqnE1 and eqnE33 from eqnEMac2.  eqnB2 is eqnVandiver with
# S(1/3, 2/5) subdivided by d = 2.  The recipe printed for eqnB9 starts "from
# eqnVandiver", but its last step subdivides S(11/36, 1/3), a sum that only
# eqnB2's term -2^t S(3/10, 1/3) provides; starting from eqnB2 reproduces
# the printed eqnB9 exactly, so that is the reading (eqnB16, B22, B30 follow
# from it as printed).
_F = lambda a, b=1: Q(a, b)
GENERAL_RECIPES = {
    "B2": ("Vandiver", [(_F(1, 3), _F(2, 5), 2)]),
    "B6": ("B2", [(_F(3, 10), _F(1, 3), 2), (_F(1, 3), _F(7, 20), 2), (_F(13, 40), _F(1, 3), 2),
                  (_F(1, 3), _F(27, 80), 2)]),
    "B9": ("B2", [(_F(1, 6), _F(1, 5), 3), (_F(4, 15), _F(5, 18), 2), (_F(7, 18), _F(2, 5), 2),
                  (_F(11, 36), _F(1, 3), 5)]),
    "B16": ("B9", [(_F(7, 36), _F(1, 5), 3), (_F(3, 10), _F(11, 36), 3), (_F(47, 180), _F(4, 15), 2),
                   (_F(47, 360), _F(2, 15), 2), (_F(83, 180), _F(7, 15), 2)]),
    "B22": ("B16", [(_F(1, 3), _F(61, 180), 3), (_F(1, 9), _F(61, 540), 2), (_F(4, 15), _F(29, 108), 2),
                    (_F(29, 108), _F(97, 360), 2), (_F(479, 1080), _F(4, 9), 2)]),
    "B30": ("B22", [(_F(43, 108), _F(2, 5), 6), (_F(4, 15), _F(173, 648), 2), (_F(4, 9), _F(241, 540), 2),
                    (_F(299, 1080), _F(5, 18), 2)]),
    "E3": ("E1", [(_F(0), _F(1, 4), 2), (_F(0), _F(1, 8), 2)]),
    "E5": ("E3", [(_F(0), _F(1, 16), 2), (_F(0), _F(1, 32), 2)]),
    "E9": ("E5", [(_F(0), _F(1, 64), 2), (_F(3, 8), _F(7, 16), 3)]),
    "E16": ("E9", [(_F(3, 16), _F(5, 24), 3), (_F(7, 16), _F(11, 24), 3), (_F(0), _F(1, 128), 2),
                   (_F(1, 8), _F(7, 48), 2), (_F(11, 24), _F(15, 32), 2)]),
    "E24": ("E16", [(_F(0), _F(1, 256), 2), (_F(1, 16), _F(5, 72), 4), (_F(41, 96), _F(7, 16), 3),
                    (_F(41, 288), _F(7, 48), 2), (_F(15, 32), _F(137, 288), 2)]),
    "E33": ("EMac2", [(_F(0), _F(1, 2 ** k * 3), 2) for k in range(2, 9)]
            + [(_F(5, 12), _F(11, 24), 3), (_F(11, 24), _F(17, 36), 3), (_F(17, 36), _F(23, 48), 3),
               (_F(23, 48), _F(35, 72), 3), (_F(5, 36), _F(11, 72), 2), (_F(5, 72), _F(11, 144), 2),
               (_F(61, 144), _F(31, 72), 3), (_F(133, 288), _F(67, 144), 3), (_F(205, 432), _F(103, 216), 3)]),
}


def general(name):
    """The general-index congruence `name` (a GENERAL_STARTS entry or a
    GENERAL_RECIPES one), built by replaying its subdivision steps."""
    if name in GENERAL_STARTS:
        return Congruence.start(name, general=True)
    base, steps = GENERAL_RECIPES[name]
    c = general(base)
    for x, y, d in steps:
        c.subdivide(x, y, d)
    return c


# ---------------------------------------------------------------------------
# transformation graphs (Section 7)
# ---------------------------------------------------------------------------

def parse_transformations(text):
    """Tokens of a transformation string in depth-first order: ('t', d) for
    tau_d (subdivision into d terms), ('s', f) for sigma_f (separation at the
    fraction f of the interval), ('r',) for rho (reflection), ('i',) for iota
    (a leaf).  Written as e.g. "t3 s1/2 i i r i"."""
    out = []
    for tok in text.split():
        if tok == "i":
            out.append(("i",))
        elif tok == "r":
            out.append(("r",))
        elif tok[0] == "t":
            out.append(("t", int(tok[1:])))
        elif tok[0] == "s":
            out.append(("s", Q(tok[1:])))
        else:
            raise ValueError(f"unknown transformation {tok!r}")
    return out


def apply_transformation_trees(side, lhs, terms, trees):
    """A derived congruence from a transformation graph (Section 7): the
    starting congruence's terms [(c, x, y)] with one tree per term, each tree
    a token list in depth-first order (parse_transformations).  Every node
    transforms its term: tau_d into its d images (x+i)/d, (y+i)/d with the
    coefficient times d^t, sigma_f into (x, x + f(y-x)) and (x + f(y-x), y),
    rho into (1-y, 1-x) with the coefficient times (-1)^t; the leaves (iota)
    are added up.  Coefficients are general-index (Poly).  Returns (the
    congruence, number of leaves)."""
    out = Congruence(side, lhs, general=True)
    refl = SIDES[side][1]
    leaves = 0
    for (c, x, y), toks in zip(terms, trees):
        pos = 0

        def visit(c, x, y):
            nonlocal pos, leaves
            tok = toks[pos]
            pos += 1
            if tok[0] == "i":
                leaves += 1
                out.add(x, y, c)
            elif tok[0] == "r":
                visit(refl * c, 1 - y, 1 - x)
            elif tok[0] == "s":
                z = x + tok[1] * (y - x)
                visit(c, x, z)
                visit(c, z, y)
            else:
                d = tok[1]
                w = c.times_power(d)
                for i in range(d):
                    visit(w, (x + i) / d, (y + i) / d)

        visit(Poly.of(c), Q(x), Q(y))
        if pos != len(toks):
            raise ValueError("tokens left over after the tree")
    return out, leaves


def load_json(obj):
    """A Congruence from to_json output."""
    c = Congruence(obj["side"], int(obj["lhs"]))
    for n, xa, xb, ya, yb in obj["terms"]:
        c.add(Q(xa, xb), Q(ya, yb), Q(int(n)))
    return c


# ---------------------------------------------------------------------------
# searches
# ---------------------------------------------------------------------------

def exhaustive(start, ds):
    """Section 2.1: every sequence of at most len(ds) subdivisions, the i-th
    with 2 <= d <= ds[i].  Returns {m: (cost, steps)} with the cheapest
    congruence found for each number of sums m (first found on ties)."""
    best = {}

    def visit(cong, depth, steps):
        m, cost = cong.n_sums(), cong.cost()
        if m not in best or cost < best[m][0]:
            best[m] = (cost, list(steps))
        if depth == len(ds):
            return
        for c, x, y in cong.pieces():
            for d in range(2, ds[depth] + 1):
                nxt = cong.copy().subdivide(x, y, d)
                steps.append((x, y, d))
                visit(nxt, depth + 1, steps)
                steps.pop()

    visit(start.copy(), 0, [])
    return best


def beam_search(start, D=6, rounds=16, beam=8, max_m=None, log=None):
    """Section 2.1's exhaustive strategy with restarts, as a beam over the
    number of sums: each round applies every single subdivision (d <= D) to
    every congruence kept, merges congruences that coincide, and keeps the
    `beam` cheapest for each number of sums m (at most max_m).  `start` is a
    congruence or a list of them (restart points).  Returns {m: (cost,
    congruence)}, the cheapest seen per m."""
    def key(c):
        return tuple((c2, x, y) for c2, x, y in c.pieces())

    starts = start if isinstance(start, (list, tuple)) else [start]
    best = {}
    for c in starts:
        if c.n_sums() not in best or c.cost() < best[c.n_sums()][0]:
            best[c.n_sums()] = (c.cost(), c)
    frontier = list(starts)
    for r in range(1, rounds + 1):
        seen = {}
        for cong in frontier:
            for c, x, y in cong.pieces():
                for d in range(2, D + 1):
                    nxt = cong.copy().subdivide(x, y, d)
                    m = nxt.n_sums()
                    if max_m is not None and m > max_m:
                        continue
                    k = key(nxt)
                    if k not in seen:
                        seen[k] = nxt
        by_m = {}
        for nxt in seen.values():
            by_m.setdefault(nxt.n_sums(), []).append(nxt)
        frontier = []
        for m, cs in by_m.items():
            cs.sort(key=lambda c: c.cost())
            frontier += cs[:beam]
            if m not in best or cs[0].cost() < best[m][0]:
                best[m] = (cs[0].cost(), cs[0])
        if log:
            log(r, best)
    return best


def greedy(start, D=8, rounds=100, lam=1, log=None, cached=True):
    """Section 2.2: each round tries every sequence of lam subdivisions with
    d <= D and moves to a cheapest result (first in piece order, then d, on
    ties); returns (final congruence, cheapest congruence seen, its round).

    With lam = 1 and cached=True the change of cost of each candidate is kept
    from round to round and recomputed only for the pieces whose value, or
    the value on one of whose images, the last subdivision changed (the
    choices, and so the result, are those of the plain scan, cached=False)."""
    cur = start.copy()
    best, best_round = cur.copy(), 0
    cache = {}   # (x, y) -> (coefficient, least cost_delta(x, y, d) over d = 2..D, first such d)
    for r in range(1, rounds + 1):
        choice = None
        if lam == 1 and cached:
            kept = {}
            for c, x, y in cur.pieces():
                ent = cache.get((x, y))
                if ent is None or ent[0] != c:
                    deltas = [cur.cost_delta(x, y, d) for d in range(2, D + 1)]
                    k = min(range(len(deltas)), key=deltas.__getitem__)   # first smallest d
                    ent = (c, deltas[k], k + 2)
                kept[(x, y)] = ent
                if choice is None or ent[1] < choice[0]:
                    choice = (ent[1], [(x, y, ent[2])])
            cache = kept
        elif lam == 1:
            # the round's candidates differ only in their change of cost
            base = cur.cost()
            for c, x, y in cur.pieces():
                for d in range(2, D + 1):
                    cost = base + cur.cost_delta(x, y, d)
                    if choice is None or cost < choice[0]:
                        choice = (cost, [(x, y, d)])
        else:
            for seq in _sequences(cur, D, lam):
                cand = cur.copy()
                for x, y, d in seq:
                    cand.subdivide(x, y, d)
                if choice is None or cand.cost() < choice[0]:
                    choice = (cand.cost(), seq)
        if choice is None:
            break
        for x, y, d in choice[1]:
            cur.subdivide(x, y, d)
            if lam == 1 and cached:
                _drop_touched(cache, cur, _changed(cur, x, y, d), D)
        if cur.cost() < best.cost():
            best, best_round = cur.copy(), r
        if log:
            log(r, cur)
    return cur, best, best_round


def _changed(cong, x, y, d):
    """Intervals of [0, 1/2] where subdivide(x, y, d) changed the coefficient
    function: the piece and its d images, reflected below 1/2."""
    out = [(x, y)]
    for i in range(d):
        a, b = (x + i) / d, (y + i) / d
        if b <= HALF:
            out.append((a, b))
        elif a >= HALF:
            out.append((1 - b, 1 - a))
        else:
            out.append((a, HALF))
            out.append((1 - b, HALF))
    return out


def _drop_touched(cache, cong, changed, D):
    """Remove the cached candidates whose images by some d <= D meet a changed
    interval.  An image ((x+i)/d, (y+i)/d) lies in (0, 1); it meets a changed
    interval (a, b) of [0, 1/2] directly or through the reflection t -> 1 - t,
    i.e. the piece (x, y) meets (d a - i, d b - i) or (d (1 - b) - i, d (1 - a) - i)."""
    bp, cf = cong.bp, cong.cf
    for a, b in changed:
        for ta, tb in ((a, b), (1 - b, 1 - a)):
            for d in range(2, D + 1):
                for i in range(d):
                    u, v = ta * d - i, tb * d - i
                    if v <= 0 or u >= HALF:
                        continue
                    j = max(bisect_right(bp, u) - 1, 0)
                    while j < len(cf) and bp[j] < v:
                        if cf[j] != 0 and bp[j + 1] > u:
                            cache.pop((bp[j], bp[j + 1]), None)
                        j += 1


def _sequences(cong, D, lam):
    if lam == 0:
        yield []
        return
    for c, x, y in cong.pieces():
        for d in range(2, D + 1):
            nxt = cong.copy().subdivide(x, y, d)
            for rest in _sequences(nxt, D, lam - 1):
                yield [(x, y, d)] + rest


def save_tables(path, tables):
    with open(path, "w") as f:
        json.dump(tables, f, indent=0)
