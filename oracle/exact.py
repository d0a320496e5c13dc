"""Exact rational and integer arithmetic for tiny primes (oracle, test infrastructure only).

Written from the definitions in Section 1 of the paper (Booker, Hathi,
Mossinghoff, Trudgian, arXiv:2101.11157):

* Bernoulli numbers by their EGF  z/(e^z - 1) = sum B_k z^k/k!.
* Euler numbers by their EGF  sec z = sum E_k z^k/k!  (secant convention; the
  footnote there notes that the hyperbolic-secant convention flips the sign
  of indices 2 mod 4).
* Glaisher's congruence (eqnGlaisher): binom(hp-1, p-1) == 1 - h(h-1)/3 p^3 B_{p-3}
  (mod p^4) for p >= 5.

Python integers and fractions.Fraction only; nothing here is fast.
"""
from fractions import Fraction
from math import comb, factorial

__all__ = [
    "bernoulli_egf", "bernoulli_recurrence", "euler_egf", "euler_recurrence",
    "rational_mod_p", "b_mod_p", "e_mod_p", "glaisher_b_mod_p", "symmetric",
]


def _series_reciprocal(a, n):
    """Coefficients 0..n of 1/A(z) for a power series A with a[0] != 0."""
    inv = [Fraction(0)] * (n + 1)
    inv[0] = Fraction(1) / a[0]
    for k in range(1, n + 1):
        acc = Fraction(0)
        for j in range(1, k + 1):
            if j < len(a) and a[j] != 0:
                acc += a[j] * inv[k - j]
        inv[k] = -acc / a[0]
    return inv


def bernoulli_egf(n):
    """B_0..B_n from the EGF: z/(e^z-1) = 1 / sum_{j>=0} z^j/(j+1)!."""
    a = [Fraction(1, factorial(j + 1)) for j in range(n + 1)]
    inv = _series_reciprocal(a, n)
    return [inv[k] * factorial(k) for k in range(n + 1)]


def bernoulli_recurrence(n):
    """B_0..B_n from sum_{j=0}^{m} C(m+1, j) B_j = 0 for m >= 1 (B_0 = 1)."""
    B = [Fraction(0)] * (n + 1)
    B[0] = Fraction(1)
    for m in range(1, n + 1):
        B[m] = -sum(comb(m + 1, j) * B[j] for j in range(m)) / (m + 1)
    return B


def euler_egf(n):
    """E_0..E_n from the EGF sec z = 1/cos z."""
    a = [Fraction(0)] * (n + 1)
    for j in range(0, n + 1, 2):
        a[j] = Fraction((-1) ** (j // 2), factorial(j))
    inv = _series_reciprocal(a, n)
    return [inv[k] * factorial(k) for k in range(n + 1)]


def euler_recurrence(n):
    """E_0..E_n (integers) from sec z cos z = 1:
    sum_{j=0}^{floor(m/2)} (-1)^j C(m, 2j) E_{m-2j} = 0 for m >= 1."""
    E = [0] * (n + 1)
    E[0] = 1
    for m in range(1, n + 1):
        E[m] = -sum((-1) ** j * comb(m, 2 * j) * E[m - 2 * j] for j in range(1, m // 2 + 1))
    return E


def rational_mod_p(x, p):
    """Residue of the rational x mod p (p must not divide the denominator)."""
    x = Fraction(x)
    if x.denominator % p == 0:
        raise ZeroDivisionError(f"{p} divides the denominator")
    return x.numerator * pow(x.denominator, -1, p) % p


def b_mod_p(p, _cache={}):
    """B_{p-3} mod p, exactly (for small p)."""
    n = p - 3
    if n not in _cache:
        _cache[n] = bernoulli_recurrence(n)[n]
    return rational_mod_p(_cache[n], p)


def e_mod_p(p):
    """E_{p-3} mod p, exactly (for small p)."""
    return euler_recurrence(p - 3)[p - 3] % p


def glaisher_b_mod_p(p, h=2):
    """B_{p-3} mod p from eqnGlaisher with integer h >= 2, p >= 5, p not dividing h(h-1)/3's numerator:
    binom(hp-1, p-1) - 1 == -h(h-1)/3 * p^3 * B_{p-3}  (mod p^4)."""
    p4 = p ** 4
    d = (comb(h * p - 1, p - 1) - 1) % p4
    if d % p ** 3 != 0:
        raise ArithmeticError("binom(hp-1,p-1) != 1 mod p^3 (Wolstenholme's congruence fails?)")
    q = (d // p ** 3) % p                      # == -h(h-1)/3 * B_{p-3} mod p
    return q * rational_mod_p(Fraction(-3, h * (h - 1)), p) % p


def symmetric(r, p):
    """The representative of r mod p in (-p/2, p/2] (Section 3, notation for Table 2)."""
    r %= p
    return r - p if 2 * r > p else r
