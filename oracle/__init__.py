"""Plain CPU oracle for B_{p-3} mod p and E_{p-3} mod p.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code, header, table or constant with the HIP product path
(``paper_2101_11157_amd``) and never imports it.

Layers (all cite Booker, Hathi, Mossinghoff, Trudgian, arXiv:2101.11157):

* ``exact``        -- Python rationals: Bernoulli/Euler numbers from their EGFs
                      (Section 1) and Glaisher's congruence (eqnGlaisher).
* ``congruences``  -- the paper's congruences typed in as data (Sections 2-5).
* ``wv_oracle.c``  -- C with unsigned __int128 and ``%``: the sums S_l(x,y) of
                      eqnDefnS, directly or by eqnComputeS, the recurrences mod p
                      (B_{p-3}, E_{p-3}, and every B_{2k}, E_{2k} with 2k <= p-3 for
                      irregular pairs), harmonic sums mod p^2 and a plain sieve.

The reference answer for a prime p (``residues``):

* p in {5, 7} and p < 2000: the recurrences implied by the EGFs, run mod p;
* otherwise ``method="root"``: Stafford-Vandiver (eqnSV at k=(p-3)/2, i.e. eqnBB1)
  for B and Glaisher's eqnE1 (sign read as (-1)^k) for E;
  ``method="table"``: the printed eqnBB30 / eqnEE33, evaluated plainly.

Where the paper is ambiguous this oracle takes one reading; the one that
changes a formula is the sign of eqnE1 (read as (-1)^k, which Table 3's
printed residues confirm).
"""
import ctypes
import os
import subprocess
from fractions import Fraction

from . import congruences, exact  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wv_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lib = None

U64 = ctypes.c_uint64
P_U64 = ctypes.POINTER(ctypes.c_uint64)
P_I64 = ctypes.POINTER(ctypes.c_int64)


def build(force=True):
    """Compile wv_oracle.c with gcc -O2 -fopenmp into oracle/_build/liboracle.so."""
    os.makedirs(_BUILD, exist_ok=True)
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_invmod.restype = U64
        L.orc_invmod.argtypes = [U64, U64]
        L.orc_interval.restype = None
        L.orc_interval.argtypes = [U64, U64, U64, U64, U64, P_U64, P_U64]
        L.orc_sum_direct.restype = U64
        L.orc_sum_direct.argtypes = [U64, U64, U64, ctypes.c_int, ctypes.c_int]
        L.orc_sum_poly_pair.restype = None
        L.orc_sum_poly_pair.argtypes = [U64, U64, U64, ctypes.c_int, ctypes.c_int, P_U64, P_U64]
        L.orc_sum_poly.restype = U64
        L.orc_sum_poly.argtypes = [U64, U64, U64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_congruence.restype = U64
        L.orc_congruence.argtypes = [U64, ctypes.c_int, P_I64, P_U64, P_U64, P_U64, P_U64,
                                     ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int]
        L.orc_congruence_many.restype = None
        L.orc_congruence_many.argtypes = [P_U64, ctypes.c_size_t, ctypes.c_int, P_I64, P_U64, P_U64,
                                          P_U64, P_U64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, P_U64]
        L.orc_bernoulli_rec.restype = U64
        L.orc_bernoulli_rec.argtypes = [U64]
        L.orc_euler_rec.restype = U64
        L.orc_euler_rec.argtypes = [U64]
        L.orc_bernoulli_all.restype = None
        L.orc_bernoulli_all.argtypes = [U64, P_U64]
        L.orc_euler_all.restype = None
        L.orc_euler_all.argtypes = [U64, P_U64]
        L.orc_harmonic2_mod_p2.restype = U64
        L.orc_harmonic2_mod_p2.argtypes = [U64]
        L.orc_harmonic1_mod_p2.restype = U64
        L.orc_harmonic1_mod_p2.argtypes = [U64]
        L.orc_primes.restype = U64
        L.orc_primes.argtypes = [U64, U64, P_U64, U64]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def max_threads():
    return lib().orc_max_threads()


def _arr(t, vals):
    return (t * max(1, len(vals)))(*vals)


# ---------------------------------------------------------------------------
# Sums and congruences
# ---------------------------------------------------------------------------

def interval(p, x, y):
    """(lo, hi) of the open interval x*p < s < y*p (eqnDefnS); lo > hi when empty."""
    x, y = Fraction(x), Fraction(y)
    lo, hi = U64(), U64()
    lib().orc_interval(p, x.numerator, x.denominator, y.numerator, y.denominator,
                       ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def sum_direct(p, lo, hi, ell, alt=False):
    """sum_{s=lo}^{hi} (+-1)^s s^-ell mod p, one inverse per term."""
    return lib().orc_sum_direct(p, lo, hi, ell, int(alt))


def sum_poly_pair(p, lo, hi, ell, alt=False):
    """(c0, c1) of prod_{s=lo}^{hi} (z + (+-1)^s s^ell) mod (p, z^2) (eqnComputeS)."""
    c0, c1 = U64(), U64()
    lib().orc_sum_poly_pair(p, lo, hi, ell, int(alt), ctypes.byref(c0), ctypes.byref(c1))
    return c0.value, c1.value


def sum_poly(p, lo, hi, ell, alt=False, nthreads=1):
    """sum (+-1)^s s^-ell by eqnComputeS (c1/c0), split over threads."""
    return lib().orc_sum_poly(p, lo, hi, ell, int(alt), nthreads)


def _congruence_arrays(cong):
    n = len(cong.terms)
    coef = _arr(ctypes.c_int64, [c for c, _, _ in cong.terms])
    xa = _arr(U64, [x.numerator for _, x, _ in cong.terms])
    xb = _arr(U64, [x.denominator for _, x, _ in cong.terms])
    ya = _arr(U64, [y.numerator for _, _, y in cong.terms])
    yb = _arr(U64, [y.denominator for _, _, y in cong.terms])
    return n, coef, xa, xb, ya, yb


def congruence_residue(p, cong, method="poly", nthreads=1):
    """X_{p-3} mod p from one congruence (None if its left side vanishes mod p)."""
    if isinstance(cong, str):
        cong = congruences.table(cong)
    n, coef, xa, xb, ya, yb = _congruence_arrays(cong)
    r = lib().orc_congruence(p, n, coef, xa, xb, ya, yb, cong.lhs, -cong.ell, int(cong.alt),
                             0 if method == "direct" else 1, nthreads)
    return None if r == 2 ** 64 - 1 else r


def congruence_residue_exact(p, cong, nthreads=1):
    """lhs^-1 * sum_i c_i S(x_i, y_i) mod p (Section 2, eqnDefnS) for a
    congruence whose integers and endpoints may have any size (derived
    congruences): endpoints by exact integer floors of the open interval,
    coefficients reduced mod p, each sum by eqnComputeS (orc_sum_poly).
    None when p divides the left side."""
    L = cong.lhs % p
    if L == 0:
        return None
    acc = 0
    for c, x, y in cong.terms:
        lo = x.numerator * p // x.denominator + 1
        hi = (y.numerator * p - 1) // y.denominator
        if hi < lo:
            continue
        acc = (acc + (c % p) * sum_poly(p, lo, hi, -cong.ell, cong.alt, nthreads=nthreads)) % p
    return acc * pow(L, -1, p) % p


def congruence_residues(primes, cong, method="poly", nthreads=None):
    """congruence_residue over a list of primes, one prime per thread."""
    if isinstance(cong, str):
        cong = congruences.table(cong)
    primes = [int(q) for q in primes]
    if not primes:
        return []
    nthreads = nthreads or max_threads()
    n, coef, xa, xb, ya, yb = _congruence_arrays(cong)
    parr = _arr(U64, primes)
    out = (U64 * len(primes))()
    lib().orc_congruence_many(parr, len(primes), n, coef, xa, xb, ya, yb, cong.lhs, -cong.ell,
                              int(cong.alt), 0 if method == "direct" else 1, nthreads, out)
    res = list(out)
    return [None if r == 2 ** 64 - 1 else r for r in res]


# ---------------------------------------------------------------------------
# Recurrences, harmonic sums, sieve
# ---------------------------------------------------------------------------

def bernoulli_rec(p):
    """B_{p-3} mod p from the EGF recurrence run in F_p (O(p^2))."""
    return lib().orc_bernoulli_rec(p)


def euler_rec(p):
    """E_{p-3} mod p from sec*cos = 1 run in F_p (O(p^2))."""
    return lib().orc_euler_rec(p)


def bernoulli_all(p):
    """[B_2, B_4, ..., B_{p-3}] mod p from the EGF recurrence in F_p (O(p^2))."""
    n = (p - 3) // 2
    out = (ctypes.c_uint64 * max(n, 1))()
    lib().orc_bernoulli_all(p, out)
    return [int(v) for v in out[:n]]


def euler_all(p):
    """[E_2, E_4, ..., E_{p-3}] mod p from sec*cos = 1 in F_p (O(p^2))."""
    n = (p - 3) // 2
    out = (ctypes.c_uint64 * max(n, 1))()
    lib().orc_euler_all(p, out)
    return [int(v) for v in out[:n]]


def irregular_pairs(p):
    """Irregular pairs (p, 2k) (p | B_{2k}) and E-irregular pairs (p | E_{2k})
    with 2 <= 2k <= p - 3 (Section 1): sorted (p, 2k, kind), kind 1 for B,
    2 for E."""
    b, e = bernoulli_all(p), euler_all(p)
    out = []
    for k in range(1, len(b) + 1):
        if b[k - 1] == 0:
            out.append((p, 2 * k, 1))
        if e[k - 1] == 0:
            out.append((p, 2 * k, 2))
    return out


def harmonic2_mod_p2(p):
    return lib().orc_harmonic2_mod_p2(p)


def harmonic1_mod_p2(p):
    return lib().orc_harmonic1_mod_p2(p)


def b_from_harmonic(p):
    """B_{p-3} mod p from H = sum_{0<k<p} k^-2 mod p^2 via the classical
    H == (2/3) p B_{p-3} (mod p^2) (Glaisher).  The factor 2/3 is not stated in
    the paper, which uses only H == 0 mod p^2 <=> Wolstenholme (eqnWolst); it is
    pinned in the tests against the recurrence and eqnGlaisher."""
    H = harmonic2_mod_p2(p)
    if H % p:
        raise ArithmeticError("sum k^-2 != 0 mod p")
    return (H // p) * 3 * pow(2, -1, p) % p


def primes(lo, hi):
    """All primes in [lo, hi) by a plain sieve."""
    n = lib().orc_primes(lo, hi, None, 0)
    out = (U64 * max(1, n))()
    lib().orc_primes(lo, hi, out, n)
    return list(out)[:n]


# ---------------------------------------------------------------------------
# Reference residues
# ---------------------------------------------------------------------------

SMALL_P = 2000


def residues(primes_list, method="root", nthreads=None):
    """[(b, e)] with b = B_{p-3} mod p, e = E_{p-3} mod p for each prime p >= 5.

    p < 2000 -> recurrences; else method 'root' (eqnBB1 and eqnE1) or 'table'
    (eqnBB30 and eqnEE33)."""
    primes_list = [int(q) for q in primes_list]
    out = [None] * len(primes_list)
    big = [(i, q) for i, q in enumerate(primes_list) if q >= SMALL_P]
    for i, q in enumerate(primes_list):
        if q < 5:
            raise ValueError("p must be >= 5")
        if q < SMALL_P:
            out[i] = (bernoulli_rec(q), euler_rec(q))
    if big:
        qs = [q for _, q in big]
        if method == "root":
            bs = congruence_residues(qs, congruences.SV, nthreads=nthreads)
            es = congruence_residues(qs, congruences.E1, nthreads=nthreads)
        elif method == "table":
            bs = congruence_residues(qs, congruences.BB30, nthreads=nthreads)
            es = congruence_residues(qs, congruences.EE33, nthreads=nthreads)
        else:
            raise ValueError(method)
        for (i, _), b, e in zip(big, bs, es):
            out[i] = (b, e)
    return out


def residue_one_parallel(p, method="table", nthreads=None):
    """(b, e) for one large prime, each sum's range split over threads."""
    nthreads = nthreads or max_threads()
    if method == "table":
        cb, ce = congruences.BB30, congruences.EE33
    else:
        cb, ce = congruences.SV, congruences.E1
    return (congruence_residue(p, cb, nthreads=nthreads),
            congruence_residue(p, ce, nthreads=nthreads))


# ---------------------------------------------------------------------------
# Residue statistics (results of Sections 3 and 5)
# ---------------------------------------------------------------------------

def residue_stats(rows, bins=2000, bound=50):
    """Histograms and near misses of a list of (p, b, e) residues.

    The histograms of Sections 3 and 5 use `bins` equal bins of <r>_p / p over
    (-1/2, 1/2]; a value falls in bin k when -1/2 + k/bins <= <r>_p/p <
    -1/2 + (k+1)/bins, i.e. k = floor((<r>_p/p + 1/2) bins), computed here with
    exact rationals.  Near misses (Tables 2 and 3): |<r>_p| < bound, as
    (p, <r>_p, which) with which 1 for B_{p-3}, 2 for E_{p-3}, ordered by p,
    then which.
    """
    hist = [[0] * bins, [0] * bins]
    near = []
    for p, b, e in rows:
        for w, r in enumerate((b, e)):
            s = exact.symmetric(r, p)
            k = int((Fraction(s, p) + Fraction(1, 2)) * bins // 1)
            hist[w][k] += 1
            if abs(s) < bound:
                near.append((p, s, w + 1))
    return hist[0], hist[1], sorted(near, key=lambda t: (t[0], t[2]))
