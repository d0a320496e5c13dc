"""wvprime: B_{p-3} mod p and E_{p-3} mod p on an AMD MI355X.

A thin ctypes binding over ``libwvprime.so`` (C ABI in ``include/wvprime.h``);
every step of the computation runs in the library's HIP kernels.  The binding
only marshals arguments.  Importing this package does not load the library:
the first call that needs it does, and raises ``WvError`` when the built
library is missing (build it with ``paper_2101_11157_amd.build.build()``).

Method: Booker, Hathi, Mossinghoff, Trudgian, "Wolstenholme and Vandiver
primes", arXiv:2101.11157 -- specialised congruences (Sections 3 and 5) whose
sums of s^-3 / s^-2 are evaluated as c1/c0 of prod(z + s^k) (eqnComputeS).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwvprime.so")

WV_OK = 0
WV_EINVAL = -1
WV_EDOMAIN = -2
WV_ENOTPRIME = -3
WV_ETRUNC = -4
WV_ENOMEM = -5
WV_EHIP = -6
WV_EBUSY = -7
WV_P_MAX = 1 << 40
WV_FLAG_WOLSTENHOLME = 1
WV_FLAG_VANDIVER = 2

TABLE_NAMES = ["BB1", "BB2", "BB6", "BB9", "BB16", "BB22", "BB30",
               "EE3", "EE5", "EE9", "EE16", "EE24", "EE33", "V12", "E1"]
TABLE_ID = {n: i for i, n in enumerate(TABLE_NAMES)}
# derived congruences shipped with the package (tables/make_tables.py): for
# each side a ladder of congruences from one greedy search, each serving the
# primes from its min_p up to the next one's (tables/ladder.json)
DERIVED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")


def _load_table(name):
    import gzip
    import json
    path = os.path.join(DERIVED_DIR, name)
    with (gzip.open(path, "rt") if name.endswith(".gz") else open(path)) as f:
        return json.load(f)


def derived_ladder(side):
    """[{"rounds", "min_p", "file", "n", "cost"}] of the shipped congruences of
    one side ('B' or 'E'), ascending in min_p (and so in rounds)."""
    return _load_table("ladder.json")[side]


def derived_min_p():
    """Smallest prime any shipped derived congruence serves (below it: the
    printed eqnBB30 / eqnEE33)."""
    return min(r["min_p"] for side in "BE" for r in derived_ladder(side))


def derived_table(side, rounds=None):
    """The JSON congruence of one rung of the ladder (default: the top one,
    the most rounds, used for the largest primes)."""
    rungs = derived_ladder(side)
    r = rungs[-1] if rounds is None else next(r for r in rungs if r["rounds"] == rounds)
    return _load_table(r["file"])


def _frac(a, b):
    from fractions import Fraction
    return Fraction(int(a), int(b))


# compiled block shapes of the term-sum kernel, in the library's order
BLOCK_SHAPES = [(1, 1), (4, 4), (8, 8), (12, 16), (16, 24), (20, 28), (24, 32), (26, 34), (28, 32), (28, 36)]

# wv_irr_pair as a numpy record (16 bytes)
IRR_PAIR_DTYPE = np.dtype([("p", "<u8"), ("two_k", "<u4"), ("kind", "<u4")])
IRR_P_MAX = 1 << 27

# wv_result as a numpy record (32 bytes)
RESULT_DTYPE = np.dtype([("p", "<u8"), ("b", "<u8"), ("e", "<u8"), ("flags", "<u4"), ("reserved", "<u4")])
# wv_near (24 bytes): a prime with a small symmetric residue; which = 1 (B) or 2 (E)
NEAR_DTYPE = np.dtype([("p", "<u8"), ("r", "<i8"), ("which", "<u4"), ("reserved", "<u4")])
NEAR_B, NEAR_E = 1, 2
MAX_BINS = 65536


class WvStats(ctypes.Structure):
    _fields_ = [
        ("ms_total", ctypes.c_double), ("ms_sieve", ctypes.c_double), ("ms_plan", ctypes.c_double),
        ("ms_sum", ctypes.c_double), ("ms_reduce", ctypes.c_double), ("ms_finalize", ctypes.c_double),
        ("n_primes", ctypes.c_uint64), ("n_sums", ctypes.c_uint64), ("n_chunks", ctypes.c_uint64),
        ("n_terms", ctypes.c_uint64), ("n_terms_b", ctypes.c_uint64), ("chunk_terms", ctypes.c_uint64),
        ("block_k_b", ctypes.c_uint32), ("block_k_e", ctypes.c_uint32), ("grid", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class WvServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("pending", ctypes.c_uint64),
        ("active", ctypes.c_uint64), ("primes_done", ctypes.c_uint64), ("terms_done", ctypes.c_uint64),
        ("steps", ctypes.c_uint64), ("readmits", ctypes.c_uint64),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
        ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double), ("wall_s", ctypes.c_double),
        ("failed", ctypes.c_uint64), ("terms_done_b", ctypes.c_uint64), ("sum_s", ctypes.c_double),
        ("block_k_b", ctypes.c_uint32), ("block_k_e", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class WvServerConfig(ctypes.Structure):
    _fields_ = [("step_terms", ctypes.c_uint64), ("max_primes", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)


class WvError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = _strerror(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


_lib = None
U64 = ctypes.c_uint64
P_U64 = ctypes.POINTER(ctypes.c_uint64)
VP = ctypes.c_void_p
SZ = ctypes.c_size_t


def lib():
    """The loaded C library (raises WvError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise WvError(WV_EHIP, f"{LIB_PATH} not built; run paper_2101_11157_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "wv_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "wv_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(VP)]),
            "wv_destroy": (ctypes.c_int, [VP]),
            "wv_set_tables": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int]),
            "wv_set_chunk_terms": (ctypes.c_int, [VP, U64]),
            "wv_set_block": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int]),
            "wv_count_primes": (ctypes.c_int, [VP, U64, U64, P_U64]),
            "wv_search_range": (ctypes.c_int, [VP, U64, U64, VP, SZ, ctypes.POINTER(SZ), P_U64, SZ,
                                               ctypes.POINTER(SZ)]),
            "wv_eval_primes": (ctypes.c_int, [VP, P_U64, SZ, VP]),
            "wv_eval_primes_async": (ctypes.c_int, [VP, VP, SZ, VP, VP]),
            "wv_eval_primes_static": (ctypes.c_int, [VP, VP, SZ, VP, VP]),
            "wv_eval_sums": (ctypes.c_int, [VP, P_U64, SZ, P_U64, P_U64]),
            "wv_search_windows": (ctypes.c_int, [VP, P_U64, P_U64, SZ, VP, SZ, ctypes.POINTER(SZ),
                                                 ctypes.POINTER(SZ)]),
            "wv_set_progress": (ctypes.c_int, [VP, PROGRESS_FN, VP, U64]),
            "wv_define_table": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_char_p, SZ, ctypes.POINTER(ctypes.c_char_p),
                                               P_U64, P_U64, P_U64, P_U64, U64, ctypes.POINTER(ctypes.c_int)]),
            "wv_set_table_below": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int]),
            "wv_range_stats": (ctypes.c_int, [VP, U64, U64, ctypes.c_uint32, U64, P_U64, P_U64, VP, SZ,
                                              ctypes.POINTER(SZ), P_U64]),
            "wv_bernoulli_euler_all": (ctypes.c_int, [VP, U64, P_U64, P_U64]),
            "wv_set_irregular_path": (ctypes.c_int, [VP, ctypes.c_int]),
            "wv_irregular_pairs": (ctypes.c_int, [VP, U64, U64, VP, SZ, ctypes.POINTER(SZ), P_U64, P_U64]),
            "wv_autotune": (ctypes.c_int, [VP, U64, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), P_U64, ctypes.POINTER(ctypes.c_double)]),
            "wv_tune_save": (ctypes.c_int, [VP, ctypes.c_char_p]),
            "wv_tune_load": (ctypes.c_int, [VP, ctypes.c_char_p]),
            "wv_server_create": (ctypes.c_int, [VP, ctypes.POINTER(WvServerConfig), ctypes.POINTER(VP)]),
            "wv_server_destroy": (ctypes.c_int, [VP]),
            "wv_server_submit_range": (ctypes.c_int, [VP, U64, U64, P_U64]),
            "wv_server_submit_primes": (ctypes.c_int, [VP, P_U64, SZ, P_U64]),
            "wv_server_step": (ctypes.c_int, [VP, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
            "wv_server_result": (ctypes.c_int, [VP, U64, VP, SZ, ctypes.POINTER(SZ),
                                                ctypes.POINTER(ctypes.c_double)]),
            "wv_server_get_stats": (ctypes.c_int, [VP, ctypes.POINTER(WvServerStats)]),
            "wv_server_inject_fault": (ctypes.c_int, [VP, ctypes.c_int]),
            "wv_get_stats": (ctypes.c_int, [VP, ctypes.POINTER(WvStats)]),
            "wv_table_info": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int64), P_U64, P_U64]),
            "wv_table_term": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(status):
    return lib().wv_strerror(status).decode()


def _check(status, what):
    if status != WV_OK:
        raise WvError(status, what)


def table_info(name_or_id):
    """(n_sums, lhs, cost_num, cost_den) of a congruence compiled into the library."""
    i = TABLE_ID[name_or_id] if isinstance(name_or_id, str) else int(name_or_id)
    n = ctypes.c_int()
    lhs = ctypes.c_int64()
    cn, cd = U64(), U64()
    _check(lib().wv_table_info(i, ctypes.byref(n), ctypes.byref(lhs), ctypes.byref(cn), ctypes.byref(cd)),
           "wv_table_info")
    return n.value, lhs.value, cn.value, cd.value


def table_terms(name_or_id):
    """[(coef, xa, xb, ya, yb)] of a congruence compiled into the library."""
    i = TABLE_ID[name_or_id] if isinstance(name_or_id, str) else int(name_or_id)
    n = table_info(i)[0]
    out = []
    for j in range(n):
        c = ctypes.c_int64()
        v = [ctypes.c_uint32() for _ in range(4)]
        _check(lib().wv_table_term(i, j, ctypes.byref(c), *[ctypes.byref(x) for x in v]), "wv_table_term")
        out.append((c.value, *[x.value for x in v]))
    return out


def prime_count_bound(lo, hi):
    """An upper bound on the number of primes in [lo, hi), for sizing output
    buffers: the odd numbers there, pi(x) < 1.25506 x / log x (Rosser and
    Schoenfeld) for the count below hi, and pi(x + y) - pi(x) <= 2 y / log y
    (Montgomery and Vaughan) for an interval of length y > 1."""
    import math
    lo, hi = int(lo), int(hi)
    if hi <= lo:
        return 0
    y = hi - lo
    bound = y // 2 + 2
    if hi > 17:
        bound = min(bound, int(1.25506 * hi / math.log(hi)) + 2)
    if y > 1:
        bound = min(bound, int(2 * y / math.log(y)) + 2)
    return bound


def symmetric(r, p):
    """Representative of r mod p in (-p/2, p/2]."""
    r = int(r) % int(p)
    return r - int(p) if r > (int(p) - 1) // 2 else r


class Context:
    """One wv_ctx: device buffers, a HIP stream and tuning state on one GPU."""

    def __init__(self, device=0):
        h = VP()
        _check(lib().wv_create(int(device), ctypes.byref(h)), "wv_create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().wv_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def set_tables(self, b_table="BB30", e_table="EE33"):
        b = TABLE_ID[b_table] if isinstance(b_table, str) else int(b_table)
        e = TABLE_ID[e_table] if isinstance(e_table, str) else int(e_table)
        _check(lib().wv_set_tables(self._h, b, e), "wv_set_tables")

    def define_table(self, deg, lhs, terms, min_p=11):
        """Register  lhs * X_{p-3} == sum c S(x, y)  (terms: (c, x, y) with
        integer c and fractions 0 <= x < y <= 1; deg 3: X = B, 2: X = E) for
        primes p >= min_p; returns the table id for set_tables."""
        from fractions import Fraction
        n = len(terms)
        coef = (ctypes.c_char_p * n)(*[str(int(c)).encode() for c, _, _ in terms])
        xs = [Fraction(x) for _, x, _ in terms]
        ys = [Fraction(y) for _, _, y in terms]
        arr = lambda v: np.ascontiguousarray(np.array(v, dtype=np.uint64))
        xa, xb = arr([x.numerator for x in xs]), arr([x.denominator for x in xs])
        ya, yb = arr([y.numerator for y in ys]), arr([y.denominator for y in ys])
        out = ctypes.c_int()
        _check(lib().wv_define_table(self._h, int(deg), str(int(lhs)).encode(), n, coef, xa.ctypes.data_as(P_U64),
                                     xb.ctypes.data_as(P_U64), ya.ctypes.data_as(P_U64), yb.ctypes.data_as(P_U64),
                                     int(min_p), ctypes.byref(out)), "wv_define_table")
        return out.value

    def define_derived_table(self, obj, min_p=None):
        """Register a congruence written by derive.Congruence.to_json (for
        primes >= min_p; default: the smallest prime the shipped ladder serves)."""
        terms = [(int(n), _frac(xa, xb), _frac(ya, yb)) for n, xa, xb, ya, yb in obj["terms"]]
        return self.define_table(3 if obj["side"] == "B" else 2, int(obj["lhs"]), terms,
                                 derived_min_p() if min_p is None else min_p)

    def set_table_below(self, table, below):
        """Primes a defined table does not serve (below its min_p, or dividing
        its left side) use `below` (a name or id)."""
        below = TABLE_ID[below] if isinstance(below, str) else int(below)
        _check(lib().wv_set_table_below(self._h, int(table), below), "wv_set_table_below")

    def use_derived_tables(self, min_p=None, top=None):
        """Define the shipped ladders of derived congruences (tables/ladder.json,
        built by tables/make_tables.py with the greedy search of Section 2.2)
        and use them: each rung serves the primes from its min_p up to the next
        rung's, the lowest from min_p when given (else its own), and the
        printed eqnBB30 / eqnEE33 the primes below.  top: use only the rungs
        of at most this many rounds.  Each rung is one defined table of the
        context's 64 (about 30 in all).  Returns (b_id, e_id) of the top
        rungs."""
        ids = []
        for side in "BE":
            rungs = [r for r in derived_ladder(side) if top is None or r["rounds"] <= top]
            if min_p is not None:
                # rungs that would serve only primes below min_p are left out
                rungs = [r for k, r in enumerate(rungs) if k + 1 == len(rungs) or rungs[k + 1]["min_p"] > int(min_p)]
            if not rungs:
                raise ValueError(f"no shipped {side} congruence of at most {top} rounds")
            below = "BB30" if side == "B" else "EE33"
            for k, r in enumerate(rungs):
                lo = r["min_p"] if (k > 0 or min_p is None) else int(min_p)
                t = self.define_derived_table(_load_table(r["file"]), lo)
                self.set_table_below(t, below)
                below = t
            ids.append(below)
        b, e = ids
        self.set_tables(b, e)
        return b, e

    def set_chunk_terms(self, n):
        _check(lib().wv_set_chunk_terms(self._h, int(n)), "wv_set_chunk_terms")

    def set_block(self, kb, ke):
        _check(lib().wv_set_block(self._h, int(kb), int(ke)), "wv_set_block")

    def count_primes(self, lo, hi):
        n = U64()
        _check(lib().wv_count_primes(self._h, int(lo), int(hi), ctypes.byref(n)), "wv_count_primes")
        return n.value

    def search_range(self, lo, hi, cap=None, hit_cap=1024):
        """Results (numpy RESULT_DTYPE, ascending p) and the hit list for [lo, hi).
        The output buffer is sized from an upper bound on the number of primes
        (a short buffer costs a second call, which the library reports with
        WV_ETRUNC before doing any work).  An explicit `cap` that is too short
        raises WvError(WV_ETRUNC)."""
        auto = cap is None
        if auto:
            cap = prime_count_bound(lo, hi)
        while True:
            out = np.zeros(max(1, cap), dtype=RESULT_DTYPE)
            hits = np.zeros(max(1, hit_cap), dtype=np.uint64)
            n_out, n_hits = SZ(), SZ()
            st = lib().wv_search_range(self._h, int(lo), int(hi), out.ctypes.data_as(VP), cap, ctypes.byref(n_out),
                                       hits.ctypes.data_as(P_U64), hit_cap, ctypes.byref(n_hits))
            if auto and st == WV_ETRUNC and n_out.value > cap:
                cap = n_out.value
                continue
            _check(st, "wv_search_range")
            return out[:n_out.value], hits[:min(n_hits.value, hit_cap)]

    def eval_primes(self, primes):
        """Results (numpy RESULT_DTYPE) for the given primes, input order."""
        arr = np.ascontiguousarray(np.asarray(primes, dtype=np.uint64))
        out = np.zeros(max(1, arr.size), dtype=RESULT_DTYPE)
        st = lib().wv_eval_primes(self._h, arr.ctypes.data_as(P_U64), arr.size, out.ctypes.data_as(VP))
        _check(st, "wv_eval_primes")
        return out[:arr.size]

    def search_windows(self, los, his):
        """Batched search: list of per-window result arrays (ascending p in each)."""
        lo = np.ascontiguousarray(np.asarray(los, dtype=np.uint64))
        hi = np.ascontiguousarray(np.asarray(his, dtype=np.uint64))
        n_out = SZ()
        offs = (SZ * (lo.size + 1))()
        st = lib().wv_search_windows(self._h, lo.ctypes.data_as(P_U64), hi.ctypes.data_as(P_U64), lo.size, None, 0,
                                     ctypes.byref(n_out), offs)
        if st not in (WV_OK, WV_ETRUNC):
            _check(st, "wv_search_windows")
        out = np.zeros(max(1, n_out.value), dtype=RESULT_DTYPE)
        st = lib().wv_search_windows(self._h, lo.ctypes.data_as(P_U64), hi.ctypes.data_as(P_U64), lo.size,
                                     out.ctypes.data_as(VP), n_out.value, ctypes.byref(n_out), offs)
        _check(st, "wv_search_windows")
        return [out[offs[w]:offs[w + 1]] for w in range(lo.size)]

    def range_stats(self, lo, hi, bins=2000, near=50, near_cap=4096):
        """Residue statistics of [lo, hi) computed on the device: (hist_b,
        hist_e, near misses (NEAR_DTYPE, sorted by p then which), n_primes).
        Bin k of the symmetric residue s counts floor((s/p + 1/2) bins) == k."""
        hb = np.zeros(bins, dtype=np.uint64)
        he = np.zeros(bins, dtype=np.uint64)
        nr = np.zeros(max(1, near_cap), dtype=NEAR_DTYPE)
        n_near, n_primes = SZ(), U64()
        st = lib().wv_range_stats(self._h, int(lo), int(hi), int(bins), int(near), hb.ctypes.data_as(P_U64),
                                  he.ctypes.data_as(P_U64), nr.ctypes.data_as(VP), near_cap, ctypes.byref(n_near),
                                  ctypes.byref(n_primes))
        if st == WV_ETRUNC:
            nr = np.zeros(n_near.value, dtype=NEAR_DTYPE)
            st = lib().wv_range_stats(self._h, int(lo), int(hi), int(bins), int(near), hb.ctypes.data_as(P_U64),
                                      he.ctypes.data_as(P_U64), nr.ctypes.data_as(VP), n_near.value,
                                      ctypes.byref(n_near), ctypes.byref(n_primes))
        _check(st, "wv_range_stats")
        return hb, he, nr[:n_near.value], n_primes.value

    def set_irregular_path(self, path):
        """Power-sum kernel of the irregular-pair calls: 0 automatic, 1 vector
        ALU, 2 matrix cores where exact (p < 2^24)."""
        _check(lib().wv_set_irregular_path(self._h, int(path)), "wv_set_irregular_path")

    def bernoulli_euler_all(self, p):
        """(b, e): B_{2k} mod p and E_{2k} mod p for 2k = 2, 4, ..., p - 3
        (uint64 arrays indexed by k - 1), from the general-index congruences."""
        n = (int(p) - 3) // 2
        b = np.zeros(max(n, 1), dtype=np.uint64)
        e = np.zeros(max(n, 1), dtype=np.uint64)
        _check(lib().wv_bernoulli_euler_all(self._h, int(p), b.ctypes.data_as(P_U64), e.ctypes.data_as(P_U64)),
               "wv_bernoulli_euler_all")
        return b[:n], e[:n]

    def irregular_pairs(self, lo, hi, cap=None):
        """Irregular (kind 1) and E-irregular (kind 2) pairs (p, 2k) of the
        primes in [lo, hi): (IRR_PAIR_DTYPE array sorted by p, 2k, kind,
        primes examined, unresolved indices).  The default buffer holds four
        pairs per expected prime (about one is typical); a short buffer costs
        a second run."""
        if cap is None:
            cap = max(4096, int(4 * (int(hi) - int(lo)) / max(1.0, np.log(max(int(hi), 3)))))
        out = np.zeros(max(1, cap), dtype=IRR_PAIR_DTYPE)
        n, n_primes, n_unres = SZ(), U64(), U64()
        st = lib().wv_irregular_pairs(self._h, int(lo), int(hi), out.ctypes.data_as(VP), cap, ctypes.byref(n),
                                      ctypes.byref(n_primes), ctypes.byref(n_unres))
        if st == WV_ETRUNC:
            out = np.zeros(n.value, dtype=IRR_PAIR_DTYPE)
            st = lib().wv_irregular_pairs(self._h, int(lo), int(hi), out.ctypes.data_as(VP), n.value,
                                          ctypes.byref(n), ctypes.byref(n_primes), ctypes.byref(n_unres))
        _check(st, "wv_irregular_pairs")
        return out[:n.value], n_primes.value, n_unres.value

    def set_progress(self, fn=None, terms_per_launch=0):
        """Callback fn(done, total) between term-sum launches of long calls (None: off)."""
        if fn is None:
            self._progress = None
            _check(lib().wv_set_progress(self._h, PROGRESS_FN(), None, 0), "wv_set_progress")
            return
        self._progress = PROGRESS_FN(lambda _u, d, t: fn(d, t))
        _check(lib().wv_set_progress(self._h, self._progress, None, int(terms_per_launch)), "wv_set_progress")

    def autotune(self, p_hint, n_sample=16):
        """Times every compiled block shape x chunk size near p_hint; returns
        (kb, ke, chunk, {(kb, ke, chunk): terms/s})."""
        kb, ke = ctypes.c_int(), ctypes.c_int()
        ch = U64()
        nv = len(BLOCK_SHAPES)
        rates = (ctypes.c_double * (3 * nv))()
        _check(lib().wv_autotune(self._h, int(p_hint), int(n_sample), ctypes.byref(kb), ctypes.byref(ke),
                                 ctypes.byref(ch), rates), "wv_autotune")
        table = {}
        for v, (a, b) in enumerate(BLOCK_SHAPES):
            for j, c in enumerate((1 << 16, 1 << 18, 0)):   # 0: automatic per batch
                table[(a, b, c)] = rates[3 * v + j]
        return kb.value, ke.value, ch.value, table

    def tune_save(self, path):
        _check(lib().wv_tune_save(self._h, os.fsencode(path)), "wv_tune_save")

    def tune_load(self, path):
        _check(lib().wv_tune_load(self._h, os.fsencode(path)), "wv_tune_load")

    def eval_sums(self, primes, nb, ne):
        """Per-sum values S_j for the configured congruences: arrays (n, nb) and (n, ne)."""
        arr = np.ascontiguousarray(np.asarray(primes, dtype=np.uint64))
        ob = np.zeros((max(1, arr.size), nb), dtype=np.uint64)
        oe = np.zeros((max(1, arr.size), ne), dtype=np.uint64)
        st = lib().wv_eval_sums(self._h, arr.ctypes.data_as(P_U64), arr.size, ob.ctypes.data_as(P_U64),
                                oe.ctypes.data_as(P_U64))
        _check(st, "wv_eval_sums")
        return ob[:arr.size], oe[:arr.size]

    def eval_primes_async(self, d_primes_ptr, n, d_out_ptr, stream_ptr=0):
        """Enqueue on a HIP stream with device pointers (e.g. torch tensor data_ptr())."""
        st = lib().wv_eval_primes_async(self._h, VP(d_primes_ptr), int(n), VP(d_out_ptr),
                                        VP(stream_ptr) if stream_ptr else None)
        _check(st, "wv_eval_primes_async")

    def eval_primes_static(self, d_primes_ptr, n, d_out_ptr, stream_ptr=0):
        """As eval_primes_async, allocating nothing (the library's fixed scratch array)."""
        st = lib().wv_eval_primes_static(self._h, VP(d_primes_ptr), int(n), VP(d_out_ptr),
                                         VP(stream_ptr) if stream_ptr else None)
        _check(st, "wv_eval_primes_static")

    def stats(self):
        s = WvStats()
        _check(lib().wv_get_stats(self._h, ctypes.byref(s)), "wv_get_stats")
        return s.as_dict()


class Server:
    """Continuous-batching request server on a Context (wv_server_*)."""

    def __init__(self, ctx, step_terms=0, max_primes=0):
        cfg = WvServerConfig(int(step_terms), int(max_primes), 0)
        h = VP()
        _check(lib().wv_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "wv_server_create")
        self._h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().wv_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit_range(self, lo, hi):
        rid = U64()
        _check(lib().wv_server_submit_range(self._h, int(lo), int(hi), ctypes.byref(rid)), "wv_server_submit_range")
        return rid.value

    def submit_primes(self, primes):
        arr = np.ascontiguousarray(np.asarray(primes, dtype=np.uint64))
        rid = U64()
        _check(lib().wv_server_submit_primes(self._h, arr.ctypes.data_as(P_U64), arr.size, ctypes.byref(rid)),
               "wv_server_submit_primes")
        return rid.value

    def step(self):
        """One scheduling step; returns (active, pending)."""
        a, p = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().wv_server_step(self._h, ctypes.byref(a), ctypes.byref(p)), "wv_server_step")
        return a.value, p.value

    def result(self, rid):
        """(results array, latency_ms), or None while the request runs."""
        n = SZ()
        lat = ctypes.c_double()
        st = lib().wv_server_result(self._h, int(rid), None, 0, ctypes.byref(n), ctypes.byref(lat))
        if st == WV_EBUSY:
            return None
        if st == WV_OK:
            return np.zeros(0, dtype=RESULT_DTYPE), lat.value
        if st != WV_ETRUNC:
            _check(st, "wv_server_result")
        out = np.zeros(n.value, dtype=RESULT_DTYPE)
        _check(lib().wv_server_result(self._h, int(rid), out.ctypes.data_as(VP), n.value, ctypes.byref(n),
                                      ctypes.byref(lat)), "wv_server_result")
        return out, lat.value

    def stats(self):
        s = WvServerStats()
        _check(lib().wv_server_get_stats(self._h, ctypes.byref(s)), "wv_server_get_stats")
        return s.as_dict()

    def inject_fault(self, after_steps):
        _check(lib().wv_server_inject_fault(self._h, int(after_steps)), "wv_server_inject_fault")
