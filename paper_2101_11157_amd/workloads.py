"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

* ``bench_windows``: consecutive sub-windows of [1e11 - 1e6, 1e11), the primes
  at the paper's search ceiling (Section 3 and 5 searches end at 1e11).
* ``batch_windows``: uneven windows, lengths log-uniform in [1e3, 1e6] and
  starts log-uniform in [1e6, 1e11], drawn in that order from
  ``numpy.random.default_rng(seed)``.
* ``serve_trace``: a Poisson stream (mean 200 requests/s) of which 70 % are
  single primes (the smallest prime >= ceil(u)) and 30 % intervals
  [floor(u), floor(u) + L), u uniform in [1e8, 1e11], L log-uniform in
  [1e2, 1e5]; draw order gaps, kinds, u, L from ``default_rng(seed)``.
"""
import numpy as np

__all__ = ["bench_windows", "batch_windows", "serve_trace", "next_prime", "is_prime"]


def is_prime(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (input generation only)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for q in small:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def next_prime(n):
    """Smallest prime >= n."""
    n = max(int(n), 2)
    while not is_prime(n):
        n += 1
    return n


def bench_windows(count, width=8192, lo=10 ** 11 - 10 ** 6, hi=10 ** 11):
    """`count` consecutive windows of `width` integers from lo (inside [lo, hi))."""
    wins = [(lo + k * width, min(hi, lo + (k + 1) * width)) for k in range(count)]
    if wins and wins[-1][0] >= hi:
        raise ValueError("windows run past the range")
    return wins


def batch_windows(seed=0, n=64, len_range=(1e3, 1e6), start_range=(1e6, 1e11)):
    rng = np.random.default_rng(seed)
    L = np.floor(10 ** rng.uniform(np.log10(len_range[0]), np.log10(len_range[1]), n)).astype(np.int64)
    s = np.floor(10 ** rng.uniform(np.log10(start_range[0]), np.log10(start_range[1]), n)).astype(np.int64)
    return [(int(a), int(a + b)) for a, b in zip(s, L)]


def serve_trace(seed=0, n=128, rate=200.0, single_frac=0.7, u_range=(1e8, 1e11), len_range=(1e2, 1e5)):
    """[(arrival_s, kind, arg)] with kind 'prime' (arg: p) or 'range' (arg: (lo, hi))."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    single = rng.random(n) < single_frac
    u = rng.uniform(u_range[0], u_range[1], n)
    L = np.floor(10 ** rng.uniform(np.log10(len_range[0]), np.log10(len_range[1]), n)).astype(np.int64)
    t = np.cumsum(gaps)
    out = []
    for k in range(n):
        if single[k]:
            out.append((float(t[k]), "prime", next_prime(int(np.ceil(u[k])))))
        else:
            a = int(np.floor(u[k]))
            out.append((float(t[k]), "range", (a, a + int(L[k]))))
    return out
