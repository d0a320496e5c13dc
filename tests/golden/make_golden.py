"""Write the stored oracle values the GPU parity tests compare against.

Calls only the oracle package (plain CPU code).  Inputs are the seeded samples
of the paper-scale workloads:

* window_1e9.json   primes in [1e9, 1e9 + 1e7): first 8, last 8 and 256 drawn
                    with random.Random(0); B_{p-3}, E_{p-3} mod p by the printed
                    eqnBB30 / eqnEE33, and 32 of them again by the root forms
                    eqnBB1 (Stafford-Vandiver) and eqnE1.
* window_1e11.json  primes in [1e11 - 1e6, 1e11): first 2, last 2 and 12 drawn
                    with random.Random(0), by eqnBB30 / eqnEE33; 4 of them also
                    by eqnBB1 / eqnE1.
* counts.json       prime counts of the sieve windows (plain sieve).
* sums_2p40.json    single sums S(x, y) for the largest primes below 2^40
                    (the top of the supported range), for the narrowest
                    intervals of eqnBB30 and eqnEE33.
* batch_seed0.json  the 64 uneven windows of workloads.batch_windows(seed 0):
                    prime count of every window, and residues (eqnBB30 /
                    eqnEE33) of its first and last prime and of 2 more drawn
                    with random.Random(window index).
* serve_seed0.json  the 128 requests of workloads.serve_trace(seed 0): for a
                    single prime its residues, for an interval its prime count
                    and the residues of one prime drawn with
                    random.Random(request index).

Usage: python tests/golden/make_golden.py [which ...]   (default: all)
"""
import json
import os
import random
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import congruences as C  # noqa: E402


def _write(name, obj):
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def sample(ps, first, last, k, seed):
    rng = random.Random(seed)
    mid = ps[first:len(ps) - last]
    pick = sorted(rng.sample(mid, k))
    return sorted(set(ps[:first] + pick + ps[len(ps) - last:]))


def both(p, cb, ce, nthreads):
    return (oracle.congruence_residue(p, cb, nthreads=nthreads),
            oracle.congruence_residue(p, ce, nthreads=nthreads))


def window(lo, hi, first, last, k, n_root, name):
    t0 = time.time()
    ps = oracle.primes(lo, hi)
    pick = sample(ps, first, last, k, 0)
    nt = oracle.max_threads()
    rows = []
    root_set = set(random.Random(1).sample(pick, n_root))
    for i, p in enumerate(pick):
        b, e = both(p, C.BB30, C.EE33, nt)
        row = {"p": p, "b": b, "e": e, "method": "eqnBB30+eqnEE33"}
        if p in root_set:
            b2, e2 = both(p, C.SV, C.E1, nt)
            if (b2, e2) != (b, e):
                raise AssertionError(f"oracle forms disagree at {p}: {(b, e)} vs {(b2, e2)}")
            row["method"] += ", eqnBB1+eqnE1"
        rows.append(row)
        print(f"{name}: {i + 1}/{len(pick)} p={p} ({time.time() - t0:.0f}s)", flush=True)
    _write(name, {"lo": lo, "hi": hi, "n_primes": len(ps), "rows": rows,
                  "sample": f"first {first}, last {last}, {k} by random.Random(0); "
                            f"{n_root} rechecked by root forms (random.Random(1))"})


def counts():
    out = {}
    for lo, hi in [(5, 10 ** 5), (10 ** 9, 10 ** 9 + 10 ** 7), (10 ** 11 - 10 ** 6, 10 ** 11),
                   (2 ** 40 - 2 ** 21, 2 ** 40)]:
        out[f"{lo},{hi}"] = len(oracle.primes(lo, hi))
    _write("counts.json", out)


def sums_2p40():
    ps = oracle.primes(2 ** 40 - 2 ** 12, 2 ** 40)[-3:]
    rows = []
    nt = oracle.max_threads()
    for cong in (C.BB30, C.EE33):
        widths = sorted(range(len(cong.terms)), key=lambda i: cong.terms[i][2] - cong.terms[i][1])
        for i in widths[:3]:
            _, x, y = cong.terms[i]
            for p in ps:
                lo, hi = oracle.interval(p, x, y)
                S = oracle.sum_poly(p, lo, hi, -cong.ell, cong.alt, nthreads=nt)
                rows.append({"p": p, "table": cong.name, "term": i, "lo": lo, "hi": hi, "S": S})
                print("sum", cong.name, i, p, hi - lo + 1, flush=True)
    _write("sums_2p40.json", {"rows": rows})


def _residue_rows(ps, nt):
    rows = []
    for p in ps:
        b, e = both(p, C.BB30, C.EE33, nt)
        rows.append({"p": p, "b": b, "e": e})
    return rows


def batch_seed0():
    from paper_2101_11157_amd import workloads
    t0 = time.time()
    nt = oracle.max_threads()
    out = []
    for i, (lo, hi) in enumerate(workloads.batch_windows(0, 64)):
        ps = oracle.primes(lo, hi)
        pick = sorted(set([ps[0], ps[-1]] + random.Random(i).sample(ps, 2)))
        out.append({"lo": lo, "hi": hi, "n_primes": len(ps), "rows": _residue_rows(pick, nt)})
        print(f"batch window {i}: [{lo}, {hi}) {len(ps)} primes ({time.time() - t0:.0f}s)", flush=True)
    _write("batch_seed0.json", {"windows": out, "method": "eqnBB30+eqnEE33",
                                "sample": "first, last and 2 by random.Random(window index)"})


def serve_seed0():
    from paper_2101_11157_amd import workloads
    t0 = time.time()
    nt = oracle.max_threads()
    out = []
    for i, (t, kind, arg) in enumerate(workloads.serve_trace(0, 128)):
        if kind == "prime":
            out.append({"kind": kind, "p": arg, "rows": _residue_rows([arg], nt)})
        else:
            ps = oracle.primes(*arg)
            pick = random.Random(i).sample(ps, 1) if ps else []
            out.append({"kind": kind, "lo": arg[0], "hi": arg[1], "n_primes": len(ps),
                        "rows": _residue_rows(pick, nt)})
        print(f"serve request {i}: {kind} ({time.time() - t0:.0f}s)", flush=True)
    _write("serve_seed0.json", {"requests": out, "method": "eqnBB30+eqnEE33",
                                "sample": "single primes; one prime per interval by random.Random(request index)"})


if __name__ == "__main__":
    which = sys.argv[1:] or ["counts", "sums", "w9", "w11", "batch", "serve"]
    if "counts" in which:
        counts()
    if "sums" in which:
        sums_2p40()
    if "w9" in which:
        window(10 ** 9, 10 ** 9 + 10 ** 7, 8, 8, 256, 32, "window_1e9.json")
    if "w11" in which:
        window(10 ** 11 - 10 ** 6, 10 ** 11, 2, 2, 12, 4, "window_1e11.json")
    if "batch" in which:
        batch_seed0()
    if "serve" in which:
        serve_seed0()
