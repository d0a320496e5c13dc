"""Build the derived congruences shipped with the package: for each side a
ladder of congruences from one greedy search, each serving a range of primes.

Greedy search of Section 2.2 (lambda = 1, D = 8; ties broken by piece order,
then d), run by paper_2101_11157_amd.derive from eqnVandiver (B, the start of
the paper's 546-sum Bernoulli congruence) and eqnEMac2 (E; the paper reports
438 sums and cost below p/30.4 after 100 rounds, which this search
reproduces).  More rounds give more, shorter sums and fewer terms in total.
On the GPU a prime's work is its terms plus a fixed cost per sum (the set-up
of a chunk's difference tables, its reduction and its share of the last,
ragged chunks), measured as about BETA = 6000 terms per sum (a least-squares
fit of time per prime against terms and sums, four congruence pairs of 4548
to 44,484 sums at each of 3e9, 1e10 and 1e11: 6193, 5682 and 6018 terms),
so the best number of rounds grows with p.  For each target p in TARGETS the search keeps the round whose
congruence minimises cost * p + BETA * sums; the distinct rounds found are the
rungs of the ladder, and each rung serves the primes from the point where its
work falls below the next smaller rung's (the lowest: below eqnBB30 /
eqnEE33's):
    min_p = BETA (n_hi - n_lo) / (c_lo - c_hi)
for consecutive rungs (n sums, cost c per unit p).  Every rung is a valid
congruence for every prime p >= 11 (subdivision factors are at most 8), so the
thresholds only move work around; results never depend on them.

The search is deterministic, so the files are reproducible; with the change of
cost of each candidate cached between rounds it takes about half a second per
round at 10,000 sums.

Writes tables/derived_<side>_<rounds>.json.gz and tables/ladder.json.
Usage: python -m paper_2101_11157_amd.tables.make_tables [B|E ...] [--rounds N]
"""
import argparse
import gzip
import json
import os
import sys
import time
from fractions import Fraction as Q

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2101_11157_amd import derive  # noqa: E402

ROUNDS = {"B": 6000, "E": 6000}
START = {"B": "Vandiver", "E": "EMac2"}
BETA = 6000                                        # terms of work per sum (measured)
TARGETS = [int(2 ** (k / 2)) for k in range(56, 77)]   # 2^28 .. 2^38, factor sqrt(2)
MIN_SPAN = 1.4                                         # narrowest range of p a rung serves
# eqnBB30 / eqnEE33 (Sections 3 and 5): sums, cost per unit p
PRINTED = {"B": (30, Q(227, 6480)), "E": (33, Q(27, 512))}


def _write_json(path, obj, gz=False):
    tmp = path + ".tmp"
    with (gzip.open(tmp, "wt", compresslevel=9) if gz else open(tmp, "w")) as f:
        json.dump(obj, f, indent=0 if not gz else None)
    os.replace(tmp, path)


def rungs_of(cand, printed):
    """Rungs (rounds, congruence, n, cost, min_p) in ascending rounds from the
    candidates {rounds: congruence}: keep a rung only where it beats the one
    below from some p on and that p rises along the ladder; then drop rungs
    that would serve less than a factor MIN_SPAN of p (their gain is
    negligible and each rung is another table to hold)."""
    cand = dict(cand)
    while True:
        out = []
        n_pr, c_pr = printed
        for r, c in sorted(cand.items()):
            n, cost = c.n_sums(), c.cost()
            while True:
                n0, c0 = (out[-1][2], out[-1][3]) if out else (n_pr, c_pr)
                if cost >= c0:
                    break
                pstar = max(11, int(-(-BETA * (n - n0) // (c0 - cost))))   # ceiling
                if out and pstar <= out[-1][4]:
                    out.pop()   # the rung below is never the cheapest
                    continue
                out.append((r, c, n, cost, pstar))
                break
        narrow = [k for k in range(len(out) - 1) if out[k + 1][4] < MIN_SPAN * out[k][4]]
        if not narrow:
            return out
        del cand[out[narrow[0]][0]]


def build(side, rounds):
    start = START[side]
    t0 = time.time()
    best = {}   # target -> (work, round, copy)

    def log(r, c):
        n, cost = c.n_sums(), c.cost()
        for p in TARGETS:
            w = cost * p + BETA * n
            if p not in best or w < best[p][0]:
                best[p] = (w, r, c.copy())
        if r % 100 == 0:
            print(f"{side}: round {r}: {n} sums, cost p/{float(1 / cost):.3f} ({time.time() - t0:.0f} s)",
                  flush=True)

    derive.greedy(derive.Congruence.start(start), D=8, rounds=rounds, log=log)
    ladder = []
    for r, c, n, cost, pstar in rungs_of({v[1]: v[2] for v in best.values()}, PRINTED[side]):
        name = f"derived_{side}_{r}.json.gz"
        obj = c.to_json(f"greedy {start}, D=8, round {r} of {rounds}")
        _write_json(os.path.join(HERE, name), obj, gz=True)
        ladder.append({"rounds": r, "min_p": pstar, "file": name, "n": n, "cost": [cost.numerator, cost.denominator]})
        print(f"{side}: rung round {r}: {n} sums, cost p/{float(1 / cost):.3f}, from p = {pstar}", flush=True)
    return ladder


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("sides", nargs="*", default=["B", "E"])
    ap.add_argument("--rounds", type=int, default=0)
    a = ap.parse_args()
    path = os.path.join(HERE, "ladder.json")
    for s in a.sides:
        rungs = build(s, a.rounds or ROUNDS[s])
        doc = {"beta": BETA, "targets": TARGETS, "min_span": MIN_SPAN}
        if os.path.exists(path):   # read just before writing: the other side may be built alongside
            with open(path) as f:
                doc.update({k: v for k, v in json.load(f).items() if k in ("B", "E")})
        doc[s] = rungs
        _write_json(path, doc)
