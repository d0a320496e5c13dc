"""Build the derived congruences shipped with the package.

Greedy search of Section 2.2 (lambda = 1, D = 8, a fixed number of rounds;
ties broken by piece order, then d), run by paper_2101_11157_amd.derive:

* derived_B.json: from eqnVandiver (the start of the paper's 546-sum
  Bernoulli congruence), ROUNDS_B rounds;
* derived_E.json: from eqnEMac2, ROUNDS_E rounds (the paper reports 438 sums
  and cost below p/30.4 for this search, which 100 rounds reproduce: 438 sums,
  cost p/30.47; the search keeps lowering the cost after that).

More rounds trade more sums for fewer terms; at p near 1e11 a sum holds
about 350,000 terms, so its fixed cost (a chunk set-up and a reduction) is
small and the cheapest congruence wins.  1200 rounds give 5849 sums at cost
p/53.79 (B) and 5545 sums at p/50.18 (E) and take about two and a half hours
per side (800 rounds: 3798 sums at p/50.73 and 3626 at p/47.03); the search
is deterministic, and continuing a saved congruence gives the same result as
running the rounds in one go.

Usage: python -m paper_2101_11157_amd.tables.make_tables [B|E ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2101_11157_amd import derive  # noqa: E402

ROUNDS_B = 1200
ROUNDS_E = 1200
PLAN = {"B": ("Vandiver", ROUNDS_B), "E": ("EMac2", ROUNDS_E)}


def build(side):
    start, rounds = PLAN[side]
    t0 = time.time()

    def log(r, c):
        if r % 10 == 0:
            print(f"{side}: round {r}: {c.n_sums()} sums, cost p/{float(1 / c.cost()):.3f} "
                  f"({time.time() - t0:.0f} s)", flush=True)

    _, best, r = derive.greedy(derive.Congruence.start(start), D=8, rounds=rounds, log=log)
    obj = best.to_json(f"greedy {start}, D=8, {rounds} rounds (best at round {r})")
    path = os.path.join(HERE, f"derived_{side}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=0)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}: {best.n_sums()} sums, cost p/{float(1 / best.cost()):.3f}", flush=True)


if __name__ == "__main__":
    for side in sys.argv[1:] or ["B", "E"]:
        build(side)
