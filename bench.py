#!/usr/bin/env python3
"""Throughput benchmark: primes tested per second at p ~ 1e11 on one MI355X.

Workload (the paper's search ceiling): the primes in [1e11 - 1e6, 1e11), all
below 2^37, each tested for both residues B_{p-3} mod p and E_{p-3} mod p with
the congruences eqnBB30 (Section 3) and eqnEE33 (Section 5).  A step is one
pass of the whole path over the next sub-window of `--window` consecutive
integers of that range (about window / 25.3 primes): segmented sieve, plan,
term sums, reductions, finalize, results copied to the host.  Warm-up steps
take the sub-windows before the timed ones, so no step repeats work.

Prints one JSON line.  `roofline` describes the term-sum kernel (the dominant
kernel), which is bound by vector-ALU issue: the full-rate VALU operations its
algorithm needs (ops_per_term below: double-precision modular products,
difference-table additions and the periodic table reductions of the blocked
Taylor-coefficient loop, times the terms it summed; plus setup_ops_per_chunk
for every blocked chunk: building its difference tables and folding the terms
after its last full block; both as written in the source), over its own
HIP-event time, against the chip's VALU issue rate (256 CUs x 4 SIMDs x 16
lanes x 2.4 GHz).  `frac_terms_only` leaves the set-up out.  Register moves
the compiler adds are not counted.
`cpu_baseline` is the plain CPU oracle timed on this host on a bounded sample
of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PAPER_V100_PRIMES_PER_S = 1.0 / (25.3e-3 + 34.1e-3)   # Section 3 and Section 5 timings at 1e11
PEAK_VALU = 256 * 4 * 16 * 2.4e9                        # full-rate VALU lane operations per second
OPS_MONT = 12       # one Montgomery product: 8 32x32->64 multiply-adds, 2 low multiplies, 2 64-bit adds
OPS_ADDM = 3        # one modular addition: add, subtract, select
OPS_FMUL = 6        # one double-precision modular product: mul, 3 fma, 2 add
OPS_FRED = 3        # one double-precision reduction: fma, add, fma
# per block of the Taylor-coefficient loop: modular products, reductions of
# the g_k entering them (g0 and g1), and plain additions or exact
# multiply-adds (d = 2: P = g0^2, g0 g2, g1^2, Q = g1^2 - 2 g0 g2 by two
# additions and the three products of the running pair's update, plus its one
# addition; d = 3: g0^2, P, g0^2 g3, g0 g2, g1^2, g1 (g1^2 - 3 g0 g2), Q, the
# two differences as multiply-adds, and the update)
BLOCK_FMUL = {2: 6, 3: 9}
BLOCK_FRED = {2: 2, 3: 2}
BLOCK_ADD = {2: 3, 3: 3}
BLOCK_XFMA = {2: 0, 3: 2}   # of BLOCK_ADD, the exact multiply-adds forming Q

# HBM bytes (read + written) of one term-sum launch on the bench's first timed
# window, measured with rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a copy of
# known size (profiles/k_sum_window_1e11_*.md).  A profile constant: valid only
# for the kernel source, shape, tables and window it was taken on (keyed by the
# hash of the kernel sources), reported as null otherwise.
MEASURED_TRAFFIC = {
    ("1e11", "derived 31184/30413", 28, 36, 8192, "bb093ffd867d"): 3805379614,
}


def kernel_source_hash():
    """Short hash of the term-sum kernel's sources (traffic figures are keyed by it)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("wv_kernels.hip", "sum_core.hpp", "mont.hpp"):
        with open(os.path.join(ROOT, "paper_2101_11157_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def rung_at(side, p):
    """The shipped derived congruence (a rung of the ladder) that serves prime
    p, or None where the printed table does."""
    import paper_2101_11157_amd as wv
    use = [r for r in wv.derived_ladder(side) if p >= r["min_p"]]
    return use[-1] if use else None


def tables_key(which, p=10 ** 11 - 1):
    """The congruences a traffic figure was measured with (derived: the sum
    counts of the rungs serving p)."""
    if which != "derived":
        return which
    rb, re_ = rung_at("B", p), rung_at("E", p)
    return f"derived {rb['n'] if rb else 30}/{re_['n'] if re_ else 33}"


def renorm_period(p):
    """Blocks between reductions of the difference tables for primes below p."""
    return 53 - int(p).bit_length()


def table_entries(d, k):
    """Entries of the difference tables of g_0 .. g_d (degrees k .. k - d)."""
    return (d + 1) * (k + 1) - d * (d + 1) // 2


def ops_per_term(d, k, period):
    """Full-rate VALU operations per term of a sum of s^-d with blocks of k terms."""
    if k == 1:   # one factor per term (Montgomery): two products, one add, d difference steps
        return 2 * OPS_MONT + 1 + d * OPS_ADDM
    sz = table_entries(d, k)
    stepped = sz - (d + 1)   # the constant top entries are not stepped
    per_block = BLOCK_FMUL[d] * OPS_FMUL + BLOCK_FRED[d] * OPS_FRED + BLOCK_ADD[d] + stepped
    return (per_block + sz * OPS_FRED / period) / k


def setup_ops_per_chunk(d, k):
    """Full-rate VALU operations of one blocked chunk's set-up, as written in
    csrc/sum_core.hpp: the terms after the last full block folded one by one
    ((k - 1) / 2 on average: s^d by modular products, the pair update, a
    reduction), the tables cleared, one update per coefficient that can be
    nonzero (blocks of four) after each of the k factors (f_mulmod_add plus
    two exact multiply-adds, none for m = 0), the factor's own value, and the
    two canonical residues at the end."""
    nt = d + 1
    upd = 0
    for j in range(k):
        for kk in range(nt):
            for mb in range((k - kk) // 4 + 1):
                if 4 * mb > j + 1 - kk:
                    continue
                for m in range(min(4 * mb + 3, k - kk), 4 * mb - 1, -1):
                    upd += 8 + (2 if m > 0 else 0)
    tail_term = (d - 1) * OPS_FMUL + 2 * OPS_FMUL + 1 + OPS_FRED
    return (k - 1) / 2 * tail_term + table_entries(d, k) + upd + 2 * k + 2 * 5


def muls_per_term(d, k, period):
    """Multiply-class instructions per term: 32x32-bit integer multiplies on
    the k = 1 path (ten per Montgomery product), f64 mul / fma on the blocked
    path (four per modular product, two per reduction)."""
    if k == 1:
        return 2 * 10
    return (BLOCK_FMUL[d] * 4 + BLOCK_FRED[d] * 2 + BLOCK_XFMA[d] + table_entries(d, k) * 2 / period) / k


def blocked_threshold(d, k):
    """Chunks shorter than this run the one-term (Montgomery) loop (chunk_blocked
    in the kernel)."""
    return 8 * (d + 1) * k if k > 1 else float("inf")


class OpsModel:
    """VALU operations of the term-sum kernel for a set of primes, from the
    congruences each prime uses (the rung of the derived ladder its size
    selects, or eqnBB30 / eqnEE33): per prime and side, the terms of the sums
    long enough for the blocked loop (ops_per_term with that prime's
    reduction period) and of the shorter ones (the one-term loop).  The term
    counts are scaled to the kernel's measured totals per side."""

    def __init__(self, tables, kb, ke):
        import numpy as np
        import paper_2101_11157_amd as wv
        self.np = np
        self.kb, self.ke = kb, ke
        self.widths = {}     # (side, rounds or None) -> (sorted widths, prefix sums)
        self.rungs = {}      # side -> [(min_p, rounds)] ascending
        for side, name in (("B", "BB30"), ("E", "EE33")):
            w = sorted(ya / yb - xa / xb for _, xa, xb, ya, yb in wv.table_terms(name))
            self.widths[(side, None)] = (np.array(w), np.concatenate([[0.0], np.cumsum(w)]))
            self.rungs[side] = []
            if tables == "derived":
                for r in wv.derived_ladder(side):
                    terms = wv.derived_table(side, r["rounds"])["terms"]
                    w = sorted(int(ya) / int(yb) - int(xa) / int(xb) for _, xa, xb, ya, yb in terms)
                    self.widths[(side, r["rounds"])] = (np.array(w), np.concatenate([[0.0], np.cumsum(w)]))
                    self.rungs[side].append((r["min_p"], r["rounds"]))

    def _side_terms(self, ps, side, d, k):
        """(blocked terms, one-term-loop terms) per prime of one side."""
        np = self.np
        blk = np.zeros(len(ps))
        one = np.zeros(len(ps))
        thr = blocked_threshold(d, k)
        mins = np.array([m for m, _ in self.rungs[side]], dtype=np.float64)
        pick = np.searchsorted(mins, ps, side="right") - 1     # -1: the printed table
        for j in np.unique(pick):
            key = (side, None if j < 0 else self.rungs[side][j][1])
            use = pick == j
            w, cum = self.widths[key]
            q = ps[use]
            cut = np.searchsorted(w, thr / q)        # sums narrower than thr / p are short
            short = cum[cut] * q
            blk[use] = (cum[-1] * q) - short
            one[use] = short
        return blk, one

    def _long_sums(self, ps, side, d, k):
        """Sums per prime long enough for the blocked loop."""
        np = self.np
        out = np.zeros(len(ps))
        thr = blocked_threshold(d, k)
        mins = np.array([m for m, _ in self.rungs[side]], dtype=np.float64)
        pick = np.searchsorted(mins, ps, side="right") - 1
        for j in np.unique(pick):
            w, _ = self.widths[(side, None if j < 0 else self.rungs[side][j][1])]
            use = pick == j
            out[use] = len(w) - np.searchsorted(w, thr / ps[use])
        return out

    def ops(self, primes, n_terms_b, n_terms, chunk=0):
        """Modelled VALU operations for the primes' term sums, scaled to the
        measured Bernoulli-side and total term counts; with the chunk size,
        also the set-up of every blocked chunk (about one per long sum plus
        one per `chunk` blocked terms; setup_ops_per_chunk)."""
        np = self.np
        ps = np.asarray(primes, dtype=np.float64)
        if len(ps) == 0 or n_terms == 0:
            return 0.0
        per = np.array([renorm_period(int(p)) for p in primes], dtype=np.float64)
        total = 0.0
        for side, d, k, measured in (("B", 3, self.kb, n_terms_b), ("E", 2, self.ke, n_terms - n_terms_b)):
            blk, one = self._side_terms(ps, side, d, k)
            est = blk.sum() + one.sum()
            if est <= 0 or measured <= 0:
                continue
            opt_blk = np.array([ops_per_term(d, k, int(t)) for t in per])
            ops = (blk * opt_blk).sum() + one.sum() * ops_per_term(d, 1, 1)
            total += ops * (measured / est)
            if chunk and k > 1:
                chunks = self._long_sums(ps, side, d, k).sum() + blk.sum() * (measured / est) / chunk
                total += chunks * setup_ops_per_chunk(d, k)
        return total

def sum_kernel_muls(st, period):
    nb = st["n_terms_b"]
    return (nb * muls_per_term(3, st["block_k_b"], period)
            + (st["n_terms"] - nb) * muls_per_term(2, st["block_k_e"], period))


def sum_kernel_ops(st, period):
    nb = st["n_terms_b"]
    ne = st["n_terms"] - nb
    return nb * ops_per_term(3, st["block_k_b"], period) + ne * ops_per_term(2, st["block_k_e"], period)

CONFIGS = {
    "1e11": (10 ** 11 - 10 ** 6, 10 ** 11, 8192),
    "1e9": (10 ** 9, 10 ** 9 + 10 ** 7, 1 << 18),
    "1e5": (5, 10 ** 5, 10 ** 5),
}
EXTRA_CONFIGS = ("batch", "serve", "irregular", "peak")

PEAK_NAMES = ["v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mul_u32_u24", "v_add_u32", "v_lshl_add_u64",
              "v_fma_f64", "v_add_co_u32", "v_addc_co_u32", "v_cndmask_b32", "v_cmp_gt_u32", "v_min_u32",
              "v_mov_b32", "v_sub_u32"]


def bench_peak(args):
    """Instruction rates of the chip (libwvpeak.so): lane operations per second
    of independent back-to-back VALU instructions of each class, and the f64
    matrix rate over instruction shape, accumulator chains and waves per SIMD.
    These are the measured ceilings behind the rooflines: the term-sum kernel
    issues f64 adds/FMAs and, on the one-term path, 32-bit multiplies."""
    import ctypes
    path = os.path.join(ROOT, "paper_2101_11157_amd", "libwvpeak.so")
    L = ctypes.CDLL(path)
    n = L.wv_peak_count()
    rates = (ctypes.c_double * n)()
    rc = L.wv_peak_rates(0, rates)
    if rc != 0:
        print(f"bench.py: wv_peak_rates failed ({rc})", file=sys.stderr)
        sys.exit(1)
    valu = {PEAK_NAMES[k]: {"lane_ops_per_s": rates[k], "of_full_rate": rates[k] / PEAK_VALU} for k in range(n)}
    cap = 64
    rows = (ctypes.c_double * (4 * cap))()
    L.wv_peak_mfma_f64_sweep.restype = ctypes.c_int
    m = L.wv_peak_mfma_f64_sweep(0, rows, cap)
    mfma = [{"instruction": "v_mfma_f64_16x16x4_f64" if rows[4 * i] == 16 else "v_mfma_f64_4x4x4_4b_f64",
             "chains": int(rows[4 * i + 1]), "waves_per_simd": int(rows[4 * i + 2]),
             "tflops": rows[4 * i + 3] / 1e12, "of_published_peak": rows[4 * i + 3] / PEAK_MFMA_F64}
            for i in range(max(m, 0))]
    print(json.dumps({"metric": "instruction rates (1 GPU)", "full_rate_valu_lane_ops_per_s": PEAK_VALU,
                      "published_f64_matrix_flops": PEAK_MFMA_F64, "valu": valu, "mfma_f64": mfma}), flush=True)


def use_tables(ctx, which, p=10 ** 11 - 1):
    """Select the congruences; returns their description (at prime size p)."""
    if which == "derived":
        import paper_2101_11157_amd as wv
        ctx.use_derived_tables()
        parts = []
        for side in "BE":
            lad = wv.derived_ladder(side)
            r = rung_at(side, p)
            at = (f"{r['n']}-sum {side} of {r['rounds']} rounds (cost {r['cost'][0]}/{r['cost'][1]})" if r
                  else f"eqnBB30/eqnEE33 for {side}")
            parts.append(f"{side}: {len(lad)} rungs from p >= {lad[0]['min_p']}, here the {at}")
        return "derived ladders (greedy, Section 2.2; eqnBB30+eqnEE33 below the lowest rung): " + "; ".join(parts)
    return "eqnBB30+eqnEE33"


def cpu_threads():
    for k in ("OMP_NUM_THREADS",):
        v = os.environ.get(k)
        if v and v.isdigit() and int(v) > 0:
            return int(v)
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(primes, nthreads):
    """The oracle as it stands: eqnBB30 + eqnEE33 evaluated plainly, one prime
    at a time with each sum's range split over threads.  Returns (primes/s,
    seconds, [(b, e)])."""
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    got = [oracle.residue_one_parallel(p, method="table", nthreads=nthreads) for p in primes]
    dt = time.perf_counter() - t0
    return len(primes) / dt, dt, got


def table_cost(tables, p=10 ** 11 - 1):
    """Terms per unit p of the congruences used at prime size p: (B, E)."""
    if tables == "derived":
        rb, re_ = rung_at("B", p), rung_at("E", p)
        return (rb["cost"][0] / rb["cost"][1] if rb else 227 / 6480,
                re_["cost"][0] / re_["cost"][1] if re_ else 27 / 512)
    return 227 / 6480, 27 / 512


def measure_plain(args, wv, wins, lo0, hi0, W):
    """The headline: consecutive sub-windows through wv_search_range."""
    ctx = wv.Context(0)
    if args.chunk:
        ctx.set_chunk_terms(args.chunk)
    if args.block:
        ctx.set_block(*[int(v) for v in args.block.split(",")])
    tables = use_tables(ctx, args.tables, hi0 - 1)
    for k in range(args.warmup):
        ctx.search_range(*wins[k])
        print(f"warmup {k}: window {wins[k]}", file=sys.stderr, flush=True)
    primes = terms = terms_b = 0
    muls = 0.0
    period = renorm_period(hi0 - 1)   # exact for every prime of the 1e11 and 1e9 ranges
    block = None
    ms_sum = ms_dev = 0.0
    timed = []
    steps_st = []
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        res, hits = ctx.search_range(*wins[k])
        st = ctx.stats()
        primes += len(res)
        terms += st["n_terms"]
        terms_b += st["n_terms_b"]
        muls += sum_kernel_muls(st, period)
        block = [st["block_k_b"], st["block_k_e"]]
        ms_sum += st["ms_sum"]
        ms_dev += st["ms_total"]
        timed.append(res)
        steps_st.append((st["n_terms_b"], st["n_terms"], st["chunk_terms"]))
        print(f"step {k - args.warmup}: {len(res)} primes, {st['n_terms']:.3e} terms, "
              f"sum kernel {st['ms_sum']:.1f} ms, device {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    ctx.close()
    # bookkeeping outside the timed region: the modelled operations of each
    # step's launch, with and without the chunks' set-up
    ops = ops_terms = 0.0
    if block:
        om = OpsModel(args.tables, block[0], block[1])
        for res, (nb, nt, C) in zip(timed, steps_st):
            plist = [int(p) for p in res["p"]]
            ops += om.ops(plist, nb, nt, chunk=C)
            ops_terms += om.ops(plist, nb, nt)
    return dict(tables=tables, primes=primes, terms=terms, terms_b=terms_b, ops=ops, ops_terms=ops_terms, muls=muls,
                block=block, ms_sum=ms_sum, ms_dev=ms_dev, wall=wall, results=timed)


def measure_batch(args, wv, nwin):
    """The batched workload: `nwin` uneven seeded windows (lengths log-uniform
    in [1e3, 1e6], starts log-uniform in [1e6, 1e11], numpy default_rng(0)) in
    one wv_search_windows call."""
    from paper_2101_11157_amd import workloads
    wins = workloads.batch_windows(0, nwin)
    ctx = wv.Context(0)
    if args.chunk:
        ctx.set_chunk_terms(args.chunk)
    tables = use_tables(ctx, args.tables)
    t_start = time.perf_counter()
    last = [0.0]

    def progress(done, total):
        t = time.perf_counter()
        if t - last[0] > 10 or done == total:
            last[0] = t
            print(f"batch progress {done}/{total} chunks at {t - t_start:.1f} s", file=sys.stderr, flush=True)

    ctx.set_progress(progress)
    t0 = time.perf_counter()
    res = ctx.search_windows([a for a, _ in wins], [b for _, b in wins])
    wall = time.perf_counter() - t0
    st = ctx.stats()
    primes = sum(len(r) for r in res)
    plist = [int(p) for r in res for p in r["p"]]
    ops = OpsModel(args.tables, st["block_k_b"], st["block_k_e"]).ops(plist, st["n_terms_b"], st["n_terms"],
                                                                       chunk=st["chunk_terms"])
    ok = None
    if args.verify:
        ctx.set_progress(None)
        order = sorted(range(len(wins)), key=lambda k: wins[k][1] - wins[k][0])[: args.verify]
        ok = True
        for k in order:
            ref, _ = ctx.search_range(*wins[k])
            same = as_pairs(ref) == as_pairs(res[k])
            ok = ok and same
            print(f"verify window {k} {wins[k]}: {len(ref)} primes, {'identical' if same else 'DIFFERENT'}",
                  file=sys.stderr, flush=True)
    ctx.close()
    return dict(workload=f"{len(wins)} seeded windows (default_rng(0)), lengths log-uniform [1e3, 1e6], "
                         f"starts log-uniform [1e6, 1e11], one wv_search_windows call",
                tables=tables, primes=primes, terms=st["n_terms"], terms_b=st["n_terms_b"], ops=ops,
                ms_sum=st["ms_sum"], wall=wall, block=[st["block_k_b"], st["block_k_e"]], verified=ok,
                n_verified=args.verify, wins=wins, results=res)


def same_windows_batched(args, wv, wins):
    """The same sub-windows of the headline range through the plain path (one
    wv_search_range call each, in order) and through one wv_search_windows
    call, on one context with the same congruences; primes/s of both over
    the wall clock and whether every result is identical."""
    if not wins:
        return None
    ctx = wv.Context(0)
    use_tables(ctx, args.tables)
    # warm-up, not timed: the batched call sizes the context's device buffers
    # (a few GB of plan records) for both paths
    ctx.search_windows([a for a, _ in wins], [b for _, b in wins])
    t0 = time.perf_counter()
    plain = [ctx.search_range(a, b)[0] for a, b in wins]
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batched = ctx.search_windows([a for a, _ in wins], [b for _, b in wins])
    t_batch = time.perf_counter() - t0
    ctx.close()
    n = sum(len(r) for r in plain)
    same = all(as_pairs(x) == as_pairs(y) for x, y in zip(plain, batched))
    print(f"same windows at 1e11: {len(wins)} windows, {n} primes, plain {t_plain:.3f} s, batched {t_batch:.3f} s",
          file=sys.stderr, flush=True)
    return {"workload": f"{len(wins)} consecutive sub-windows of {wins[0][1] - wins[0][0]} integers after the timed "
                        f"ones ({wins[0][0]}..{wins[-1][1]})",
            "primes": n, "plain_primes_per_s": n / t_plain, "batched_primes_per_s": n / t_batch,
            "batched_over_plain": t_plain / t_batch, "identical_results": same}


def per_window_plain(args, wv, wins, batched):
    """The plain per-window path on the same windows: one wv_search_range call
    per window, in order, on a fresh context with the same congruences;
    returns (primes/s over the wall clock, results identical to the batched
    call's)."""
    ctx = wv.Context(0)
    use_tables(ctx, args.tables)
    same = True
    primes = 0
    t0 = time.perf_counter()
    for k, (a, b) in enumerate(wins):
        res, _ = ctx.search_range(a, b)
        primes += len(res)
        same = same and as_pairs(res) == as_pairs(batched[k])
    wall = time.perf_counter() - t0
    ctx.close()
    print(f"per-window plain path: {len(wins)} windows, {primes} primes in {wall:.1f} s", file=sys.stderr, flush=True)
    return primes / wall, wall, same


def requests_alone(args, wv, trace, served):
    """The requests of a serving trace through the plain path one at a time
    (wv_eval_primes for a single prime, wv_search_range for an interval), all
    available at once; returns (primes/s over the wall clock, every result
    identical to the served one)."""
    ctx = wv.Context(0)
    use_tables(ctx, args.tables)
    same = True
    primes = 0
    t0 = time.perf_counter()
    for k, (_, kind, arg) in enumerate(trace):
        res = ctx.eval_primes([arg]) if kind == "prime" else ctx.search_range(*arg)[0]
        primes += len(res)
        same = same and as_pairs(res) == as_pairs(served[k])
    wall = time.perf_counter() - t0
    ctx.close()
    print(f"requests alone: {len(trace)} requests, {primes} primes in {wall:.1f} s", file=sys.stderr, flush=True)
    return primes / wall, wall, same


def rate_summary(primes, terms, ops, wall, ms_sum):
    """primes/s and terms/s over the wall clock, and the term-sum kernel's
    modelled VALU rate over its own time (frac of the issue peak)."""
    achieved = ops / (ms_sum * 1e-3) / 1e12 if ms_sum > 0 else 0.0
    return {"primes_per_s": primes / wall, "terms_per_s": terms / wall, "primes": primes, "terms": terms,
            "wall_s": wall, "sum_kernel_ms": ms_sum, "valu_tops": achieved, "frac": achieved / (PEAK_VALU / 1e12)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="1e11", choices=sorted(CONFIGS) + list(EXTRA_CONFIGS))
    ap.add_argument("--windows", type=int, default=64, help="batch: number of seeded windows")
    ap.add_argument("--verify", type=int, default=0,
                    help="batch: windows re-run alone and compared (smallest first); serve: nonzero compares "
                         "every request with the same request run alone")
    ap.add_argument("--requests", type=int, default=128, help="serve: requests in the seeded trace")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: mean arrivals per second")
    ap.add_argument("--step-terms", type=int, default=0, help="serve: terms per scheduling step")
    ap.add_argument("--load", type=float, default=0.0,
                    help="serve: also replay the trace at this fraction of the measured capacity")
    ap.add_argument("--window", type=int, default=0, help="integers per step (0: config default)")
    ap.add_argument("--chunk", type=int, default=0, help="terms per lane chunk (0: automatic)")
    ap.add_argument("--block", default="", help="term-sum block shape KB,KE (default: the library's)")
    ap.add_argument("--tables", default="derived", choices=["derived", "printed"],
                    help="derived: the package's ladders of greedy-derived congruences (Section 2.2), "
                         "printed: eqnBB30 + eqnEE33")
    ap.add_argument("--irr-path", default="auto", choices=["auto", "valu", "mfma"],
                    help="irregular: power-sum kernel (auto: matrix cores below 2^24)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="1e11: leave the batched workload out of the line")
    ap.add_argument("--no-serve", action="store_true", help="1e11: leave the served trace out of the line")
    ap.add_argument("--no-same-work", action="store_true",
                    help="1e11: skip the plain path on the batched windows and the served requests")
    ap.add_argument("--cpu-primes", type=int, default=4, help="primes in the oracle sample")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device fill and one copy of this many bytes (torch): kernels of known "
                         "traffic that scale the HBM byte counters of a profiler run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported (primes are independent: "
              "split the range by cost, one process per GPU, and gather the results)", file=sys.stderr)
        sys.exit(2)

    if args.copy_bytes:
        import torch   # before the library: torch loads its own HIP runtime first
        x = torch.empty(args.copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        y = x.clone()
        torch.cuda.synchronize()
        print(f"copy calibration: fill + copy of {x.numel() * 4} bytes", file=sys.stderr, flush=True)
        del x, y

    import paper_2101_11157_amd as wv

    if args.config == "batch":
        return bench_batch(args, wv)
    if args.config == "serve":
        return bench_serve(args, wv)
    if args.config == "irregular":
        return bench_irregular(args, wv)
    if args.config == "peak":
        return bench_peak(args)

    lo0, hi0, wdef = CONFIGS[args.config]
    W = args.window or wdef
    nwin = args.warmup + args.steps
    if lo0 + nwin * W > hi0 and args.config != "1e5":
        print(f"bench.py: {nwin} windows of {W} do not fit in [{lo0}, {hi0})", file=sys.stderr)
        sys.exit(2)
    from paper_2101_11157_amd import workloads
    wins = workloads.bench_windows(nwin, W, lo0, hi0) if args.config != "1e5" else [(lo0, hi0)] * nwin

    m = measure_plain(args, wv, wins, lo0, hi0, W)
    value = m["primes"] / m["wall"]
    # the next 8 sub-windows (work the timed steps did not do) for the
    # batched-against-plain comparison at the headline's size
    wins_extra = (workloads.bench_windows(nwin + 8, W, lo0, hi0)[nwin:]
                  if args.config == "1e11" and lo0 + (nwin + 8) * W <= hi0 else [])
    achieved = m["ops"] / (m["ms_sum"] * 1e-3) / 1e12
    achieved_terms = m["ops_terms"] / (m["ms_sum"] * 1e-3) / 1e12
    peak = PEAK_VALU / 1e12
    mul_rate = m["muls"] / (m["ms_sum"] * 1e-3) / 1e12
    block = m["block"]
    traffic_key = (args.config, tables_key(args.tables, hi0 - 1), block[0], block[1], W, kernel_source_hash())
    line = {
        "metric": "primes tested/sec at p~1e11 (1 GPU), both B_{p-3} and E_{p-3} mod p",
        "value": value,
        "unit": "primes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_V100_PRIMES_PER_S if args.config == "1e11" else None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"primes in [{lo0}, {hi0}), sub-windows of {W} integers per step",
            "tables": m["tables"],
            "primes_timed": m["primes"],
            "terms_timed": m["terms"],
            "terms_per_s": m["terms"] / m["wall"],
            "sum_kernel_ms": m["ms_sum"],
            "device_ms": m["ms_dev"],
            "block": block,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "Tops/s (full-rate VALU lane ops)",
            "frac": achieved / peak,
            "achieved_terms_only": achieved_terms,
            "frac_terms_only": achieved_terms / peak,
            "traffic": MEASURED_TRAFFIC.get(traffic_key),
            "traffic_source": ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source on this window, scaled "
                               "by a copy of known size (profile constant)" if traffic_key in MEASURED_TRAFFIC
                               else "not measured for this kernel source / configuration"),
        },
    }
    # the multiply view: the blocked loop needs few multiplies per term, so
    # this fraction is low although the kernel is bound by VALU issue
    line["multiply_ops"] = {"achieved": mul_rate, "peak": peak, "unit": "Tops/s", "frac": mul_rate / peak}

    if args.config == "1e11" and not args.no_batch and not args.no_same_work:
        line["batched_1e11"] = same_windows_batched(args, wv, wins_extra)
    if args.config == "1e11" and not args.no_batch:
        b = measure_batch(args, wv, args.windows)
        line["batched"] = dict({"workload": b["workload"], "tables": b["tables"], "block": b["block"]},
                               **rate_summary(b["primes"], b["terms"], b["ops"], b["wall"], b["ms_sum"]))
        if not args.no_same_work:
            v, w, same = per_window_plain(args, wv, b["wins"], b["results"])
            line["batched"]["per_window_plain"] = {
                "primes_per_s": v, "wall_s": w, "identical_results": same,
                "batched_over_per_window": line["batched"]["primes_per_s"] / v,
                "how": "the same 64 windows, one wv_search_range call each, in order"}
    if args.config == "1e11" and not args.no_serve:
        from paper_2101_11157_amd import workloads as wl
        trace = wl.serve_trace(0, args.requests, rate=args.rate)
        ctx = wv.Context(0)
        use_tables(ctx, args.tables)
        sv, sv_out = run_trace(wv, ctx, trace, args.step_terms, args.tables)
        ctx.close()
        served = {"workload": f"seeded Poisson trace (default_rng(0)), {len(trace)} requests at {args.rate:g}/s, "
                              f"70% single primes, 30% intervals of 1e2..1e5, u in [1e8, 1e11]",
                  "p50_ms": sv["p50_ms"], "p99_ms": sv["p99_ms"], "mean_ms": sv["mean_ms"],
                  "primes_per_s": sv["value"], "terms_per_s": sv["terms"] / sv["wall_s"],
                  "capacity_terms_per_s": sv["capacity_terms_per_s"],
                  "offered_over_capacity": sv["offered_over_capacity"], "primes": sv["primes"],
                  "terms": sv["terms"], "wall_s": sv["wall_s"], "busy_s": sv["busy_s"], "steps": sv["steps"],
                  "valu_tops": sv["valu_tops"], "frac": sv["frac"]}
        if not args.no_same_work:
            v, w, same = requests_alone(args, wv, trace, sv_out)
            served["alone_plain"] = {
                "primes_per_s": v, "wall_s": w, "identical_results": same,
                "served_over_alone": sv["value"] / v,
                "how": "the same 128 requests through the plain path one at a time, all available at once"}
        line["served"] = served
    if "batched" in line or "served" in line:
        # against the headline window (other primes and congruences): the
        # term-sum kernel's modelled VALU rate and terms/s (ops per term differ
        # between the Bernoulli and Euler sides and with p, and each rung of the
        # derived ladder trades terms for sums, so terms/s depends on the mix);
        # the same work through the plain path is in per_window_plain /
        # alone_plain above
        line["vs_plain"] = {k: {"frac_ratio": line[k]["frac"] / line["roofline"]["frac"],
                                "terms_per_s_ratio": line[k]["terms_per_s"] / line["config"]["terms_per_s"]}
                            for k in ("batched", "served") if k in line}

    if not args.no_cpu_baseline and m["results"]:
        first = m["results"][0]
        k = max(1, args.cpu_primes)
        idx = [int(round(i * (len(first) - 1) / max(1, k - 1))) for i in range(k)] if len(first) > 1 else [0]
        sample = [int(first["p"][i]) for i in sorted(set(idx))]
        gpu = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in first}
        nt = cpu_threads()
        v, dt, got = cpu_baseline(sample, nt)
        cb, ce = table_cost(args.tables, hi0 - 1)
        match = all(gpu[p] == g for p, g in zip(sample, got))
        line["cpu_baseline"] = {
            "value": v, "unit": "primes/s", "cores": nt, "kind": "oracle",
            "sample": f"{len(sample)} primes spread over the first timed window ({sample[0]}..{sample[-1]}), "
                      f"eqnBB30+eqnEE33 evaluated plainly (each sum split over {nt} threads), {dt:.1f} s; "
                      f"residues {'identical to' if match else 'DIFFERENT from'} the GPU's",
            "cpu_model": cpu_model(),
            "residues_match_gpu": match,
            "terms_per_prime_ratio_oracle_over_gpu": (227 / 6480 + 27 / 512) / (cb + ce),
        }
    print(json.dumps(line), flush=True)


def mfma_f64_attained():
    """f64 matrix flops per second that independent back-to-back
    v_mfma_f64_16x16x4_f64 operations attain (libwvpeak.so); None if the
    library is not built."""
    import ctypes
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2101_11157_amd", "libwvpeak.so")
    if not os.path.exists(path):
        return None
    L = ctypes.CDLL(path)
    L.wv_peak_mfma_f64.restype = ctypes.c_int
    L.wv_peak_mfma_f64.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    v = ctypes.c_double(0.0)
    return v.value if L.wv_peak_mfma_f64(0, ctypes.byref(v)) == 0 else None


# one (s, t) pair of the all-exponent power sums on the matrix cores: one f64
# multiply-add (2 flops) of the power tables s^(t0 + 2N m) and s^(2j)
FLOPS_IRR_PAIR = 2
# the same pair on the vector ALU: an exact modular product (5 lane operations)
# and an exact addition (2)
OPS_IRR_PAIR_VALU = 7
PEAK_MFMA_F64 = 78.6e12                  # dense f64 matrix peak of MI355X


def bench_irregular(args, wv):
    """Irregular-pair census: every B_{2k} and E_{2k} mod p (2k <= p - 3) of the
    primes in [2^15, 2^16), a step being the next window of `--window` (default
    4096) integers; the pairs found are compared with the oracle on the first
    timed window's smallest primes.  `roofline` describes the power-sum kernel
    on the matrix cores (one f64 multiply-add per (s, t) pair)."""
    import numpy as np
    lo0, hi0 = 1 << 15, 1 << 16
    W = args.window or 4096
    nwin = args.warmup + args.steps
    if lo0 + nwin * W > hi0:
        print(f"bench.py: {nwin} windows of {W} do not fit in [{lo0}, {hi0})", file=sys.stderr)
        sys.exit(2)
    wins = [(lo0 + k * W, lo0 + (k + 1) * W) for k in range(nwin)]
    ctx = wv.Context(0)
    ctx.set_irregular_path({"auto": 0, "valu": 1, "mfma": 2}[args.irr_path])
    attained = mfma_f64_attained() if args.irr_path != "valu" else None
    for k in range(args.warmup):
        ctx.irregular_pairs(*wins[k])
        print(f"warmup {k}: window {wins[k]}", file=sys.stderr, flush=True)
    primes = npairs = 0
    pairs_st = 0.0
    ms_sum = 0.0
    first = None
    t0 = time.perf_counter()
    for k in range(args.warmup, nwin):
        got, n, unresolved = ctx.irregular_pairs(*wins[k])
        st = ctx.stats()
        primes += n
        npairs += len(got)
        pairs_st += st["n_terms"]
        ms_sum += st["ms_sum"]
        if first is None:
            first = (wins[k], got)
        print(f"step {k - args.warmup}: {n} primes, {len(got)} pairs, unresolved {unresolved}, "
              f"power-sum kernel {st['ms_sum']:.1f} ms", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    ctx.close()
    value = primes / wall
    achieved = FLOPS_IRR_PAIR * pairs_st / (ms_sum * 1e-3) / 1e12
    line = {
        "metric": "primes/s with every irregular and E-irregular pair (all 2k <= p-3), p in [2^15, 2^16) (1 GPU)",
        "value": value,
        "unit": "primes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"primes in [{lo0}, {hi0}), windows of {W} integers per step",
            "primes_timed": primes,
            "pairs_found": npairs,
            "power_sum_terms": pairs_st,
            "power_sum_kernel_ms": ms_sum,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_MFMA_F64 / 1e12,
            "unit": "TFLOP/s (f64 matrix)",
            "frac": achieved / (PEAK_MFMA_F64 / 1e12),
            "traffic": None,
        },
    }
    if attained:
        # context for the published peak: what back-to-back independent f64
        # matrix operations attain on this device
        line["mfma_f64_attained"] = {"value": attained / 1e12, "unit": "TFLOP/s",
                                     "frac": achieved / (attained / 1e12)}
    if args.irr_path == "valu":
        # the vector kernel: one exact modular product and one exact addition
        # (OPS_IRR_PAIR_VALU lane operations) per (s, t) pair on the VALU
        ops = OPS_IRR_PAIR_VALU * pairs_st / (ms_sum * 1e-3) / 1e12
        line["roofline"] = {"bound": "alu", "achieved": ops, "peak": PEAK_VALU / 1e12,
                            "unit": "Tops/s (full-rate VALU lane ops)", "frac": ops / (PEAK_VALU / 1e12),
                            "traffic": None}
        line["config"]["kernel"] = "vector ALU"
    if not args.no_cpu_baseline and first is not None:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        (wlo, whi), got = first
        nt = min(cpu_threads(), 16)
        sample = oracle.primes(wlo, whi)[:nt]
        t1 = time.perf_counter()
        with ThreadPoolExecutor(nt) as ex:
            want = [x for lst in ex.map(oracle.irregular_pairs, sample) for x in lst]
        dt = time.perf_counter() - t1
        have = [(int(r["p"]), int(r["two_k"]), int(r["kind"])) for r in got if int(r["p"]) <= sample[-1]]
        line["cpu_baseline"] = {
            "value": len(sample) / dt, "unit": "primes/s", "cores": len(sample), "kind": "oracle",
            "sample": f"the {len(sample)} smallest primes of the first timed window ({sample[0]}..{sample[-1]}), "
                      f"EGF recurrences mod p, one prime per thread, {dt:.1f} s; pairs "
                      f"{'identical' if have == sorted(want) else 'DIFFERENT'}",
        }
    print(json.dumps(line), flush=True)


def bench_batch(args, wv):
    """Uneven seeded windows (lengths log-uniform in [1e3, 1e6], starts in
    [1e6, 1e11], numpy default_rng(0)) in one batched call."""
    b = measure_batch(args, wv, args.windows)
    r = rate_summary(b["primes"], b["terms"], b["ops"], b["wall"], b["ms_sum"])
    print(json.dumps({
        "metric": "batched windows: primes tested/sec (1 GPU)", "value": r["primes_per_s"], "unit": "primes/s",
        "config": dict({"workload": b["workload"], "tables": b["tables"], "block": b["block"],
                        "verified_windows": b["n_verified"], "verified_identical": b["verified"]}, **r),
    }), flush=True)


def run_trace(wv, ctx, trace, step_terms, tables="derived"):
    """Submit each request at its arrival time, step the server, collect
    results; latency is measured from arrival."""
    srv = wv.Server(ctx, step_terms=step_terms)
    t0 = time.perf_counter()
    ids, arrive, lat, out = {}, {}, {}, {}
    nxt = 0
    last = t0
    primes = 0
    while len(lat) < len(trace):
        now = time.perf_counter() - t0
        while nxt < len(trace) and trace[nxt][0] <= now:
            at, kind, arg = trace[nxt]
            rid = srv.submit_primes([arg]) if kind == "prime" else srv.submit_range(*arg)
            ids[rid] = nxt
            arrive[rid] = (at, time.perf_counter() - t0)
            nxt += 1
        srv.step()
        for rid in list(ids):
            if rid in lat:
                continue
            r = srv.result(rid)
            if r is not None:
                res, server_ms = r
                at, sub = arrive[rid]
                lat[rid] = server_ms + (sub - at) * 1e3     # from arrival, not from submission
                out[ids[rid]] = res
                primes += len(res)
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            st = srv.stats()
            print(f"serve: {len(lat)}/{len(trace)} done, active {st['active']}, pending {st['pending']}",
                  file=sys.stderr, flush=True)
        if nxt < len(trace) and not srv.stats()["active"] and not srv.stats()["pending"]:
            time.sleep(max(0.0, min(0.01, trace[nxt][0] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    served = [int(p) for res in out.values() for p in res["p"]]
    # the server's steps pick their own chunk sizes; at these sizes nearly
    # every sum is one chunk whatever the size, so a nominal 2^18 stands in
    ops = OpsModel(tables, st["block_k_b"], st["block_k_e"]).ops(served, st["terms_done_b"], st["terms_done"],
                                                                 chunk=1 << 18)
    valu = ops / st["sum_s"] / 1e12 if st["sum_s"] > 0 else 0.0
    v = sorted(lat.values())
    pct = lambda q: v[min(len(v) - 1, int(round(q * (len(v) - 1))))]
    span = trace[-1][0] if trace else 0.0
    capacity = st["terms_done"] / st["busy_s"] if st["busy_s"] > 0 else 0.0
    offered = st["terms_done"] / span if span > 0 else float("inf")
    summary = {"value": primes / wall, "p50_ms": pct(0.5), "p99_ms": pct(0.99), "mean_ms": sum(v) / len(v),
               "max_ms": v[-1], "requests": len(trace), "primes": primes, "terms": st["terms_done"],
               "wall_s": wall, "busy_s": st["busy_s"], "steps": st["steps"], "offered_terms_per_s": offered,
               "capacity_terms_per_s": capacity, "offered_over_capacity": offered / capacity if capacity else None,
               "sum_kernel_s": st["sum_s"], "valu_tops": valu, "frac": valu / (PEAK_VALU / 1e12)}
    return summary, out


def bench_serve(args, wv):
    """Seeded Poisson trace of single primes and intervals through the request
    server; arrivals submitted at their times, latency from arrival.  With
    --load f the same trace is replayed with its arrival times stretched so
    that the offered load is f x the capacity measured on the first run."""
    from paper_2101_11157_amd import workloads
    trace = workloads.serve_trace(0, args.requests, rate=args.rate)
    ctx = wv.Context(0)
    tables = use_tables(ctx, args.tables)
    main_run, out = run_trace(wv, ctx, trace, args.step_terms, args.tables)
    ok = None
    if args.verify:
        ok = True
        for k, (at, kind, arg) in enumerate(trace):
            alone = ctx.eval_primes([arg]) if kind == "prime" else ctx.search_range(*arg)[0]
            same = as_pairs(alone) == as_pairs(out[k])
            ok = ok and same
            if not same:
                print(f"verify request {k} ({kind} {arg}): DIFFERENT", file=sys.stderr, flush=True)
        print(f"verify: {len(trace)} requests against the same request alone: "
              f"{'identical' if ok else 'DIFFERENT'}", file=sys.stderr, flush=True)
    line = {
        "metric": "served queries: p50/p99 latency and primes tested/sec (1 GPU)", "value": main_run["value"],
        "unit": "primes/s", "p50_ms": main_run["p50_ms"], "p99_ms": main_run["p99_ms"],
        "mean_ms": main_run["mean_ms"],
        "config": dict({"workload": f"seeded Poisson trace (default_rng(0)), {len(trace)} requests, "
                                    f"{args.rate:g}/s, 70% single primes, 30% intervals of 1e2..1e5, "
                                    f"u in [1e8, 1e11]", "tables": tables, "verified_identical": ok}, **main_run),
    }
    if args.load:
        per_req = main_run["terms"] / len(trace)
        rate = args.load * main_run["capacity_terms_per_s"] / per_req
        print(f"supplementary run: {rate:.3f} requests/s ({args.load:g} x capacity)", file=sys.stderr, flush=True)
        sup, _ = run_trace(wv, ctx, workloads.serve_trace(0, args.requests, rate=rate), args.step_terms, args.tables)
        line["supplementary"] = dict({"rate_per_s": rate, "load": args.load}, **sup)
    ctx.close()
    print(json.dumps(line), flush=True)


def as_pairs(res):
    return [(int(r["p"]), int(r["b"]), int(r["e"])) for r in res]


if __name__ == "__main__":
    main()
