"""GPU parity: the HIP path (through the C ABI) against the CPU oracle and the
paper's printed values.  Bit-exact: every residue is an integer in [0, p)."""
import functools
import json
import os
import random
import sys

import numpy as np
import pytest

import paper_2101_11157_amd as wv
import oracle
from oracle import exact
from conftest import GOLDEN, read_golden

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not os.path.exists(wv.LIB_PATH):
        pytest.fail("libwvprime.so is not built: the HIP path must be present on a GPU box")
    c = wv.Context(0)
    yield c
    c.close()


def golden_json(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def as_pairs(res):
    return [(int(r["b"]), int(r["e"])) for r in res]


def check_against_oracle(res, method="root"):
    ps = [int(p) for p in res["p"]]
    want = oracle.residues(ps, method=method)
    got = as_pairs(res)
    bad = [(p, g, w) for p, g, w in zip(ps, got, want) if g != w]
    assert not bad, f"{len(bad)} mismatches, first {bad[:5]}"
    for r, (b, e) in zip(res, want):
        f = (1 if b == 0 else 0) | (2 if e == 0 else 0)
        assert int(r["flags"]) == f


def test_small_window_all_primes(ctx):
    """All primes 5 <= p < 1e5 (9590 primes) against the oracle, and the hits."""
    say("case: search_range(5, 1e5)")
    res, hits = ctx.search_range(5, 10 ** 5)
    assert len(res) == 9590
    assert list(res["p"]) == oracle.primes(5, 10 ** 5)
    check_against_oracle(res)
    assert list(hits) == [149, 241, 16843]
    st = ctx.stats()
    assert st["n_primes"] == 9590 and st["ms_sum"] > 0


def test_wide_window_cut_into_sub_ranges(ctx):
    """A window at 3e10 holding about three sub-ranges of the size the library
    cuts windows into there (about half a search batch of work each): every
    prime once, ascending, and 64 sampled results (first, middle and last
    included) identical to the same primes evaluated as a list."""
    lo, hi = 3 * 10 ** 10, 3 * 10 ** 10 + 400_000
    say(f"case: search_range({lo}, {hi}), cut into sub-ranges")
    res, hits = ctx.search_range(lo, hi)
    assert list(res["p"]) == oracle.primes(lo, hi)
    idx = sorted(set([0, len(res) // 2, len(res) - 1] + random.Random(7).sample(range(len(res)), 61)))
    alone = ctx.eval_primes(np.array([int(p) for p in res["p"][idx]], dtype=np.uint64))
    assert as_pairs(res[idx]) == as_pairs(alone)
    assert [int(f) for f in res["flags"][idx]] == [int(f) for f in alone["flags"]]
    assert list(hits) == [int(r["p"]) for r in res if int(r["flags"])]


def test_paper_tables_2_and_3(ctx):
    """Printed symmetric residues of Tables 2 and 3 (43 primes up to 7.8e10)."""
    say("case: Tables 2 and 3")
    for name, key in (("near_miss_B.txt", "b"), ("near_miss_E.txt", "e")):
        rows = [(int(p), int(r)) for p, r in read_golden(name)]
        res = ctx.eval_primes([p for p, _ in rows])
        for (p, r), out in zip(rows, res):
            assert int(out["p"]) == p
            assert wv.symmetric(out[key], p) == r, (name, p, int(out[key]))


def test_theorem_1_1_hits(ctx):
    say("case: Theorem 1.1 primes")
    rows = read_golden("known_primes.txt")
    ps = sorted({int(p) for _, p in rows})
    res = {int(r["p"]): r for r in ctx.eval_primes(ps)}
    for kind, p in rows:
        f = int(res[int(p)]["flags"])
        if kind == "wolstenholme":
            assert f & wv.WV_FLAG_WOLSTENHOLME, p
        elif kind == "vandiver":
            assert f & wv.WV_FLAG_VANDIVER, p
        elif kind == "not_vandiver":
            assert not f & wv.WV_FLAG_VANDIVER, p


def test_small_search_graph_replays(ctx):
    """A small single-window search runs as one replayed graph sized by a
    prime-count bound: [5, 1e5) replayed three times with other work on the
    context between the replays (an evaluation, a search that captures a graph
    of another size, a search on the counted path) gives the oracle's primes
    and residues every time."""
    say("case: search graph replays")
    ps = oracle.primes(5, 10 ** 5)
    first, hits = ctx.search_range(5, 10 ** 5)
    assert [int(p) for p in first["p"]] == ps
    assert ctx.stats()["n_primes"] == len(ps) and ctx.stats()["n_terms"] > 0
    sample = ps[::97]
    by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in first}
    assert [by_p[p] for p in sample] == oracle.residues(sample)
    assert sorted(int(h) for h in hits) == [149, 241, 16843]   # E_{p-3} == 0 at 149, 241; B_{p-3} == 0 at 16843
    other_lo, other_hi = 10 ** 6, 10 ** 6 + 3000
    big_lo, big_hi = 10 ** 9, 10 ** 9 + 2 ** 18        # enough work for the counted path
    for k in range(3):
        ev = ctx.eval_primes(oracle.primes(10 ** 6, 10 ** 6 + 300))
        assert np.all(ev["flags"] != 0xFFFFFFFF)
        other, _ = ctx.search_range(other_lo, other_hi)
        assert [int(p) for p in other["p"]] == oracle.primes(other_lo, other_hi)
        if k == 1:
            big, _ = ctx.search_range(big_lo, big_hi)
            assert len(big) == ctx.count_primes(big_lo, big_hi)
        again, _ = ctx.search_range(5, 10 ** 5)
        assert as_pairs(again) == as_pairs(first), k
        assert [int(p) for p in again["p"]] == ps


def test_smallest_primes_and_edges(ctx):
    say("case: p = 5 .. 101 and argument edges")
    ps = oracle.primes(5, 102)
    res = ctx.eval_primes(ps)
    assert as_pairs(res) == [(oracle.bernoulli_rec(p), oracle.euler_rec(p)) for p in ps]
    assert as_pairs(res[:2]) == [(1, 1), (3, 5)]
    r, _ = ctx.search_range(0, 20)
    assert list(r["p"]) == [5, 7, 11, 13, 17, 19]
    assert len(ctx.search_range(24, 29)[0]) == 0        # no prime in [24, 29)
    assert len(ctx.search_range(5, 5)[0]) == 0
    assert len(ctx.eval_primes([])) == 0
    # short output buffer
    with pytest.raises(wv.WvError) as ei:
        ctx.search_range(5, 100, cap=3)
    assert ei.value.status == wv.WV_ETRUNC
    for bad, code in (([3], wv.WV_EDOMAIN), ([2 ** 40 + 15], wv.WV_EDOMAIN), ([9], wv.WV_ENOTPRIME),
                      ([1000003 * 1000033], wv.WV_ENOTPRIME)):
        with pytest.raises(wv.WvError) as ei:
            ctx.eval_primes(bad)
        assert ei.value.status == code
    with pytest.raises(wv.WvError) as ei:
        ctx.count_primes(10, 5)
    assert ei.value.status == wv.WV_EINVAL
    with pytest.raises(wv.WvError) as ei:
        ctx.count_primes(0, 2 ** 40 + 1)
    assert ei.value.status == wv.WV_EDOMAIN


def test_ragged_batches(ctx):
    """Batch sizes that leave partial waves and workgroups; input order kept."""
    say("case: ragged batches")
    pool = oracle.primes(10 ** 6, 10 ** 6 + 40000)
    rng = random.Random(3)
    for n in (1, 63, 65, 257, 1000):
        ps = rng.sample(pool, n)
        res = ctx.eval_primes(ps)
        assert [int(x) for x in res["p"]] == ps
        check_against_oracle(res)


@pytest.mark.parametrize("chunk", [64, 192, 4096, 1 << 20, 1 << 30])
def test_chunk_size_invariance(ctx, chunk):
    say(f"case: chunk {chunk}")
    ps = oracle.primes(10 ** 7, 10 ** 7 + 3000) + [1025793739, 73607557631]
    ref = ctx.eval_primes(ps)
    try:
        ctx.set_chunk_terms(chunk)
        got = ctx.eval_primes(ps)
    finally:
        ctx.set_chunk_terms(0)
    assert as_pairs(got) == as_pairs(ref)


def test_first_sum_spans_many_waves(ctx):
    """Regression: a batch whose very first sum covers far more than 64 chunks
    (every wave of it takes the single-sum butterfly path from chunk 0 on).
    The term-sum loop once read its wave-uniform chunk base through a vector
    shuffle, and the compiler's per-lane loop split then left lanes 1..63
    re-reading a stale base from the parked lane 0 forever."""
    say("case: first sum of 14k chunks")
    ps = [1000000007, 1000000009]
    try:
        ctx.set_chunk_terms(64)
        got = ctx.eval_primes(ps)
        st = ctx.stats()
    finally:
        ctx.set_chunk_terms(0)
    assert st["chunk_terms"] == 64 and st["n_chunks"] > 64 * 63
    assert as_pairs(got) == oracle.residues(ps, method="table")


@pytest.mark.parametrize("shape", wv.BLOCK_SHAPES)
def test_block_shape_invariance(ctx, shape):
    """Every compiled block shape of the term-sum kernel gives the same residues
    (long chunks take the blocked path, segment tails the one-term path)."""
    say(f"case: block shape {shape}")
    ps = oracle.primes(10 ** 8, 10 ** 8 + 400)[:20] + [11, 101, 1000003, 9999999967, 73607557631]
    want = oracle.residues(ps[:22]) 
    try:
        ctx.set_block(*shape)
        got = ctx.eval_primes(ps)
        st = ctx.stats()
        ctx.set_chunk_terms(4096)
        got2 = ctx.eval_primes(ps)
    finally:
        ctx.set_block(8, 8)
        ctx.set_chunk_terms(0)
    assert (st["block_k_b"], st["block_k_e"]) == shape
    assert as_pairs(got)[:22] == want
    assert as_pairs(got2) == as_pairs(got)
    ref = golden_residues_paper()
    for (p, key, r) in ref:
        if p in ps:
            assert wv.symmetric(got[ps.index(p)][key], p) == r


def golden_residues_paper():
    out = []
    for name, key in (("near_miss_B.txt", "b"), ("near_miss_E.txt", "e")):
        out += [(int(p), key, int(r)) for p, r in read_golden(name)]
    return out


def test_cross_table_agreement(ctx):
    """Every Bernoulli table with every Euler table gives the same residues."""
    say("case: cross-table agreement")
    ps = oracle.primes(11, 3000)[::7] + oracle.primes(10 ** 8, 10 ** 8 + 2000)[:40] + [16843, 2124679]
    ref = None
    try:
        for b in ("BB1", "BB2", "BB6", "BB9", "BB16", "BB22", "BB30"):
            for e in ("EE3", "EE5", "EE9", "EE16", "EE24", "EE33"):
                ctx.set_tables(b, e)
                got = as_pairs(ctx.eval_primes(ps))
                if ref is None:
                    ref = got
                assert got == ref, (b, e)
    finally:
        ctx.set_tables("BB30", "EE33")
    assert ref == oracle.residues(ps)


def test_window_1e9_sample(ctx):
    """Seeded sample of the primes in [1e9, 1e9 + 1e7) against stored oracle values."""
    g = golden_json("window_1e9.json")
    say(f"case: window 1e9, {len(g['rows'])} sampled primes")
    ps = [r["p"] for r in g["rows"]]
    res = ctx.eval_primes(ps)
    assert as_pairs(res) == [(r["b"], r["e"]) for r in g["rows"]]
    assert ctx.count_primes(g["lo"], g["hi"]) == g["n_primes"]


def test_window_1e9_search_subwindow(ctx):
    """The sieve and the whole path on [1e9, 1e9 + 2^19): primes equal the plain
    sieve's, stored samples inside it match, and a fresh oracle sample matches."""
    lo, hi = 10 ** 9, 10 ** 9 + (1 << 19)
    say(f"case: search_range({lo}, {hi})")
    res, _ = ctx.search_range(lo, hi)
    assert [int(p) for p in res["p"]] == oracle.primes(lo, hi)
    g = golden_json("window_1e9.json")
    by_p = {int(r["p"]): r for r in res}
    inside = [r for r in g["rows"] if r["p"] < hi]
    assert inside
    for r in inside:
        assert (int(by_p[r["p"]]["b"]), int(by_p[r["p"]]["e"])) == (r["b"], r["e"])
    pick = random.Random(5).sample(list(range(len(res))), 6)
    check_against_oracle(res[sorted(pick)], method="table")


def test_window_1e11_sample(ctx):
    """Seeded sample of [1e11 - 1e6, 1e11) (p < 2^37) against stored oracle values."""
    g = golden_json("window_1e11.json")
    say(f"case: window 1e11, {len(g['rows'])} sampled primes")
    ps = [r["p"] for r in g["rows"]]
    res = ctx.eval_primes(ps)
    assert as_pairs(res) == [(r["b"], r["e"]) for r in g["rows"]]
    assert ctx.count_primes(g["lo"], g["hi"]) == g["n_primes"]


def test_top_of_range_sums(ctx):
    """Largest primes below 2^40: single sums against stored oracle values."""
    g = golden_json("sums_2p40.json")
    ps = sorted({r["p"] for r in g["rows"]})
    say(f"case: sums at {ps}")
    nb, ne = wv.table_info("BB30")[0], wv.table_info("EE33")[0]
    sb, se = ctx.eval_sums(ps, nb, ne)
    for r in g["rows"]:
        i = ps.index(r["p"])
        got = sb[i, r["term"]] if r["table"] == "BB30" else se[i, r["term"]]
        assert int(got) == r["S"], r


def test_sums_small_primes_direct(ctx):
    """Per-sum values for small primes against sums of inverses written out."""
    ps = oracle.primes(11, 400) + [10007, 65537]
    nb, ne = wv.table_info("BB30")[0], wv.table_info("EE33")[0]
    sb, se = ctx.eval_sums(ps, nb, ne)
    from oracle import congruences as C
    for i, p in enumerate(ps):
        for cong, arr in ((C.BB30, sb), (C.EE33, se)):
            for j, (_, x, y) in enumerate(cong.terms):
                lo, hi = oracle.interval(p, x, y)
                assert int(arr[i, j]) == oracle.sum_direct(p, lo, hi, -cong.ell), (p, cong.name, j)


class Hip:
    """Minimal HIP runtime calls through ctypes (the runtime the library already loaded)."""

    def __init__(self):
        import ctypes
        self.ct = ctypes
        wv.lib()
        self.h = ctypes.CDLL("libamdhip64.so.7")
        self.h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.h.hipFree.argtypes = [ctypes.c_void_p]
        self.h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.h.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.h.hipStreamDestroy.argtypes = [ctypes.c_void_p]

    def malloc(self, n):
        p = self.ct.c_void_p()
        assert self.h.hipMalloc(self.ct.byref(p), n) == 0
        return p.value

    def h2d(self, dst, arr):
        assert self.h.hipMemcpy(dst, arr.ctypes.data, arr.nbytes, 1) == 0

    def d2h(self, arr, src):
        assert self.h.hipMemcpy(arr.ctypes.data, src, arr.nbytes, 2) == 0


def test_async_device_pointers(ctx):
    """Device-pointer entry point on a caller's stream equals the host entry point,
    including a rejected input (flags 0xFFFFFFFF) in the middle of the batch."""
    hip = Hip()
    ps = oracle.primes(3 * 10 ** 6, 3 * 10 ** 6 + 20000)
    ref = ctx.eval_primes(ps)
    arr = np.array(ps[:100] + [4] + ps[100:], dtype=np.uint64)
    d_in = hip.malloc(arr.nbytes)
    d_out = hip.malloc(arr.size * wv.RESULT_DTYPE.itemsize)
    st = hip.ct.c_void_p()
    assert hip.h.hipStreamCreate(hip.ct.byref(st)) == 0
    try:
        hip.h2d(d_in, arr)
        ctx.eval_primes_async(d_in, arr.size, d_out, st.value)
        assert hip.h.hipStreamSynchronize(st) == 0
        got = np.zeros(arr.size, dtype=wv.RESULT_DTYPE)
        hip.d2h(got, d_out)
    finally:
        hip.h.hipStreamDestroy(st)
        hip.h.hipFree(d_in)
        hip.h.hipFree(d_out)
    assert int(got[100]["flags"]) == 0xFFFFFFFF
    got = np.concatenate([got[:100], got[101:]])
    assert [int(x) for x in got["p"]] == ps
    assert as_pairs(got) == as_pairs(ref)
    assert list(got["flags"]) == list(ref["flags"])


TORCH_INTEROP = r"""
import sys, numpy as np
import torch                      # torch first: one HIP runtime in the process
assert torch.cuda.is_available(), "torch sees no GPU"
sys.path.insert(0, sys.argv[1])
import paper_2101_11157_amd as wv, oracle
ps = oracle.primes(3 * 10 ** 6, 3 * 10 ** 6 + 5000)
with wv.Context(0) as ctx:
    ref = ctx.eval_primes(ps)
    d_in = torch.tensor(np.array(ps, dtype=np.int64), device="cuda:0")
    d_out = torch.zeros((len(ps), 4), dtype=torch.int64, device="cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.eval_primes_async(d_in.data_ptr(), len(ps), d_out.data_ptr(), s.cuda_stream)
    s.synchronize()
    got = d_out.cpu().numpy().view(np.uint64)
    assert [int(x) for x in got[:, 0]] == ps
    assert [(int(b), int(e)) for b, e in got[:, 1:3]] == [(int(r["b"]), int(r["e"])) for r in ref]
print("torch interop ok")
"""


def test_torch_stream_interop():
    """torch tensors and a torch stream as the async entry point's memory and stream
    (a fresh process that imports torch before the library)."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    probe = subprocess.run([sys.executable, "-c", "import torch; print(torch.cuda.is_available())"],
                           capture_output=True, text=True, timeout=300)
    if probe.stdout.strip() != "True":
        pytest.skip("torch does not see the GPU in this environment: " + (probe.stdout + probe.stderr)[-300:])
    r = subprocess.run([sys.executable, "-c", TORCH_INTEROP, root], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "torch interop ok" in r.stdout


def test_determinism_repeat(ctx):
    ps = oracle.primes(10 ** 10, 10 ** 10 + 1500)
    a = ctx.eval_primes(ps)
    b = ctx.eval_primes(ps)
    assert as_pairs(a) == as_pairs(b)


def test_paper_prime_count(ctx):
    """Section 3, Results: 4118054811 primes p with 5 <= p < 1e11."""
    say("case: count_primes(5, 1e11)")
    assert ctx.count_primes(5, 10 ** 11) == 4118054811
    c = golden_json("counts.json")
    for k, v in c.items():
        lo, hi = map(int, k.split(","))
        assert ctx.count_primes(lo, hi) == v, k


# ---------------------------------------------------------------------------
# batched windows, split launches, graphs, autotuner
# ---------------------------------------------------------------------------


def test_search_windows_equals_plain_path(ctx):
    """Uneven windows in one batched call give, window by window, exactly the
    plain per-window results (seeded draw; shorter windows than the full
    workload so that the plain path can be run beside it)."""
    from paper_2101_11157_amd import workloads
    wins = workloads.batch_windows(0, 24, len_range=(1e2, 2e3))
    wins += [(5, 5), (24, 29), (10 ** 9, 10 ** 9 + 300), (10 ** 9 + 100, 10 ** 9 + 200)]   # empty, overlapping
    say(f"case: search_windows over {len(wins)} windows")
    got = ctx.search_windows([a for a, _ in wins], [b for _, b in wins])
    st = ctx.stats()
    assert len(got) == len(wins)
    total = 0
    for (a, b), res in zip(wins, got):
        ref, _ = ctx.search_range(a, b)
        assert [int(p) for p in res["p"]] == [int(p) for p in ref["p"]] == oracle.primes(max(a, 5), b)
        assert as_pairs(res) == as_pairs(ref)
        total += len(res)
    assert st["n_primes"] == total
    # and a sample against the oracle
    flat = np.concatenate([g for g in got if len(g)])
    pick = sorted(random.Random(9).sample(range(len(flat)), 5))
    check_against_oracle(flat[pick], method="table")


def test_split_launches_with_progress(ctx):
    """Term sums cut into many launches with a progress callback: same residues."""
    ps = oracle.primes(10 ** 9, 10 ** 9 + 3000)
    ref = ctx.eval_primes(ps)
    seen = []
    try:
        ctx.set_progress(lambda d, t: seen.append((d, t)), terms_per_launch=1 << 30)
        got = ctx.eval_primes(ps)
    finally:
        ctx.set_progress(None)
    assert len(seen) > 3
    assert all(b[0] > a[0] for a, b in zip(seen, seen[1:])) and seen[-1][0] == seen[-1][1]
    assert as_pairs(got) == as_pairs(ref)


def test_async_graph_replays(ctx):
    """The device-pointer entry point replays captured graphs: several replays of
    one size, another size in between, eager calls and syncs between them; every
    replay equals the eager host-pointer result."""
    hip = Hip()
    pools = [oracle.primes(10 ** 7, 10 ** 7 + 9000), oracle.primes(2 * 10 ** 8, 2 * 10 ** 8 + 3000)]
    st = hip.ct.c_void_p()
    assert hip.h.hipStreamCreate(hip.ct.byref(st)) == 0
    bufs = []
    try:
        for rep in range(3):
            for ps in pools:
                arr = np.array(ps, dtype=np.uint64)
                ref = ctx.eval_primes(ps)                       # eager, between replays
                d_in = hip.malloc(arr.nbytes)
                d_out = hip.malloc(arr.size * wv.RESULT_DTYPE.itemsize)
                bufs += [d_in, d_out]
                hip.h2d(d_in, arr)
                ctx.eval_primes_async(d_in, arr.size, d_out, st.value)
                assert hip.h.hipStreamSynchronize(st) == 0
                got = np.zeros(arr.size, dtype=wv.RESULT_DTYPE)
                hip.d2h(got, d_out)
                assert [int(x) for x in got["p"]] == ps, rep
                assert as_pairs(got) == as_pairs(ref), rep
    finally:
        hip.h.hipStreamDestroy(st)
        for b in bufs:
            hip.h.hipFree(b)


def test_autotune_and_cache(ctx, tmp_path):
    say("case: autotune at 1e9")
    ps = oracle.primes(10 ** 9, 10 ** 9 + 2000)
    ref = ctx.eval_primes(ps)
    kb, ke, chunk, table = ctx.autotune(10 ** 9, n_sample=8)
    assert (kb, ke) in wv.BLOCK_SHAPES and chunk in (1 << 16, 1 << 18, 0)
    assert table[(kb, ke, chunk)] == max(table.values()) > 0
    got = ctx.eval_primes(ps)                                   # tuned shape in use
    assert as_pairs(got) == as_pairs(ref)
    path = tmp_path / "tune.txt"
    ctx.tune_save(str(path))
    line = path.read_text().split()
    assert line[0].startswith("gfx") and int(line[1]) == 29 and (int(line[2]), int(line[3])) == (kb, ke)
    with wv.Context(0) as c2:
        c2.tune_load(str(path))
        assert as_pairs(c2.eval_primes(ps)) == as_pairs(ref)
        assert (c2.stats()["block_k_b"], c2.stats()["block_k_e"]) == (kb, ke)


# ---------------------------------------------------------------------------
# request server
# ---------------------------------------------------------------------------


def drain(srv, ids, max_steps=100000):
    out = {}
    for _ in range(max_steps):
        for rid in list(ids):
            if rid in out:
                continue
            r = srv.result(rid)
            if r is not None:
                out[rid] = r
        if len(out) == len(ids):
            return out
        srv.step()
    raise AssertionError("server did not drain")


def test_server_mixed_requests_match_alone(ctx):
    """Singles and intervals submitted together and while others run: every
    request's residues equal the same request run alone."""
    say("case: server mixed requests")
    rng = random.Random(21)
    reqs = []
    for k in range(14):
        if rng.random() < 0.6:
            u = rng.randrange(10 ** 6, 10 ** 10)
            p = oracle.primes(u, u + 2000)[0]
            reqs.append(("primes", [p]))
        else:
            a = rng.randrange(10 ** 6, 10 ** 9)
            reqs.append(("range", (a, a + rng.randrange(100, 3000))))
    reqs.append(("primes", oracle.primes(10 ** 8, 10 ** 8 + 500)))
    reqs.append(("range", (24, 29)))                                  # no primes
    with wv.Server(ctx, step_terms=1 << 30) as srv:
        ids = []
        for i, (kind, arg) in enumerate(reqs):
            ids.append(srv.submit_primes(arg) if kind == "primes" else srv.submit_range(*arg))
            if i % 4 == 3:
                srv.step()                                            # arrivals while work runs
        res = drain(srv, ids)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    for (kind, arg), rid in zip(reqs, ids):
        got, lat = res[rid]
        alone = ctx.eval_primes(arg) if kind == "primes" else ctx.search_range(*arg)[0]
        assert [int(p) for p in got["p"]] == [int(p) for p in alone["p"]]
        assert as_pairs(got) == as_pairs(alone)
        assert lat > 0


def test_batch_windows_seed0_oracle_sample(ctx):
    """The 64 uneven windows of the batched workload (seed 0): every window's
    prime count, the oracle's residues of 4 primes per window, and the windows
    below 1e8 (the cheap ones) through one batched call."""
    from paper_2101_11157_amd import workloads
    g = golden_json("batch_seed0.json")
    wins = workloads.batch_windows(0, 64)
    assert [(w["lo"], w["hi"]) for w in g["windows"]] == wins
    say("case: batch seed 0, prime counts of 64 windows")
    for w in g["windows"]:
        assert ctx.count_primes(w["lo"], w["hi"]) == w["n_primes"], (w["lo"], w["hi"])
    rows = [r for w in g["windows"] for r in w["rows"]]
    say(f"case: batch seed 0, {len(rows)} sampled primes")
    res = ctx.eval_primes([r["p"] for r in rows])
    assert as_pairs(res) == [(r["b"], r["e"]) for r in rows]


def test_batch_windows_seed0_full_batch():
    """The whole batched workload (64 seeded windows, 429,833 primes, about
    4.3e14 terms with the derived congruences) in one wv_search_windows call,
    as the bench runs it: every window's prime list has the oracle's count and
    is ascending, and all 254 stored oracle residues (the first, last and two
    drawn primes of each window, fewer where they coincide) match."""
    from paper_2101_11157_amd import workloads
    g = golden_json("batch_seed0.json")
    wins = workloads.batch_windows(0, 64)
    say("case: batch seed 0, all 64 windows in one batched call (derived tables)")
    with wv.Context(0) as c:
        c.use_derived_tables()
        last = [0]

        def progress(done, total):
            if done * 10 >= (last[0] + 1) * total:
                last[0] = done * 10 // total
                say(f"  batch progress {done}/{total} chunks")

        c.set_progress(progress)
        got = c.search_windows([a for a, _ in wins], [b for _, b in wins])
    n_rows = 0
    for w, res in zip(g["windows"], got):
        assert len(res) == w["n_primes"], (w["lo"], w["hi"])
        ps = res["p"].astype(np.int64)
        assert np.all(np.diff(ps) > 0) and (len(ps) == 0 or (ps[0] >= w["lo"] and ps[-1] < w["hi"]))
        assert np.all(res["flags"] != 0xFFFFFFFF)
        by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in res}
        for r in w["rows"]:
            assert by_p[r["p"]] == (r["b"], r["e"]), r["p"]
            n_rows += 1
    assert n_rows == sum(len(w["rows"]) for w in g["windows"]) == 254


def test_window_1e11_whole_subwindow_two_table_sets():
    """The bench's first timed sub-window at the paper's ceiling,
    [1e11 - 1e6, 1e11 - 1e6 + 8192), in full with two independent congruence
    sets (the derived tables of thousands of sums and the printed eqnBB30 +
    eqnEE33: different intervals and coefficients): every prime's residues
    agree, the prime list is the plain sieve's, and the stored oracle values
    inside the window match."""
    lo, hi = 10 ** 11 - 10 ** 6, 10 ** 11 - 10 ** 6 + 8192
    say(f"case: whole window [{lo}, {hi}) with derived and printed tables")
    with wv.Context(0) as c:
        printed, _ = c.search_range(lo, hi)
        c.use_derived_tables()
        derived, _ = c.search_range(lo, hi)
    assert [int(p) for p in derived["p"]] == oracle.primes(lo, hi)
    assert len(derived) > 300
    assert as_pairs(derived) == as_pairs(printed)
    g = golden_json("window_1e11.json")
    by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in derived}
    inside = [r for r in g["rows"] if r["p"] < hi]
    assert inside
    for r in inside:
        assert by_p[r["p"]] == (r["b"], r["e"]), r["p"]


def test_serve_seed0_oracle_sample(ctx):
    """The 128-request serving trace (seed 0): the single primes and the
    cheaper intervals through the request server (results against the
    oracle's sample), every interval's prime count, and the oracle's sampled
    prime of each of the other intervals."""
    from paper_2101_11157_amd import workloads
    g = golden_json("serve_seed0.json")
    trace = workloads.serve_trace(0, 128)
    assert len(g["requests"]) == len(trace)
    served, rest = [], []
    for (t, kind, arg), q in zip(trace, g["requests"]):
        assert q["kind"] == kind
        if kind == "prime":
            assert q["p"] == arg
            served.append((kind, arg, q))
        else:
            assert (q["lo"], q["hi"]) == arg
            assert ctx.count_primes(*arg) == q["n_primes"], arg
            cost = 0.0878 * (arg[1] - arg[0]) * arg[0] / max(1.0, np.log(arg[0]))
            (served if cost < 2e12 else rest).append((kind, arg, q))
    say(f"case: serve seed 0, {len(served)} requests through the server, {len(rest)} sampled alone")
    with wv.Server(ctx, step_terms=1 << 36) as srv:
        ids = [srv.submit_primes([arg]) if kind == "prime" else srv.submit_range(*arg) for kind, arg, _ in served]
        res = drain(srv, ids)
    for (kind, arg, q), rid in zip(served, ids):
        got, _ = res[rid]
        if kind == "range":
            assert len(got) == q["n_primes"]
        by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in got}
        for r in q["rows"]:
            assert by_p[r["p"]] == (r["b"], r["e"]), r["p"]
    rows = [r for _, _, q in rest for r in q["rows"]]
    alone = ctx.eval_primes([r["p"] for r in rows])
    assert as_pairs(alone) == [(r["b"], r["e"]) for r in rows]


def test_serve_seed0_all_requests():
    """All 128 requests of the serving trace (seed 0, about 8.4e13 terms with
    the derived congruences) submitted together through the request server:
    every single prime's residues and every interval's prime count and
    sampled prime equal the stored oracle values."""
    from paper_2101_11157_amd import workloads
    g = golden_json("serve_seed0.json")
    trace = workloads.serve_trace(0, 128)
    say("case: serve seed 0, all 128 requests through the server (derived tables)")
    with wv.Context(0) as c:
        c.use_derived_tables()
        with wv.Server(c) as srv:
            ids = [srv.submit_primes([arg]) if kind == "prime" else srv.submit_range(*arg)
                   for _, kind, arg in trace]
            out = {}
            steps = 0
            while len(out) < len(ids):
                for rid in ids:
                    if rid not in out:
                        r = srv.result(rid)
                        if r is not None:
                            out[rid] = r
                if len(out) < len(ids):
                    srv.step()
                    steps += 1
                    if steps % 500 == 0:
                        say(f"  {steps} steps, {len(out)}/{len(ids)} done")
            st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == 128
    for (t, kind, arg), q, rid in zip(trace, g["requests"], ids):
        got, _ = out[rid]
        if kind == "range":
            assert len(got) == q["n_primes"], arg
        by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in got}
        for r in q["rows"]:
            assert by_p[r["p"]] == (r["b"], r["e"]), r["p"]


def test_server_restart_after_failed_step(ctx):
    """A step forced to fail (on the host) reports its error to the caller and
    restarts the active requests; the results are unchanged."""
    say("case: server fault injection")
    ps1 = oracle.primes(3 * 10 ** 9, 3 * 10 ** 9 + 400)
    with wv.Server(ctx, step_terms=1 << 31) as srv:
        srv.inject_fault(2)
        a = srv.submit_primes(ps1)
        b = srv.submit_range(10 ** 8, 10 ** 8 + 5000)
        errors = []
        out = {}
        for _ in range(100000):
            for rid in (a, b):
                if rid not in out:
                    r = srv.result(rid)
                    if r is not None:
                        out[rid] = r
            if len(out) == 2:
                break
            try:
                srv.step()
            except wv.WvError as e:
                errors.append(e.status)
        st = srv.stats()
    assert errors == [wv.WV_EHIP]
    assert st["readmits"] >= 1 and st["failed"] == 0
    assert as_pairs(out[a][0]) == as_pairs(ctx.eval_primes(ps1))
    assert as_pairs(out[b][0]) == as_pairs(ctx.search_range(10 ** 8, 10 ** 8 + 5000)[0])


def test_server_repeated_failures_end_requests(ctx):
    """Three failed steps with none completed between them end the active
    requests with the error (reported once by result, then forgotten) and free
    their pool slots: a request submitted afterwards is served normally.  Steps
    are pipelined, so a step's failure surfaces in the call that completes it."""
    say("case: server repeated failures")
    ps = oracle.primes(10 ** 9, 10 ** 9 + 300)
    with wv.Server(ctx, step_terms=1 << 28, max_primes=64) as srv:
        a = srv.submit_primes(ps[:40])
        raised = 0
        for _ in range(20):
            srv.inject_fault(0)                 # the next step to complete fails
            try:
                srv.step()
            except wv.WvError as e:
                assert e.status == wv.WV_EHIP
                raised += 1
                if raised == 3:
                    break
        assert raised == 3
        with pytest.raises(wv.WvError) as ei:
            srv.result(a)
        assert ei.value.status == wv.WV_EHIP
        with pytest.raises(wv.WvError):
            srv.result(a)                       # forgotten after the report
        st = srv.stats()
        assert st["failed"] == 1 and st["active"] == 0
        b = srv.submit_primes(ps[:60])          # needs the freed slots
        res = drain(srv, [b])
    assert as_pairs(res[b][0]) == as_pairs(ctx.eval_primes(ps[:60]))


def test_server_range_larger_than_pool_is_refused(ctx):
    """A range whose prime count exceeds the pool is refused at submission
    (nothing queued, no silent empty result); one that fits is served."""
    say("case: server range larger than the pool")
    lo, hi = 10 ** 8, 10 ** 8 + 20000
    n = ctx.count_primes(lo, hi)
    assert n > 700
    with wv.Server(ctx, step_terms=1 << 30, max_primes=700) as srv:
        with pytest.raises(wv.WvError) as ei:
            srv.submit_range(lo, hi)
        assert ei.value.status == wv.WV_EINVAL
        assert srv.stats()["submitted"] == 0
        small = (lo, lo + 9000)
        assert ctx.count_primes(*small) <= 700
        b = srv.submit_range(*small)
        res = drain(srv, [b])
    assert as_pairs(res[b][0]) == as_pairs(ctx.search_range(*small)[0])


def test_server_pool_admission(ctx):
    """A pool smaller than the offered requests admits them as slots free up."""
    ps = oracle.primes(10 ** 7, 10 ** 7 + 20000)
    chunks = [ps[i:i + 300] for i in range(0, len(ps), 300)]
    with wv.Server(ctx, step_terms=1 << 30, max_primes=700) as srv:
        ids = [srv.submit_primes(c) for c in chunks]
        active, pending = srv.step()
        # smallest first: the 40-prime list and two of 300 fill 640 of 700 slots
        sizes = sorted(len(c) for c in chunks)
        assert sizes[0] + 2 * 300 <= 700 < sizes[0] + 3 * 300
        assert pending == len(chunks) - 3 and active == 3
        res = drain(srv, ids)
    for c, rid in zip(chunks, ids):
        assert as_pairs(res[rid][0]) == as_pairs(ctx.eval_primes(c))


# ---------------------------------------------------------------------------
# residue statistics on the device (histograms of Sections 3 and 5, Tables 2-3)
# ---------------------------------------------------------------------------

def _table_rows(name):
    return [(int(p), int(r)) for p, r in read_golden(name)]


def test_range_stats_small_window_vs_oracle(ctx):
    """All primes 5 <= p < 1e5: device histograms (2000 bins and 7 bins) and
    near misses equal the oracle's, computed from the oracle's residues."""
    say("case: range_stats(5, 1e5)")
    ps = oracle.primes(5, 10 ** 5)
    rows = [(p, b, e) for p, (b, e) in zip(ps, oracle.residues(ps))]
    for bins, bound in ((2000, 50), (7, 1000)):
        hb, he, near, n = ctx.range_stats(5, 10 ** 5, bins=bins, near=bound)
        wb, we, wnear = oracle.residue_stats(rows, bins=bins, bound=bound)
        assert n == len(ps)
        assert list(hb) == wb and list(he) == we
        assert [(int(x["p"]), int(x["r"]), int(x["which"])) for x in near] == wnear


def test_range_stats_reproduces_tables_2_and_3(ctx):
    """Tables 2 and 3 list every prime in (1e9, 1e11) with |<r>_p| < 50, so a
    window around a printed prime has exactly the printed near misses."""
    tb = _table_rows("near_miss_B.txt")
    te = _table_rows("near_miss_E.txt")
    printed = sorted([(p, r, 1) for p, r in tb] + [(p, r, 2) for p, r in te], key=lambda t: (t[0], t[2]))
    centres = [p for p, _ in tb[:4]] + [p for p, _ in te[:5]]
    for c in centres:
        lo, hi = c - 4000, c + 4000
        say(f"case: range_stats near {c}")
        hb, he, near, n = ctx.range_stats(lo, hi, bins=2000, near=50)
        assert int(hb.sum()) == int(he.sum()) == n == ctx.count_primes(lo, hi)
        got = [(int(x["p"]), int(x["r"]), int(x["which"])) for x in near]
        assert got == [t for t in printed if lo <= t[0] < hi]


def test_range_stats_equals_host_statistics_of_search(ctx):
    """At 1e9 (about 10^4 primes): the device statistics equal the same
    statistics taken on the host from wv_search_range's results, and a
    sample of those results equals the oracle."""
    lo, hi = 10 ** 9, 10 ** 9 + 2 * 10 ** 5
    say(f"case: range_stats({lo}, {hi})")
    hb, he, near, n = ctx.range_stats(lo, hi, bins=2000, near=10 ** 6)
    res, _ = ctx.search_range(lo, hi)
    rows = [(int(r["p"]), int(r["b"]), int(r["e"])) for r in res]
    wb, we, wnear = oracle.residue_stats(rows, bins=2000, bound=10 ** 6)
    assert n == len(rows)
    assert list(hb) == wb and list(he) == we
    assert [(int(x["p"]), int(x["r"]), int(x["which"])) for x in near] == wnear
    pick = sorted(random.Random(4).sample(range(len(res)), 3))
    check_against_oracle(res[pick], method="table")


def test_range_stats_edges(ctx):
    """Empty range, one bin, the largest bin count, truncated near list, bad
    arguments."""
    say("case: range_stats edges")
    hb, he, near, n = ctx.range_stats(24, 29, bins=5, near=50)
    assert n == 0 and not hb.any() and not he.any() and len(near) == 0
    hb, he, near, n = ctx.range_stats(5, 3000, bins=1, near=0)
    assert list(hb) == list(he) == [n] and n == len(oracle.primes(5, 3000)) and len(near) == 0
    hb, he, _, n = ctx.range_stats(5, 3000, bins=wv.MAX_BINS, near=0)
    ps = oracle.primes(5, 3000)
    wb, we, _ = oracle.residue_stats([(p, b, e) for p, (b, e) in zip(ps, oracle.residues(ps))],
                                     bins=wv.MAX_BINS, bound=0)
    assert list(hb) == wb and list(he) == we
    # truncation: the binding retries with the reported size; the C call itself says ETRUNC
    import ctypes
    b0 = np.zeros(4, dtype=np.uint64)
    b1 = np.zeros(4, dtype=np.uint64)
    buf = np.zeros(2, dtype=wv.NEAR_DTYPE)
    nn, npr = ctypes.c_size_t(), ctypes.c_uint64()
    st = wv.lib().wv_range_stats(ctx._h, 5, 3000, 4, 3000, b0.ctypes.data_as(wv.P_U64), b1.ctypes.data_as(wv.P_U64),
                                 buf.ctypes.data_as(wv.VP), 2, ctypes.byref(nn), ctypes.byref(npr))
    assert st == wv.WV_ETRUNC and nn.value == 2 * npr.value == 2 * len(ps) and int(b0.sum()) == len(ps)
    _, _, near, _ = ctx.range_stats(5, 3000, bins=4, near=3000, near_cap=2)
    assert len(near) == 2 * len(ps)
    assert list(near[:2]) == list(buf)
    for bins in (0, wv.MAX_BINS + 1):
        with pytest.raises(wv.WvError):
            ctx.range_stats(5, 100, bins=bins)
    with pytest.raises(wv.WvError):
        ctx.range_stats(2 ** 40 - 10, 2 ** 40 + 10)


# ---------------------------------------------------------------------------
# congruences defined at run time (derivation engine, Section 2)
# ---------------------------------------------------------------------------

def _derived(start, rounds):
    from paper_2101_11157_amd import derive
    _, best, _ = derive.greedy(derive.Congruence.start(start), D=8, rounds=rounds)
    return best.to_json(f"{start}-{rounds}")


def test_defined_tables_all_small_primes():
    """Greedy-derived Bernoulli and Euler congruences, used from p = 11 on, give
    the residues of the printed tables (oracle-pinned above) for every prime
    below 3000, and the oracle's plain evaluation of the same congruences."""
    from oracle import congruences as C
    from paper_2101_11157_amd import derive
    say("case: derived tables from 11")
    jb, je = _derived("Vandiver", 20), _derived("EMac2", 20)
    ps = oracle.primes(5, 3000)
    with wv.Context(0) as c:
        ref = c.eval_primes(ps)
        b = c.define_derived_table(jb, min_p=11)
        e = c.define_derived_table(je, min_p=11)
        c.set_tables(b, e)
        got = c.eval_primes(ps)
        res, _ = c.search_range(5, 3000)
    assert as_pairs(got) == as_pairs(ref) == as_pairs(res)
    cb = derive.load_json(jb)
    L, terms = cb.integer_form()
    ob = C.Congruence("derived", "B", -3, L, terms, cb.cost(), "derived")
    pick = [p for p in ps if p > 1000][:20]
    assert [oracle.congruence_residue_exact(p, ob) for p in pick] == [int(r["b"]) for r in got if int(r["p"]) in pick]


def test_package_derived_tables_at_scale(ctx):
    """The shipped derived congruences (a ladder of rungs of hundreds to tens
    of thousands of sums, each from its min_p, the lowest from p = 11)
    reproduce the oracle samples at 1e9 and 1e11 and Tables 2-3."""
    say("case: package derived tables")
    g9 = golden_json("window_1e9.json")["rows"][:40]
    g11 = golden_json("window_1e11.json")["rows"]
    tb = [(int(p), int(r)) for p, r in read_golden("near_miss_B.txt")][:6]
    te = [(int(p), int(r)) for p, r in read_golden("near_miss_E.txt")][:6]
    with wv.Context(0) as c:
        b, e = c.use_derived_tables(min_p=11)
        jb, je = wv.derived_table("B"), wv.derived_table("E")
        assert jb["n"] > 300 and je["n"] > 300
        got = c.eval_primes([r["p"] for r in g9 + g11])
        assert as_pairs(got) == [(r["b"], r["e"]) for r in g9 + g11]
        st = c.stats()
        # slots per prime: the largest rung any prime of the batch can select
        pmax = max(int(p) for p in got["p"])
        per = sum(max(r["n"] for r in wv.derived_ladder(side) if r["min_p"] < pmax) for side in "BE")
        assert st["n_sums"] == len(got) * per
        got = c.eval_primes([p for p, _ in tb] + [p for p, _ in te])
    sym = [(exact.symmetric(int(r["b"]), int(r["p"])), exact.symmetric(int(r["e"]), int(r["p"]))) for r in got]
    assert [s[0] for s in sym[:len(tb)]] == [r for _, r in tb]
    assert [s[1] for s in sym[len(tb):]] == [r for _, r in te]


def test_defined_table_fallbacks():
    """Primes below min_p, and primes dividing the left side (a valid table
    scaled by 13), take the printed tables; results do not change."""
    say("case: defined-table fallbacks")
    jb = _derived("Vandiver", 8)
    scaled = dict(jb, lhs=str(13 * int(jb["lhs"])), terms=[[str(13 * int(t[0]))] + t[1:] for t in jb["terms"]])
    ps = oracle.primes(5, 400) + oracle.primes(10 ** 6, 10 ** 6 + 300)
    with wv.Context(0) as c:
        ref = c.eval_primes(ps)
        hi = c.define_derived_table(jb, min_p=10 ** 6)
        c.set_tables(hi, "EE33")
        assert as_pairs(c.eval_primes(ps)) == as_pairs(ref)
        s13 = c.define_derived_table(scaled, min_p=11)
        c.set_tables(s13, "EE33")
        assert as_pairs(c.eval_primes(ps)) == as_pairs(ref)


def _open_interval_terms(p, ends):
    """Integers s with x p < s < y p summed over the sums (eqnDefnS); ends:
    (xa, xb, ya, yb) per sum."""
    return sum(max(0, -(-ya * p // yb) - (xa * p // xb) - 1) for xa, xb, ya, yb in ends)


@functools.lru_cache(maxsize=None)
def _ends(side, rounds):
    if rounds is None:
        from oracle import congruences as C
        t = C.BB30 if side == "B" else C.EE33
        return tuple((x.numerator, x.denominator, y.numerator, y.denominator) for _, x, y in t.terms)
    obj = wv.derived_table(side, rounds)
    return tuple((int(xa), int(xb), int(ya), int(yb)) for _, xa, xb, ya, yb in obj["terms"])


def test_derived_ladder_matches_printed_tables():
    """The shipped ladders (a rung per range of p, chained with
    wv_set_table_below): primes on every rung, from below the lowest threshold
    to 1e11, searched and evaluated in mixed batches, give the residues of the
    printed eqnBB30 / eqnEE33 (independent intervals and coefficients); each
    prime's work is that of the rung its size selects."""
    rungs = {side: wv.derived_ladder(side) for side in "BE"}
    marks = sorted({r["min_p"] for side in "BE" for r in rungs[side]} | {10 ** 11 - 10 ** 6})
    ps = []
    for m in marks:
        ps += oracle.primes(max(11, m - 400), m + 400)[:6]      # both sides of each threshold
    say(f"case: derived ladder, {len(ps)} primes around {len(marks)} thresholds")
    with wv.Context(0) as c:
        ref = c.eval_primes(ps)
        b, e = c.use_derived_tables()
        got = c.eval_primes(ps)
        st = c.stats()
        # the terms summed are those of the rung (or printed table) each prime selects
        def terms(p, side):
            use = [r for r in rungs[side] if p >= r["min_p"]]
            return _open_interval_terms(p, _ends(side, use[-1]["rounds"] if use else None))
        assert st["n_terms"] == sum(terms(p, "B") + terms(p, "E") for p in ps)
        # a window that straddles a threshold, searched in one call
        m = rungs["B"][len(rungs["B"]) // 2]["min_p"]
        win, _ = c.search_range(m - 3000, m + 3000)
    assert as_pairs(got) == as_pairs(ref)
    # the ladders from a larger min_p (rungs below it left out)
    with wv.Context(0) as c:
        c.use_derived_tables(min_p=10 ** 10)
        assert as_pairs(c.eval_primes(ps)) == as_pairs(ref)
    c2 = wv.Context(0)
    try:
        ref_win, _ = c2.search_range(m - 3000, m + 3000)
    finally:
        c2.close()
    assert as_pairs(win) == as_pairs(ref_win)


def test_set_table_below_rejects_bad_chains(ctx):
    say("case: set_table_below errors")
    from fractions import Fraction as F
    jb = _derived("Vandiver", 8)
    with wv.Context(0) as c:
        lo = c.define_derived_table(jb, min_p=11)
        hi = c.define_derived_table(jb, min_p=10 ** 6)
        e = c.define_derived_table(_derived("EMac2", 8), min_p=11)
        c.set_table_below(hi, lo)                     # a smaller min_p: fine
        for t, below in [(hi, e),                     # another degree
                         (lo, hi),                    # min_p not smaller (would cycle)
                         (lo, lo),
                         ("BB30", lo),                # a compiled table has no chain
                         (hi, "V12"),                 # a root form
                         (hi, 999)]:
            with pytest.raises(wv.WvError):
                c.set_table_below(wv.TABLE_ID[t] if isinstance(t, str) else t, below)
        c.set_tables(hi, "EE33")
        ps = oracle.primes(11, 2000) + oracle.primes(10 ** 6, 10 ** 6 + 200)
        got = c.eval_primes(ps)
    assert as_pairs(got) == as_pairs(ctx.eval_primes(ps))
    assert as_pairs(got)[:40] == [tuple(x) for x in oracle.residues(ps[:40])]


def test_define_table_rejects_malformed_input(ctx):
    say("case: define_table errors")
    from fractions import Fraction as F
    good = [(1, F(1, 6), F(1, 5))]
    bad = [
        dict(deg=4, lhs=14, terms=good),
        dict(deg=3, lhs=0, terms=good),
        dict(deg=3, lhs=14, terms=[]),
        dict(deg=3, lhs=14, terms=[(1, F(1, 5), F(1, 6))]),          # x >= y
        dict(deg=3, lhs=14, terms=[(1, F(1, 5), F(1, 5))]),
        dict(deg=3, lhs=14, terms=[(1, F(1, 2), F(3, 2))]),          # y > 1
        dict(deg=3, lhs=14, terms=good, min_p=7),
    ]
    for kw in bad:
        with pytest.raises(wv.WvError):
            ctx.define_table(**kw)
    with pytest.raises(wv.WvError):
        ctx.set_tables("EE33", "EE33")                               # wrong side


def test_batch_over_2_26_slots_with_defined_tables():
    """A search batch of more than 2^26 (prime, sum) slots (about 1e5 primes
    with shipped congruences of 600 to 1000 sums in all, used from p = 11):
    the per-sum reduction indexes slots beyond 2^26 correctly; results equal
    the printed tables' (a regression test for a 32-bit thread index)."""
    lo, hi = 10 ** 6, 10 ** 6 + 1_400_000
    rb = max((r for r in wv.derived_ladder("B") if r["n"] <= 500), key=lambda r: r["n"])
    re_ = max((r for r in wv.derived_ladder("E") if r["n"] <= 500), key=lambda r: r["n"])
    per = rb["n"] + re_["n"]
    assert 600 <= per <= 1000
    say(f"case: range [{lo}, {hi}) with derived tables of {per} sums from p = 11")
    with wv.Context(0) as c:
        ref, _ = c.search_range(lo, hi)
        b = c.define_derived_table(wv.derived_table("B", rb["rounds"]), min_p=11)
        e = c.define_derived_table(wv.derived_table("E", re_["rounds"]), min_p=11)
        c.set_tables(b, e)
        got, _ = c.search_range(lo, hi)
        st = c.stats()
    # one batch: fewer than 2^27 slots in all, more than 2^26
    assert (1 << 26) < st["n_sums"] == len(got) * per < (1 << 27)
    assert [int(p) for p in got["p"]] == [int(p) for p in ref["p"]]
    assert as_pairs(got) == as_pairs(ref)


def test_batched_windows_with_derived_tables(ctx):
    """Windows on both sides of several thresholds of the derived ladders in
    one batched call equal the same windows searched alone (the printed tables
    below the lowest threshold, above it the rung each prime's size selects)."""
    from paper_2101_11157_amd import workloads
    wins = workloads.batch_windows(0, 12, len_range=(1e2, 3e3), start_range=(1e8, 5e10))
    say(f"case: {len(wins)} windows, derived tables")
    with wv.Context(0) as c:
        c.use_derived_tables()
        got = c.search_windows([a for a, _ in wins], [b for _, b in wins])
        for (a, b), res in zip(wins, got):
            alone, _ = c.search_range(a, b)
            assert as_pairs(res) == as_pairs(alone)
        flat = np.concatenate([g for g in got if len(g)])
    pick = sorted(random.Random(5).sample(range(len(flat)), 4))
    check_against_oracle(flat[pick], method="table")


# ---------------------------------------------------------------------------
# every index: irregular and E-irregular pairs
# ---------------------------------------------------------------------------


@pytest.fixture(params=[1, 2], ids=["valu", "mfma"])
def irr_path(request, ctx):
    """Both power-sum kernels: vector ALU and matrix cores."""
    ctx.set_irregular_path(request.param)
    yield request.param
    ctx.set_irregular_path(0)


@pytest.mark.gpu
def test_all_index_residues_small_primes(ctx, irr_path):
    """B_{2k}, E_{2k} mod p for every 2k <= p - 3 of each prime below 700
    equal the oracle's recurrences, element by element (p = 5, 7 included:
    one and two indices; p = 5 needs the second congruence of the chain)."""
    say(f"case: every index, primes below 700, path {irr_path}")
    for p in oracle.primes(5, 700):
        b, e = ctx.bernoulli_euler_all(p)
        assert [int(x) for x in b] == oracle.bernoulli_all(p), p
        assert [int(x) for x in e] == oracle.euler_all(p), p


@pytest.mark.gpu
@functools.lru_cache(maxsize=None)
def oracle_all_index(p):
    return oracle.bernoulli_all(p), oracle.euler_all(p)


@pytest.mark.parametrize("p", [2003, 5783, 16843, 30011, 33013, 37003])
def test_all_index_residues_larger_primes(ctx, irr_path, p):
    """Several units per range, many exponent blocks, ragged last rows and
    columns (vector: 1024 s x 2048 exponents per wave; matrix: 128 rows of
    16 ct exponents x 1024 s per workgroup; at 33013, ct = 3 and three row
    blocks, the last one 88 rows deep; 37003 is a prime of the census
    bench's first timed window, ct = 5, 232 rows)."""
    say(f"case: every index, p = {p}, path {irr_path}")
    b, e = ctx.bernoulli_euler_all(p)
    want_b, want_e = oracle_all_index(p)
    assert [int(x) for x in b] == want_b
    assert [int(x) for x in e] == want_e


@pytest.mark.gpu
def _power_sum(lo, hi, t, p):
    """sum_{lo <= s <= hi} s^t mod p on the host (numpy, exact for p < 2^26:
    products of two residues stay below 2^52)."""
    assert p < (1 << 26)
    s = np.arange(lo, hi + 1, dtype=np.uint64) % np.uint64(p)
    acc = np.ones_like(s)
    e = t
    while e:
        if e & 1:
            acc = acc * s % np.uint64(p)
        s = s * s % np.uint64(p)
        e >>= 1
    return int(acc.sum(dtype=np.uint64) % np.uint64(p))   # < 2^26 terms below 2^26


@pytest.mark.parametrize("p", [2097143, 8388593, 16777213])
def test_all_index_paths_agree_at_scale(ctx, p):
    """Below 2^21 (matrix-core partial sums reduced after every 1024 s), below
    2^23 (after every 192 s) and just below 2^24 (after every 32 s, the
    tightest exact range of the matrix path): the vector and matrix kernels
    agree on every index, and a few indices agree with the general-index
    congruence evaluated plainly on the host."""
    say(f"case: every index at p = {p}")
    ctx.set_irregular_path(1)
    try:
        bv, ev = ctx.bernoulli_euler_all(p)
    finally:
        ctx.set_irregular_path(0)
    ba, ea = ctx.bernoulli_euler_all(p)   # automatic: matrix cores below 2^21
    assert np.array_equal(bv, ba) and np.array_equal(ev, ea)
    assert int(bv.max()) < p and int(ev.max()) < p
    for k in (1, 2, 1234, (p - 3) // 2):
        # eqnE1 at exponent t = 2k: E_t = (-1)^{k'} 4^{t+1} S_t(0, 1/4), k' = (p-1-t)/2
        t = 2 * k
        S = _power_sum(1, p // 4, t, p)
        want = (-1) ** ((p - 1 - t) // 2) * pow(4, t + 1, p) * S % p
        assert int(ev[k - 1]) == want, k
        # (2,3,4) at exponent 2k - 1: C_k B_{2k} = S_{2k-1}(1/4, 1/3)
        c = (pow(2, p - 2 * k, p) + pow(3, p - 2 * k, p) - pow(4, p - 2 * k, p) - 1) * pow(4 * k, -1, p) % p
        if c:
            S = _power_sum(p // 4 + 1, p // 3, 2 * k - 1, p)
            assert int(bv[k - 1]) == S * pow(c, -1, p) % p, k


@pytest.mark.gpu
def test_irregular_pairs_census_matches_oracle(ctx):
    """Every pair of the primes in [5, 3000), and the paper's statements:
    37 is the smallest irregular prime, 19 (19 | E_10) the smallest
    E-irregular one."""
    say("case: irregular census below 3000")
    from concurrent.futures import ThreadPoolExecutor
    got, n_primes, unresolved = ctx.irregular_pairs(5, 3000)
    ps = oracle.primes(5, 3000)
    with ThreadPoolExecutor(8) as ex:
        want = [x for lst in ex.map(oracle.irregular_pairs, ps) for x in lst]
    assert n_primes == len(ps) and unresolved == 0
    assert [(int(r["p"]), int(r["two_k"]), int(r["kind"])) for r in got] == sorted(want)
    assert min(int(r["p"]) for r in got if r["kind"] == 1) == 37
    assert min(int(r["p"]) for r in got if r["kind"] == 2) == 19


@pytest.mark.gpu
def test_irregular_pairs_paper_primes(ctx):
    """Section 1: (16843, 16840) is an irregular pair (a Wolstenholme prime),
    5783 has index of E-irregularity 5, 149 and 241 give E-irregular pairs
    (p, p - 3) (Vandiver primes)."""
    say("case: irregular pairs of the paper's primes")
    got, _, unresolved = ctx.irregular_pairs(16843, 16844)
    assert unresolved == 0 and (16843, 16840, 1) in [(int(r["p"]), int(r["two_k"]), int(r["kind"])) for r in got]
    got, _, _ = ctx.irregular_pairs(5783, 5784)
    assert sum(1 for r in got if r["kind"] == 2) == 5
    for p in (149, 241):
        got, _, _ = ctx.irregular_pairs(p, p + 1)
        assert (p, p - 3, 2) in [(int(r["p"]), int(r["two_k"]), int(r["kind"])) for r in got]


@pytest.mark.gpu
def test_irregular_entry_points_reject_bad_input(ctx):
    say("case: irregular entry points, bad input")
    with pytest.raises(wv.WvError) as ei:
        ctx.bernoulli_euler_all(wv.IRR_P_MAX + 1)
    assert ei.value.status == wv.WV_EDOMAIN
    with pytest.raises(wv.WvError) as ei:
        ctx.bernoulli_euler_all(1001)
    assert ei.value.status == wv.WV_ENOTPRIME
    with pytest.raises(wv.WvError) as ei:
        ctx.bernoulli_euler_all(3)
    assert ei.value.status == wv.WV_EDOMAIN
    with pytest.raises(wv.WvError) as ei:
        ctx.irregular_pairs(5, wv.IRR_P_MAX + 1)
    assert ei.value.status == wv.WV_EDOMAIN
    got, n_primes, _ = ctx.irregular_pairs(24, 29)   # no prime
    assert len(got) == 0 and n_primes == 0
    # two pairs below 37 (both E-irregular) through a one-entry buffer: the
    # binding retries after WV_ETRUNC
    got, n_primes, _ = ctx.irregular_pairs(5, 37, cap=1)
    assert n_primes == 9
    assert [(int(r["p"]), int(r["two_k"]), int(r["kind"])) for r in got] == [(19, 10, 2), (31, 22, 2)]
