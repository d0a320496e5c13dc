"""The allocation-free entry point wv_eval_primes_static, through the C ABI,
against the existing device-pointer entry point wv_eval_primes_async on the
same inputs: two calls in a row (the second smaller, so the scratch array
holds the first call's data when the second starts), an invalid input in the
middle of a batch, the derived congruences near 1e11, and the size limits."""
import ctypes
import os
import sys

import numpy as np
import pytest

import paper_2101_11157_amd as wv
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class Hip:
    """HIP runtime calls through ctypes (the runtime the library loaded)."""

    def __init__(self):
        wv.lib()
        self.h = ctypes.CDLL("libamdhip64.so.7")
        self.h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.h.hipFree.argtypes = [ctypes.c_void_p]
        self.h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.h.hipStreamCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.h.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.h.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        self.bufs = []

    def malloc(self, n):
        p = ctypes.c_void_p()
        assert self.h.hipMalloc(ctypes.byref(p), n) == 0
        self.bufs.append(p.value)
        return p.value

    def h2d(self, dst, arr):
        assert self.h.hipMemcpy(dst, arr.ctypes.data, arr.nbytes, 1) == 0

    def d2h(self, arr, src):
        assert self.h.hipMemcpy(arr.ctypes.data, src, arr.nbytes, 2) == 0

    def free_all(self):
        for p in self.bufs:
            self.h.hipFree(p)
        self.bufs = []


def run_both(ctx, hip, stream, primes):
    """(static results, async results) for the same device input."""
    arr = np.ascontiguousarray(np.asarray(primes, dtype=np.uint64))
    nbytes = arr.size * wv.RESULT_DTYPE.itemsize
    d_in = hip.malloc(arr.nbytes)
    d_static, d_async = hip.malloc(nbytes), hip.malloc(nbytes)
    hip.h2d(d_in, arr)
    ctx.eval_primes_static(d_in, arr.size, d_static, stream)
    ctx.eval_primes_async(d_in, arr.size, d_async, stream)
    assert hip.h.hipStreamSynchronize(stream) == 0
    got_s = np.zeros(arr.size, dtype=wv.RESULT_DTYPE)
    got_a = np.zeros(arr.size, dtype=wv.RESULT_DTYPE)
    hip.d2h(got_s, d_static)
    hip.d2h(got_a, d_async)
    return got_s, got_a


def same(a, b):
    return ([(int(r["p"]), int(r["b"]), int(r["e"]), int(r["flags"])) for r in a] ==
            [(int(r["p"]), int(r["b"]), int(r["e"]), int(r["flags"])) for r in b])


def test_static_entry_matches_async_entry():
    hip = Hip()
    st = ctypes.c_void_p()
    assert hip.h.hipStreamCreate(ctypes.byref(st)) == 0
    try:
        with wv.Context(0) as ctx:
            # call 1: 1,300 primes near 3e6 with an invalid input (4) in the middle
            ps = oracle.primes(3 * 10 ** 6, 3 * 10 ** 6 + 20000)
            big = ps[:700] + [4] + ps[700:]
            say(f"case: static entry, call 1: {len(big)} inputs near 3e6 (printed tables)")
            s1, a1 = run_both(ctx, hip, st.value, big)
            assert same(s1, a1)
            assert int(s1[700]["flags"]) == 0xFFFFFFFF
            assert [int(x) for x in np.delete(s1, 700)["p"]] == ps
            # call 2, smaller: 120 primes near 1e9 (the array holds call 1's data)
            ps2 = oracle.primes(10 ** 9, 10 ** 9 + 2700)
            say(f"case: static entry, call 2: {len(ps2)} primes near 1e9")
            s2, a2 = run_both(ctx, hip, st.value, ps2)
            assert same(s2, a2)
            assert [int(x) for x in s2["p"]] == ps2
            # the residues are the oracle's on a few of them (eqnBB30 + eqnEE33)
            pick = [ps2[0], ps2[len(ps2) // 2], ps2[-1]]
            want = oracle.residues(pick, method="table")
            by_p = {int(r["p"]): (int(r["b"]), int(r["e"])) for r in s2}
            assert [by_p[p] for p in pick] == want
            # derived congruences near 1e11 (thousands of sums per prime): as
            # many primes as the fixed slot area holds, whose partial-pair
            # area forces chunks longer than the automatic size
            # the largest rungs of the ladder that leave room for 40 primes
            cap = min(max(r["rounds"] for r in wv.derived_ladder(side) if r["n"] <= (1 << 19) // 80)
                      for side in "BE")
            ctx.use_derived_tables(top=cap)
            per = sum(max(r["n"] for r in wv.derived_ladder(side) if r["rounds"] <= cap) for side in "BE")
            room = (1 << 19) // per
            ps3 = oracle.primes(10 ** 11 - 10 ** 6, 10 ** 11 - 10 ** 6 + 3600)[:room]
            assert len(ps3) >= 40
            say(f"case: static entry, call 3: {len(ps3)} primes near 1e11 (derived tables)")
            s3, a3 = run_both(ctx, hip, st.value, ps3)
            assert same(s3, a3)
            assert np.all(s3["flags"] != 0xFFFFFFFF)
            # limits: refused before anything is enqueued
            d = hip.malloc(8 * 256)
            with pytest.raises(wv.WvError) as ei:
                ctx.eval_primes_static(d, room + 1, d, st.value)   # more slots than 2^19
            assert ei.value.status == wv.WV_EINVAL
            with pytest.raises(wv.WvError) as ei:
                ctx.eval_primes_static(d, (1 << 16) + 1, d, st.value)
            assert ei.value.status == wv.WV_EINVAL
            ctx.eval_primes_static(d, 0, d, st.value)          # n = 0: nothing to do
            assert hip.h.hipStreamSynchronize(st) == 0
    finally:
        hip.h.hipStreamDestroy(st)
        hip.free_all()
