"""CPU-side checks of the product: the C ABI library loads and exports every
declared entry point, its compiled-in congruence data matches the paper, its
error paths work without a GPU, and the device arithmetic and hot loop pass a
host build of their unit test."""
import ctypes
import os
import re
import subprocess
import sys
from fractions import Fraction

import pytest

import paper_2101_11157_amd as wv
from paper_2101_11157_amd import build as wv_build
from oracle import congruences as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wvprime.h")


@pytest.fixture(scope="module")
def lib():
    if wv_build.is_stale():
        wv_build.build()
    return wv.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*\*?\s*\*?\s*(wv_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n != "wv_symmetric"))


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(lib, n), f"{n} missing from libwvprime.so"
    # and the exported list (nm) holds them as C symbols
    out = subprocess.run(["nm", "-D", "--defined-only", wv.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_strerror(lib):
    assert wv._strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6):
        assert wv._strerror(code) not in ("ok", "unknown status")
    assert wv._strerror(-99) == "unknown status"


NAMES = ["BB1", "BB2", "BB6", "BB9", "BB16", "BB22", "BB30", "EE3", "EE5", "EE9", "EE16", "EE24", "EE33"]


@pytest.mark.parametrize("name", NAMES + ["V12", "E1"])
def test_compiled_tables_match_paper(lib, name):
    """Costs recomputed from the library's own endpoints equal the printed costs,
    and every term equals the oracle's separately typed copy."""
    n, lhs, cn, cd = wv.table_info(name)
    terms = wv.table_terms(name)
    assert len(terms) == n
    cost = sum((Fraction(ya, yb) - Fraction(xa, xb) for _, xa, xb, ya, yb in terms), Fraction(0))
    assert cost == Fraction(cn, cd)
    ref = C.table(name if name != "E1" else "E1")
    assert cost == ref.cost
    assert lhs == ref.lhs
    assert [(c, Fraction(xa, xb), Fraction(ya, yb)) for c, xa, xb, ya, yb in terms] == ref.terms
    # left sides have no prime factor above 7, so every table is usable for p >= 11
    m = abs(lhs)
    for q in (2, 3, 5, 7):
        while m % q == 0:
            m //= q
    assert m == 1


def test_bad_table_ids(lib):
    assert lib.wv_table_info(99, None, None, None, None) == wv.WV_EINVAL
    assert lib.wv_table_term(0, 5, None, None, None, None, None) == wv.WV_EINVAL


def test_null_arguments_rejected_without_gpu(lib):
    assert lib.wv_create(0, None) == wv.WV_EINVAL
    assert lib.wv_destroy(None) == wv.WV_OK
    assert lib.wv_set_tables(None, 6, 12) == wv.WV_EINVAL
    assert lib.wv_set_table_below(None, 15, 6) == wv.WV_EINVAL
    assert lib.wv_count_primes(None, 0, 10, None) == wv.WV_EINVAL
    assert lib.wv_eval_primes(None, None, 0, None) == wv.WV_EINVAL
    assert lib.wv_get_stats(None, None) == wv.WV_EINVAL
    assert lib.wv_bernoulli_euler_all(None, 37, None, None) == wv.WV_EINVAL
    assert lib.wv_irregular_pairs(None, 5, 100, None, 0, None, None, None) == wv.WV_EINVAL


def test_create_reports_missing_device():
    """No GPU in this container: wv_create must fail cleanly, not crash."""
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = wv.lib().wv_create(0, ctypes.byref(h))
    assert rc in (wv.WV_EINVAL, wv.WV_EHIP)
    assert not h.value


def test_symmetric_helper():
    assert wv.symmetric(0, 11) == 0
    assert wv.symmetric(5, 11) == 5
    assert wv.symmetric(6, 11) == -5
    assert wv.symmetric(10, 11) == -1


def test_device_arithmetic_host_build(tmp_path):
    """mont.hpp and sum_core.hpp built as plain C++ against __int128 reference."""
    exe = tmp_path / "test_core"
    src = os.path.join(ROOT, "tests", "cpp", "test_core.cpp")
    inc = os.path.join(ROOT, "paper_2101_11157_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-I", inc, src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("OK ")


def test_device_arithmetic_host_build_sanitized(tmp_path):
    """Same test under AddressSanitizer and UBSan (host code only)."""
    exe = tmp_path / "test_core_asan"
    src = os.path.join(ROOT, "tests", "cpp", "test_core.cpp")
    inc = os.path.join(ROOT, "paper_2101_11157_amd", "csrc")
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-I", inc, src, "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime unavailable: " + r.stderr[-200:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why,
    before touching any device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus 2 is not supported" in r.stderr and r.stdout == ""


def test_peak_library_exports():
    """The microbenchmark library behind the rooflines loads and exports its
    entry points (no device call)."""
    path = os.path.join(ROOT, "paper_2101_11157_amd", "libwvpeak.so")
    if not os.path.exists(path):
        wv_build.build()
    L = ctypes.CDLL(path)
    for name in ("wv_peak_count", "wv_peak_rates", "wv_peak_mfma_f64"):
        assert hasattr(L, name), name
    L.wv_peak_count.restype = ctypes.c_int
    assert L.wv_peak_count() == 14
