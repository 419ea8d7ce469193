"""CPU checks of the C ABI (include/bsm.h) and its host logic.

No test here launches device work: the library is loaded, its exports are
checked against the header, struct layouts are checked against the header
as compiled by gcc, and the host-only paths (pattern generation, argument
validation that runs before any device call) are exercised.
"""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1402_2020_amd import _bsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsm.h")
PEAKS_HEADER = os.path.join(ROOT, "include", "bsm_peaks.h")


@pytest.fixture(scope="module")
def lib():
    return _bsm.load()


def _declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bsm_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(_bsm.EXPORTS)
    assert _declared_functions(PEAKS_HEADER) == sorted(_bsm.PEAK_EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    declared = _declared_functions() + _declared_functions(PEAKS_HEADER)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _bsm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (bsm_[a-z_]+)$", out, flags=re.M))
    assert set(declared) <= exported


STRUCTS = (("bsm_params", "Params"), ("bsm_pair", "Pair"), ("bsm_times", "Times"),
           ("bsm_tuning", "Tuning"), ("bsm_serve_counters", "ServeCounters"),
           ("bsm_peaks", "Peaks"))


def test_struct_layouts_match_header(tmp_path):
    # sizes and every field offset, from the C compiler vs the ctypes classes
    lines = []
    for T, cname in STRUCTS:
        lines.append(f'  printf("{T} %zu\\n", sizeof({T}));')
        for fname, _ in getattr(_bsm, cname)._fields_:
            lines.append(f'  printf("{T}.{fname} %zu\\n", offsetof({T}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"bsm_peaks.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(ln.rsplit(" ", 1) for ln in subprocess.run([str(exe)], capture_output=True,
                                                           text=True).stdout.splitlines())
    for T, cname in STRUCTS:
        cls = getattr(_bsm, cname)
        assert int(got[T]) == C.sizeof(cls), T
        for fname, _ in cls._fields_:
            assert int(got[f"{T}.{fname}"]) == getattr(cls, fname).offset, (T, fname)


@pytest.mark.parametrize("seed,n,S,sigma", [(0, 64, 3, 0.8), (14022020, 256, 15, 4 * 15 / 26),
                                            (1402202000000001, 1024, 31, 4 * 31 / 26),
                                            (7, 4096, 26, 4.0), (2**64 - 1, 100, 63, 9.0)])
def test_library_pattern_equals_oracle(orc, seed, n, S, sigma):
    # both sides implement splitmix64 + Box-Muller from the published
    # definitions; they must agree bit for bit
    assert np.array_equal(_bsm.bsm_make_pattern(seed, n, S, sigma),
                          orc.make_pattern(seed, n, S, sigma))


def test_make_pattern_validation(lib):
    out = np.zeros((8, 4), np.int8)
    p = out.ctypes.data_as(C.POINTER(C.c_int8))
    assert lib.bsm_make_pattern(1, 8, 1, 1.0, p) == _bsm.EINVAL
    assert "window" in _bsm.bsm_last_error()
    assert lib.bsm_make_pattern(1, 8, 64, 1.0, p) == _bsm.EINVAL
    assert lib.bsm_make_pattern(1, 8, 9, 0.0, p) == _bsm.EINVAL
    assert lib.bsm_make_pattern(1, 0, 9, 1.0, p) == _bsm.EINVAL
    assert lib.bsm_make_pattern(1, 8, 9, 1.0, None) == _bsm.EINVAL
    assert lib.bsm_make_pattern(1, 8, 9, 1.0, p) == _bsm.OK
    assert _bsm.bsm_last_error() == ""


@pytest.mark.parametrize("field,value", [("n_bits", 0), ("n_bits", 100), ("n_bits", 8192),
                                         ("window", 1), ("window", 64), ("mask_rank", -1),
                                         ("mask_rank", 257), ("use_mask", 2)])
def test_create_rejects_bad_params_before_device(lib, field, value):
    p = _bsm.Params(256, 15, 0.0, 1, None, 0, 1)
    setattr(p, field, value)
    h = C.c_void_p()
    assert lib.bsm_create(C.byref(p), 0, C.byref(h)) == _bsm.EINVAL
    assert not h.value


def test_create_rejects_pattern_outside_window(lib):
    pat = np.zeros((64, 4), np.int8)
    pat[3, 2] = 8   # window 15 allows [-7, 7]
    p = _bsm.Params(64, 15, 0.0, 1, pat.ctypes.data_as(C.POINTER(C.c_int8)), 0, 1)
    h = C.c_void_p()
    assert lib.bsm_create(C.byref(p), 0, C.byref(h)) == _bsm.EINVAL
    assert "pair 4" in _bsm.bsm_last_error()


def test_null_context_is_rejected(lib):
    assert lib.bsm_match(None, None, None, 4, 4, 12, 1, None, None, None) == _bsm.EINVAL
    assert lib.bsm_describe(None, None, 4, 4, 12, None, None, None) == _bsm.EINVAL
    assert lib.bsm_cost_wta(None, None, None, None, 4, 4, 1, None, None, None) == _bsm.EINVAL
    assert lib.bsm_footprint(None, 4, 4, 1, 0) == 0
    lib.bsm_destroy(None)


@pytest.mark.parametrize("hbm_bytes,reps,null_out", [(4 << 30, 0, False), (1 << 20, 3, False),
                                                     ((256 << 20) + 4096, 3, False),
                                                     (4 << 30, 3, True)])
def test_measure_peaks_rejects_bad_arguments_before_device(lib, hbm_bytes, reps, null_out):
    out = None if null_out else C.byref(_bsm.Peaks())
    assert lib.bsm_measure_peaks(0, hbm_bytes, reps, out) == _bsm.EINVAL
    assert _bsm.bsm_last_error()
