"""CPU checks of the C ABI boundary: the library loads, exports every entry
point that include/krr.h declares, and rejects bad arguments before touching
the device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2409_01712_amd as krr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "krr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(krr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(krr.LIB_PATH):
        from paper_2409_01712_amd import build
        build.build()
    return krr.load()


def test_header_declares_the_four_phases():
    names = _declared()
    for f in ("krr_build_kernel", "krr_factor", "krr_solve", "krr_predict", "krr_create",
              "krr_destroy", "krr_status_string"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    bound = {s[0] for s in krr._SIGS}
    assert bound == set(names), set(names) ^ bound


def test_status_strings(lib):
    for s in range(9):
        assert lib.krr_status_string(s)
        assert lib.krr_status_string(s) != b"unknown status"
    assert b"genotype" in lib.krr_status_string(krr.KRR_ERROR_BAD_GENOTYPE)


def test_invalid_arguments_rejected_on_host(lib):
    P = ctypes.c_void_p
    h = P()
    # null output handle / null context: rejected before any device call
    assert lib.krr_create(None, 0, None, None) == krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_build_kernel(None, None, 10, 10, 16, 0.1, 0.1, ctypes.byref(h)) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_factor(None, None, None, ctypes.byref(h)) == krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_solve(None, None, None, 1, 1, None, 1, None, None) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_predict(None, None, None, 1, 16, None, 1, 1, None, 1) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_destroy(None) == krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_kernel_release(None) == krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_factor_release(None) == krr.KRR_ERROR_INVALID_VALUE
    info = krr.krr_factor_info()
    assert lib.krr_factor_get_info(None, ctypes.byref(info)) == krr.KRR_ERROR_INVALID_VALUE
    # bad tile option is rejected before the device is queried
    opts = krr.krr_options(300, 0, 0)
    assert lib.krr_create(ctypes.byref(h), 0, None, ctypes.byref(opts)) == \
        krr.KRR_ERROR_INVALID_VALUE
    # an allocator without its free function (or the reverse) is rejected
    opts = krr.krr_options(512, 0, 0)
    opts.device_alloc = krr.KRR_ALLOC_FN(lambda b, u: None)
    assert lib.krr_create(ctypes.byref(h), 0, None, ctypes.byref(opts)) == \
        krr.KRR_ERROR_INVALID_VALUE


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives the header."""
    structs = {
        "krr_options": krr.krr_options,
        "krr_precision_policy": krr.krr_precision_policy,
        "krr_refine_opts": krr.krr_refine_opts,
        "krr_solve_info": krr.krr_solve_info,
        "krr_factor_info": krr.krr_factor_info,
        "krr_kernel_desc": krr.krr_kernel_desc,
        "krr_tuning": krr.krr_tuning,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "krr.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (name, name))
        for fname, _ in cls._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));'
                         % (name, fname, name, fname))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().split("\n") if l)
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got["%s.%s" % (name, fname)]) == getattr(cls, fname).offset, (name, fname)


def test_product_path_does_not_import_oracle():
    """The library package never imports the CPU oracle or the input generator."""
    pkg = os.path.join(ROOT, "paper_2409_01712_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "krr_oracle" not in txt, f


def test_batched_arguments_rejected_on_host(lib):
    P = ctypes.c_void_p
    outs = (P * 2)()
    n = (ctypes.c_int64 * 2)(10, 10)
    assert lib.krr_build_kernel_batched(None, 2, None, n, 16, n, None, None, outs) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_build_kernel_batched(None, 0, None, None, 16, None, None, None, outs) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_factor_batched(None, 2, None, None, outs) == krr.KRR_ERROR_INVALID_VALUE
    assert outs[0] is None and outs[1] is None
    assert lib.krr_solve_batched(None, 2, None, None, 1, None, None, None, None, None) == \
        krr.KRR_ERROR_INVALID_VALUE


def test_noalloc_limits_on_host(lib):
    """The no-allocation Predict's size check needs no GPU."""
    b, fits = krr.krr_noalloc_limits(32768, 20000, 16)
    assert b == krr.KRR_NOALLOC_SCRATCH_BYTES == 64 << 20 and fits
    assert not krr.krr_noalloc_limits(200000, 20000, 128)[1]  # X alone is 205 MB
    assert not krr.krr_noalloc_limits(1000, 20_000_000, 1)[1]  # test-row norms 80 MB
    assert not krr.krr_noalloc_limits(1000, 10, 5000)[1]  # more columns than Predict takes
    b, f = ctypes.c_int64(), ctypes.c_int32()
    assert lib.krr_noalloc_limits(0, 1, 1, 512, ctypes.byref(b), ctypes.byref(f)) == \
        krr.KRR_ERROR_INVALID_VALUE
    assert lib.krr_predict_noalloc(None, None, None, 1, 16, None, 1, 1, None, 1) == \
        krr.KRR_ERROR_INVALID_VALUE


def test_tuning_cache_round_trip(lib, tmp_path):
    """The autotuner's cache file (host code, no GPU): entries are added and
    replaced by key, survive a re-read, absent keys and files read as not found,
    and malformed entries or invalid tunings are rejected."""
    path = str(tmp_path / "tune.json")
    assert krr.krr_tuning_cache_load(path, "k1") is None  # no file yet
    a = {"tile": 512, "panel_group": 8, "residual_split": 8, "sweep_pairs": 1, "lookahead": 1,
         "aux_cu_eighths": 7}
    b = {"tile": 256, "panel_group": 4, "residual_split": 16, "sweep_pairs": 0, "lookahead": -1,
         "aux_cu_eighths": 0}
    krr.krr_tuning_cache_store(path, "gfx950|cu256|n32768|m65536|r16|mode1|d641|ref1", a, 85.25)
    krr.krr_tuning_cache_store(path, "k2", b, 12.5)
    assert krr.krr_tuning_cache_load(path, "gfx950|cu256|n32768|m65536|r16|mode1|d641|ref1") == \
        (a, 85.25)
    assert krr.krr_tuning_cache_load(path, "k2") == (b, 12.5)
    krr.krr_tuning_cache_store(path, "k2", a, 10.0)  # replaced, the other kept
    assert krr.krr_tuning_cache_load(path, "k2") == (a, 10.0)
    assert krr.krr_tuning_cache_load(path, "k3") is None
    import json
    doc = json.load(open(path))  # the file is plain JSON
    assert set(doc) == {"gfx950|cu256|n32768|m65536|r16|mode1|d641|ref1", "k2"}
    assert doc["k2"]["ms"] == 10.0
    bad = dict(a, tile=300)
    with pytest.raises(krr.KRRError):
        krr.krr_tuning_cache_store(path, "k4", bad, 1.0)
    with open(path, "a") as f:
        f.write('"k5": {"tile": 512, "panel_group": oops}\n')
    with pytest.raises(krr.KRRError):
        krr.krr_tuning_cache_load(path, "k5")
    assert krr.krr_tuning_cache_load(path, "k2") == (a, 10.0)
    # a tuning is validated before it reaches a context
    t = krr.krr_tuning(300, 0, 0, -1, -1, 0)
    assert lib.krr_set_tuning(None, ctypes.byref(t)) == krr.KRR_ERROR_INVALID_VALUE
