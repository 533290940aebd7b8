"""Host-side checks of the C ABI: the library builds, loads and exports every
entry point that include/skh.h declares; argument validation that needs no GPU."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skh.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared_functions()
    for required in ("skh_create", "skh_destroy", "skh_softmin", "skh_sinkhorn_divergence",
                     "skh_last_error", "skh_params_default", "skh_set_stream"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2107_02010_amd import _lib
    lib = _lib.load()
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows a signature for each of them
    assert set(_declared_functions()) <= set(_lib.SIGNATURES)


def test_params_default_and_struct_layout():
    from paper_2107_02010_amd import _lib
    p = _lib.default_params()
    assert p.blur == 0.05 and math.isinf(p.reach) and p.scaling == 0.9
    assert p.tol == 0.0 and p.extra_iters == 0 and p.max_iters == 1000 and p.check_every == 5
    assert p.precision == _lib.SKH_FP32 and p.init == 0 and p.timing == 0
    assert p.multiscale == 0 and p.jump_scale == 0.0 and p.trunc_theta == 20.0
    assert p.n_clusters == 0 and p.kmeans_iters == 10


def test_struct_layout_matches_c_compiler(tmp_path):
    # Offsets and sizes as the C compiler lays out the header's structs.
    from paper_2107_02010_amd import _lib
    fields = {"skh_params": [f for f, _ in _lib.SkhParams._fields_],
              "skh_stats": [f for f, _ in _lib.SkhStats._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "skh.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for st, cls in (("skh_params", _lib.SkhParams), ("skh_stats", _lib.SkhStats)):
        assert int(got[st]) == ctypes.sizeof(cls)
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_null_context_and_arguments_are_rejected():
    from paper_2107_02010_amd import _lib
    lib = _lib.load()
    assert lib.skh_softmin(None, None, 1, None, 1, 3, None, None, 1.0, 1.0, 0, None) == \
        _lib.SKH_EINVAL
    P = _lib.default_params()
    assert lib.skh_sinkhorn_divergence(None, None, None, 1, None, None, 1, 3, ctypes.byref(P),
                                       None, None, None, None, None, None) == _lib.SKH_EINVAL
    out = ctypes.c_void_p()
    assert lib.skh_create(None, 0, None) == _lib.SKH_EINVAL
    assert lib.skh_create(ctypes.byref(out), -1, None) != _lib.SKH_OK
    assert lib.skh_last_error(None)  # a message is recorded for the failed create


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2107_02010_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_bench_refuses_several_gpus():
    # the benchmark is single-device: --gpus N > 1 exits with a message, before any
    # GPU work
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
