"""Host-side checks of the C ABI (no GPU needed).

The shared library must load, export every function include/gve.h declares,
and reject bad arguments on the host before any device work.
"""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gve.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gve_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2608_14112_amd as g

    lib = ctypes.CDLL(g.LIB_PATH)
    names = declared_functions()
    assert "gve_refine" in names and "gve_evaluate" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    assert sorted(set(g.EXPORTED)) == names


def test_default_options_and_status_strings():
    import paper_2608_14112_amd as g

    o = g.default_options()
    assert o.k == 3.0 and o.brick == 8 and o.brick_z == 32 and o.deterministic == 0
    assert o.schedule == g.SCHED_XCD
    assert abs(o.lr - 8e-3) < 1e-9 and abs(o.beta1 - 0.9) < 1e-7 and abs(o.beta2 - 0.999) < 1e-7
    assert math.isinf(o.ell_min) and math.isinf(o.ell_max)
    for s in range(7):
        assert g._lib.gve_status_string(s)
    assert g._lib.gve_status_string(99) == b"unknown status"
    assert g._lib.gve_last_error(None) == b""


def test_null_arguments_are_rejected():
    import paper_2608_14112_amd as g

    lib = g._lib
    assert lib.gve_default_options(None) == g.INVALID_ARGUMENT
    assert lib.gve_create(None, None, None) == g.INVALID_ARGUMENT
    assert lib.gve_destroy(None) == g.INVALID_ARGUMENT
    assert lib.gve_params_destroy(None) == g.INVALID_ARGUMENT
    n = ctypes.c_int64()
    assert lib.gve_params_size(None, ctypes.byref(n)) == g.INVALID_ARGUMENT
    assert lib.gve_evaluate(None, None, g.GridC(1, 1, 1, 0, 0, 0), None) == g.INVALID_ARGUMENT
    assert lib.gve_refine(None, None, None, g.GridC(1, 1, 1, 0, 0, 0), 1, None) == g.INVALID_ARGUMENT
    assert lib.gve_get_stats(None, None) == g.INVALID_ARGUMENT


@pytest.mark.parametrize("field,value,status", [
    ("k", -1.0, 1), ("k", float("nan"), 1), ("k", 0.0, 1), ("brick", 4, 6), ("brick", 7, 6),
    ("brick_z", 4, 6), ("brick_z", 24, 6),
    ("lr", -1.0, 1), ("beta1", 1.0, 1), ("beta2", -0.1, 1), ("eps", 0.0, 1),
    ("ell_min", 3.0, 1), ("deterministic", 2, 1), ("brick_waves", 3, 6),
])
def test_bad_options_fail_before_any_device_call(field, value, status):
    import paper_2608_14112_amd as g

    o = g.default_options()
    setattr(o, field, value)
    if field == "ell_min":
        o.ell_max = 2.0
    h = ctypes.c_void_p()
    assert g._lib.gve_create(ctypes.byref(h), ctypes.byref(o), None) == status
    assert not h.value


def test_export_and_checkpoint_sizes():
    import paper_2608_14112_amd as g
    from oracle import field as F

    lib = ctypes.CDLL(g.LIB_PATH)
    lib.gve_export_size.argtypes = [ctypes.c_int64]
    lib.gve_export_size.restype = ctypes.c_size_t
    lib.gve_checkpoint_size.argtypes = [ctypes.c_int64]
    lib.gve_checkpoint_size.restype = ctypes.c_size_t
    for n in (1, 2000, 1_400_000):
        assert lib.gve_export_size(n) == F.encoded_bytes(n, g.EXPORT_HEADER)
        assert lib.gve_checkpoint_size(n) == 32 + 3 * 44 * n
    assert lib.gve_export_size(0) == g.EXPORT_HEADER
    assert lib.gve_export_size(-5) == g.EXPORT_HEADER


STRUCTS = [("gve_grid", "GridC"), ("gve_options", "OptionsC"), ("gve_stats", "StatsC"),
           ("gve_alloc_info", "AllocInfoC"), ("gve_probe_rates", "ProbeC"),
           ("gve_tune_entry", "TuneEntryC"), ("gve_paper_options", "PaperOptionsC")]


def test_binding_structs_match_the_header(tmp_path):
    """Size and field offsets of every ABI struct, as the C compiler lays them
    out from include/gve.h, equal the binding's ctypes mirrors."""
    import shutil
    import subprocess

    import paper_2608_14112_amd as g
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gve.h"', "int main(void) {"]
    for cname, pyname in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in getattr(g, pyname)._fields_:
            lines.append(f'  printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], check=True, capture_output=True, text=True)
               .stdout.splitlines())
    for cname, pyname in STRUCTS:
        cls = getattr(g, pyname)
        assert int(out[f"{cname} size"]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(out[f"{cname}.{field}"]) == getattr(cls, field).offset, (cname, field)


def test_binding_maps_one_hip_runtime():
    """Importing the binding (in a fresh process, before anything else) leaves
    one HIP runtime mapped, torch's: the library's dependency resolves to it."""
    import subprocess
    import sys

    code = ("import paper_2608_14112_amd\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"
