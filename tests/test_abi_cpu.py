"""Host-only checks of the C ABI: the library loads and exports every
function include/gbs.h declares; struct layouts match the header."""
import ctypes
import os
import subprocess
import re

import pytest

from paper_2501_13382_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbs_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgbs.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert _lib.load().gbs_version() == 4


def test_struct_sizes_match_c_layout():
    assert ctypes.sizeof(_lib.GbsRays) == 40
    assert ctypes.sizeof(_lib.GbsSegs) == 72
    assert ctypes.sizeof(_lib.GbsFaces) == 16
    assert ctypes.sizeof(_lib.GbsParams) == 56
    assert ctypes.sizeof(_lib.GbsStats) == 72
    assert ctypes.sizeof(_lib.GbsScene) == 32
    assert ctypes.sizeof(_lib.GbsFan) == 56


def test_struct_layouts_match_the_header(tmp_path):
    """Every field offset of the ctypes mirrors equals the C compiler's
    offsetof for include/gbs.h (host compiler, no device code)."""
    structs = {"gbs_rays": _lib.GbsRays, "gbs_segs": _lib.GbsSegs, "gbs_faces": _lib.GbsFaces,
               "gbs_params": _lib.GbsParams, "gbs_stats": _lib.GbsStats, "gbs_scene": _lib.GbsScene,
               "gbs_fan": _lib.GbsFan}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "gbs.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_create_without_gpu_fails_cleanly():
    """With no visible device the context is refused with an error code, no crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgbs.so not built")
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.gbs_create(ctypes.byref(h), 0, None)
    assert rc in (_lib.GBS_E_INVALID, _lib.GBS_E_HIP)
    assert not h.value
    assert lib.gbs_last_error(None) == b"null context"


def test_air_absorption_helper_matches_the_oracle():
    """gbs_air_absorption_db is host code: callable without a device; it
    agrees with the oracle's ISO 9613-1 coefficient and rejects bad input."""
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgbs.so not built")
    import math

    import numpy as np

    import oracle
    lib = _lib.load()
    f = np.geomspace(20.0, 20000.0, 25)
    for T, rh, p in ((20.0, 70.0, 1.0), (-10.0, 30.0, 0.9), (35.0, 95.0, 1.05), (15.0, 0.0, 1.0)):
        got = np.array([lib.gbs_air_absorption_db(x, T, rh, p) for x in f])
        np.testing.assert_allclose(got, oracle.air_absorption_db(f, T, rh, p), rtol=1e-12)
    for bad in ((0.0, 20.0, 70.0, 1.0), (1e3, 20.0, 120.0, 1.0), (1e3, 20.0, 70.0, 0.0)):
        assert math.isnan(lib.gbs_air_absorption_db(*bad))

