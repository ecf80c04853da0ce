"""The product path stands on the HIP library alone: no module of the
package imports the oracle or the scene generators, and with the library
missing every entry point raises instead of computing on the CPU."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2501_13382_amd")


def test_package_imports_neither_oracle_nor_scenes():
    for name in os.listdir(PKG):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, name)).read())
        for node in ast.walk(tree):
            mods = []
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            for m in mods:
                assert not m.split(".")[0] in ("oracle", "scenes"), (name, m)
    for name in os.listdir(os.path.join(PKG, "csrc")):
        text = open(os.path.join(PKG, "csrc", name)).read()
        assert "gbso_" not in text and "oracle" not in text.lower(), name


def test_missing_library_raises():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2501_13382_amd import _lib\n"
        "_lib.LIB_PATH = '/nonexistent/libgbs.so'\n"
        "import paper_2501_13382_amd as gbs\n"
        "try:\n"
        "    gbs.air_absorption([1000.0])\n"
        "except RuntimeError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('computed')\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert "raised" in r.stdout and "not built" in r.stdout, r.stdout + r.stderr


def test_autograd_takes_eps_e2_as_an_input_only():
    """GBSFunction differentiates anisotropic beams through its last input;
    eps_e2 smuggled in through the options is refused before any work (it
    would get no gradient)."""
    import pytest
    import torch

    sys.path.insert(0, ROOT)
    import paper_2501_13382_amd as gbs
    g = torch.zeros(1, dtype=torch.complex128, requires_grad=True)
    r = torch.zeros((1, 3), dtype=torch.float64, requires_grad=True)
    e = torch.ones((1, 1), dtype=torch.float64, requires_grad=True)
    with pytest.raises(ValueError):
        gbs.GBSFunction.apply(g, r, e, None, torch.ones(1, dtype=torch.float64), {"eps_e2": torch.ones(1)})
