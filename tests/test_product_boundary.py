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
