"""The C-ABI library loads and exports every function include/tufrg.h declares
(CPU only: no compute call is made)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tufrg.h")
LIB = os.path.join(ROOT, "paper_1710_08830_amd", "libtufrg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tufrg_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tufrg_bubble", "tufrg_project", "tufrg_rhs", "tufrg_flow", "tufrg_create",
                     "tufrg_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import __graft_entry__ as g

        g.build()
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1710_08830_amd import tufrg

    assert sorted(tufrg.SYMBOLS) == declared_functions()


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No fallback: importing the binding from a package copy that lacks
    libtufrg.so raises ImportError naming the missing file."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1710_08830_amd"
    pkg.mkdir()
    for f in ("__init__.py", "tufrg.py"):
        shutil.copy(os.path.join(ROOT, "paper_1710_08830_amd", f), pkg / f)
    r = subprocess.run([sys.executable, "-c", "import paper_1710_08830_amd.tufrg"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libtufrg.so is missing" in r.stderr
