"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpmul.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(polymul\w*)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("polymul", "polymul_ex", "polymul_ctx_create", "polymul_ctx_destroy",
                 "polymul_addfft", "polymul_iaddfft", "polymul_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1803_11301_amd import fpmul
    if not os.path.exists(fpmul.LIB_PATH):
        pytest.skip("libfpmul.so not built")
    L = ctypes.CDLL(fpmul.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) <= set(fpmul.SIGNATURES)
    assert fpmul.version().startswith("fpmul")


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_1803_11301_amd import fpmul
    monkeypatch.setattr(fpmul, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fpmul, "_lib", None)
    with pytest.raises(FileNotFoundError):
        fpmul.lib()


def test_library_exports_nothing_undeclared():
    # every polymul* function the library exports is declared in fpmul.h
    import shutil
    import subprocess
    from paper_1803_11301_amd import fpmul
    if not os.path.exists(fpmul.LIB_PATH) or not shutil.which("nm"):
        pytest.skip("libfpmul.so not built or nm missing")
    out = subprocess.run(["nm", "-D", "--defined-only", fpmul.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {f[2] for f in (line.split() for line in out.splitlines())
                if len(f) == 3 and f[1] == "T" and f[2].startswith("polymul")}
    assert exported, "no polymul* symbols found"
    assert exported <= set(declared_functions()), sorted(exported - set(declared_functions()))
