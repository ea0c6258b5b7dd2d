"""The C-ABI library loads and exports every symbol declared in include/mrlt.h
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mrlt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mr_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("mr_init", "mr_adapt", "mr_lt_step", "mr_reconstruct"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1905_08717_amd import build, mrlt
    if not os.path.exists(mrlt.LIB_PATH):
        build.build()
    lib = ctypes.CDLL(mrlt.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(mrlt.EXPORTS) == _declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1905_08717_amd import mrlt
    monkeypatch.setattr(mrlt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mrlt, "_lib", None)
    try:
        mrlt.load_library()
    except ImportError:
        return
    raise AssertionError("binding loaded without the library")
