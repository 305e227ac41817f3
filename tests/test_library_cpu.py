"""Host-side checks of the C-ABI library that need no GPU: it loads, and it
exports every entry point that include/sgsolve.h declares (no compute call
is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgsolve.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    # function declarations (typedefs of function pointers are not entry points)
    names = re.findall(r"^(?!\s*typedef)\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*"
                       r"([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_method_calls():
    names = _declared()
    for call in ("sg_build_triples", "sg_assemble", "sg_matvec", "ras_apply", "amg_vcycle",
                 "fgmres_solve", "newton_solve"):
        assert call in names


def test_library_exports_every_declared_symbol():
    from paper_2310_14649_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(binding.exported_symbols()) <= set(_declared())
    assert binding.lib().sg_version() >= 1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2310_14649_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()
