"""The C-ABI library builds, loads and exports every symbol the header
declares (CPU only: no compute calls)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "vembddc.h")).read()
    return sorted(set(re.findall(r"\b(vb_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vb_create", "vb_assemble", "vb_setup", "vb_apply", "vb_pcg_solve",
                     "vb_get_local_solution", "vb_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2304_09770_amd.build import build
        build()
    lib = binding.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(binding.exported_symbols()) == _declared()


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    from paper_2304_09770_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.load()
