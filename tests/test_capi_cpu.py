"""Host-only checks of the C-ABI library: it loads and exports every entry
point that include/msm.h declares (no compute call; there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("msm_setup", "msm_energy_forces", "msm_destroy", "msm_get_status", "parareal_run",
                     "msm_vv_run", "msm_md_bind"):
        assert required in names
    assert len(names) >= 12


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1309_1889_amd import binding
    path = binding.lib_path()
    if not os.path.exists(path):
        pytest.fail("libmsmx.so is not built; run `python -m paper_1309_1889_amd.build`")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    from paper_1309_1889_amd import binding
    binding.lib()
    assert binding.status_string(0) == "ok"
    assert "domain" in binding.status_string(-2)
    assert "unknown" in binding.status_string(-99)


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    from paper_1309_1889_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "lib_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        binding.lib()
