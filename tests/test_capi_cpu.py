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


def test_setup_validates_parameters_before_touching_a_device():
    """msm_setup checks its parameters first: invalid ones are rejected with
    MSM_ERR_ARG (-1) or MSM_ERR_UNSUPPORTED (-6) without any HIP call (on a
    host with no GPU, valid ones get as far as the device query)."""
    import ctypes as C
    from paper_1309_1889_amd import binding

    def setup(**kw):
        p = binding._Params()
        p.a, p.h, p.levels, p.precision = 1.2, 0.25, 0, binding.MSM_FP32
        for d in range(3):
            p.lo[d], p.hi[d] = 0.0, 3.0
        p.coulomb_k, p.max_atoms, p.max_systems = 138.935458, 100, 1
        p.method, p.smoothing, p.basis, p.alpha = 0, 2, 3, 0.0
        for k, v in kw.items():
            setattr(p, k, v)
        h = C.c_void_p()
        return binding.lib().msm_setup(C.byref(p), None, C.byref(h))

    assert setup(a=-1.0) == -1
    assert setup(method=7) == -1
    assert setup(method=2, alpha=-1.0) == -1
    assert setup(method=2, alpha=float("nan")) == -1
    assert setup(smoothing=4) == -6
    assert setup(basis=4) == -6
    assert setup(h=0.01) == -6          # a/h beyond the stencil's reach
    assert setup(method=1, h=0.01) != -6   # no stencil for the cutoff method
