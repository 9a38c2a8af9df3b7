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
                     "parareal_window_run", "msm_vv_run", "msm_vv_mts_run", "msm_md_bind"):
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


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field
    offsets (a C program built from include/msm.h prints them)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_1309_1889_amd import binding
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"msm_params": binding._Params, "msm_md_model": binding._Model,
               "parareal_params": binding._PararealParams, "parareal_report": binding._PararealReport,
               "parareal_window_params": binding._WindowParams, "parareal_window_state": binding.WindowState,
               "msm_tuning": binding._Tuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "msm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_window_run_validates_arguments_before_touching_a_device():
    import ctypes as C
    from paper_1309_1889_amd import binding
    pp = binding._WindowParams()
    st = binding.WindowState()
    L = binding.lib()
    assert L.parareal_window_run(None, None, C.byref(pp), 3, None, None, None, None, C.byref(st)) == -1


def test_binding_validates_tensors_and_offsets():
    """The C side cannot check buffer sizes, so the binding rejects tensors
    of the wrong dtype, shape, device or layout and offsets that do not
    partition the atoms, before any library call."""
    import numpy as np
    import torch
    from paper_1309_1889_amd import binding
    cpu = torch.device("cpu")
    binding._require(None, "x", torch.float32, cpu, (3,))
    binding._require(torch.zeros(3), "x", torch.float32, cpu, (3,))
    with pytest.raises(ValueError):
        binding._require(torch.zeros(3, dtype=torch.float64), "x", torch.float32, cpu, (3,))
    with pytest.raises(ValueError):
        binding._require(torch.zeros(4), "x", torch.float32, cpu, (3,))
    with pytest.raises(ValueError):
        binding._require(torch.zeros(3, 2).t(), "x", torch.float32, cpu, (2, 3))
    if torch.cuda.is_available():
        with pytest.raises(ValueError):
            binding._require(torch.zeros(3), "x", torch.float32, torch.device("cuda", 0), (3,))
    assert list(binding._offsets(None, 5)) == [0, 5]
    assert list(binding._offsets([0, 2, 5], 5)) == [0, 2, 5]
    for bad in ([1, 5], [0, 4], [0, 3, 2, 5], [0]):
        with pytest.raises(ValueError):
            binding._offsets(bad, 5)
    dom, ptr = binding._domains(np.zeros(12), 2)
    assert dom.shape == (2, 6) and ptr is not None
    with pytest.raises(ValueError):
        binding._domains(np.zeros(6), 2)
