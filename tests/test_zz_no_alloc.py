"""msm_energy_forces_noalloc (every work array in the library's static device
array) against msm_energy_forces on a context with the default launch
configuration: two calls in a row, the second with a smaller input, in both
precisions; a system too large for the array is refused before any launch.
Both entry points run the same kernels in the same order, so the results
must agree bitwise (the bar for floating point is the 1e-12 relative
tolerance of the FP64 parity tests; bitwise equality is checked too)."""
import numpy as np
import pytest

from workloads import named, water_box

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _reference(w, precision):
    import paper_1309_1889_amd as m
    dt = np.float32 if precision == "fp32" else np.float64
    ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, levels=w.levels, precision=precision, max_atoms=w.n)
    ctx.set_tuning(concurrent=0)
    xyzq = torch.tensor(w.xyzq(dt), device="cuda")
    e, f, p = ctx.energy_forces(xyzq)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    out = (e.cpu().numpy().copy(), f.cpu().numpy().copy(), p.cpu().numpy().copy())
    ctx.close()
    return xyzq, out


def _noalloc(w, precision, xyzq):
    import paper_1309_1889_amd as m
    e, f, p, st = m.energy_forces_noalloc(xyzq, w.a, w.h, w.lo, w.hi, levels=w.levels, precision=precision)
    torch.cuda.synchronize()
    return int(st.item()), (e.cpu().numpy(), f.cpu().numpy(), p.cpu().numpy())


def _agree(got, ref, what):
    for g, r, name in zip(got, ref, ("energy", "forces", "potentials")):
        g = np.asarray(g, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        err = np.abs(g - r).max() / max(np.abs(r).max(), 1e-300)
        assert err <= 1e-12, f"{what} {name}: max rel {err:.3e}"
        assert np.array_equal(g, r), f"{what} {name}: not bitwise equal (max rel {err:.3e})"


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_context_two_calls(precision):
    big = named("water_99999")
    small = water_box(3333, (15, 15, 15), (4.6, 4.6, 4.6), seed=7, margin=0.3, name="water_9999")
    print(f"noalloc {precision}: {big.n} atoms, then {small.n}", flush=True)
    xb, ref_b = _reference(big, precision)
    xs, ref_s = _reference(small, precision)
    st, got_b = _noalloc(big, precision, xb)
    assert st == 0
    _agree(got_b, ref_b, f"{precision} first call ({big.n} atoms)")
    st, got_s = _noalloc(small, precision, xs)
    assert st == 0
    _agree(got_s, ref_s, f"{precision} second call ({small.n} atoms)")


def test_noalloc_refuses_what_does_not_fit_and_reports_status():
    import paper_1309_1889_amd as m
    w = named("charges_2000")
    x = torch.tensor(w.xyzq(np.float64), device="cuda")
    # a 60 nm domain: its grids exceed the static array
    with pytest.raises(m.MsmError) as e:
        m.energy_forces_noalloc(x, w.a, w.h, (0.0, 0.0, 0.0), (60.0, 60.0, 60.0), precision="fp64")
    assert e.value.code == -4
    # an atom outside the domain is reported through the status word
    x2 = x.clone()
    x2[5, 0] = 4.6
    _, _, _, st = m.energy_forces_noalloc(x2, w.a, w.h, w.lo, w.hi, levels=w.levels, precision="fp64")
    torch.cuda.synchronize()
    assert int(st.item()) == -2
    # and the next call starts clean
    _, _, _, st = m.energy_forces_noalloc(x, w.a, w.h, w.lo, w.hi, levels=w.levels, precision="fp64")
    torch.cuda.synchronize()
    assert int(st.item()) == 0
