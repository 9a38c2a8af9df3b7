"""Full-size workloads on the GPU, and the autograd path.

- 999,999-atom water box in FP32 through ``msm_energy`` (autograd): the
  backward gradient against central finite differences of the FP64 GPU
  energy at 64 random atoms (step 1e-4 nm), the charge gradient against the
  exact central difference of the quadratic form, and the whole gradient
  against the FP64 oracle.
- 12,675,000-atom water slab (the paper's 30 x 65 x 65 nm box) against one
  full FP64 oracle evaluation: FP32 outputs and all eight levels' grids at
  the single-precision bound, FP64 ones at rounding level, and the
  grid-charge moments against the atoms' moments.
"""
import numpy as np
import pytest

import oracle
from workloads import named, uniform_pm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def m():
    import paper_1309_1889_amd as msmx
    return msmx


def rel_rms(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))


def max_rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def test_autograd_gradcheck_small_fp64():
    msmx = m()
    w = uniform_pm(40, 2.0, seed=9, a=0.7, h=0.25)
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp64", ke=1.0, max_atoms=w.n)
    pos = torch.tensor(w.xyz, dtype=torch.float64, device="cuda", requires_grad=True)
    q = torch.tensor(w.q, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda p_, q_: msmx.msm_energy(p_, q_, ctx), (pos, q), eps=1e-6, atol=1e-6,
                                    rtol=1e-5)


def test_autograd_999999_fd_and_oracle():
    msmx = m()
    w = named("water_999999").as_dtype(np.float32)
    n = w.n
    ctx32 = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=n)
    ctx64 = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp64", max_atoms=n)
    pos = torch.tensor(w.xyz, dtype=torch.float32, device="cuda", requires_grad=True)
    q = torch.tensor(w.q, dtype=torch.float32, device="cuda", requires_grad=True)
    U = msmx.msm_energy(pos, q, ctx32)
    U.sum().backward()
    torch.cuda.synchronize()
    ctx32.check()
    gpos = pos.grad.double().cpu().numpy()
    gq = q.grad.double().cpu().numpy()

    # central finite differences of the FP64 GPU energy (step 1e-4 nm) at 64 atoms
    rng = np.random.default_rng(33)
    atoms = rng.choice(n, 64, replace=False)
    x64 = torch.tensor(w.xyzq(np.float64), device="cuda")
    delta = 1e-4
    fd = np.zeros((64, 3))
    for k, i in enumerate(atoms):
        for d in range(3):
            x64[i, d] += delta
            ep = ctx64.energy_forces(x64, want=("energy",))[0].item()
            x64[i, d] -= 2 * delta
            em = ctx64.energy_forces(x64, want=("energy",))[0].item()
            x64[i, d] += delta
            fd[k, d] = (ep - em) / (2 * delta)
    ctx64.check()
    assert rel_rms(gpos[atoms], fd) < 1e-4
    # the energy is quadratic in the charges: the central difference is exact
    for i in atoms[:8]:
        x64[i, 3] += 0.01
        ep = ctx64.energy_forces(x64, want=("energy",))[0].item()
        x64[i, 3] -= 0.02
        em = ctx64.energy_forces(x64, want=("energy",))[0].item()
        x64[i, 3] += 0.01
        assert gq[i] == pytest.approx((ep - em) / 0.02, rel=1e-4, abs=1e-3)
    # the whole gradient against the FP64 oracle
    eo, fo, po = oracle.msm(oracle.OracleParams.of(w), w.xyz, w.q)
    assert rel_rms(-gpos, fo) < 1e-4
    assert rel_rms(gq, po) < 1e-4
    assert U.item() == pytest.approx(eo, rel=1e-5)


@pytest.fixture(scope="module")
def slab():
    """The 12,675,000-atom slab (float-rounded inputs) and one full FP64
    oracle evaluation of it with every grid (about a minute on 16 cores)."""
    w = named("water_12675000").as_dtype(np.float32)
    print(f"slab: oracle on {w.n} atoms, {oracle.threads()} threads", flush=True)
    eo, fo, po, st = oracle.msm(oracle.OracleParams.of(w), w.xyz, w.q, stages=True)
    return w, (eo, fo, po, st)


def grid_rel_rms(g, ref):
    return rel_rms(g.cpu().numpy(), ref)


@pytest.mark.timeout(1200)
def test_water_slab_12675000_fp32_against_oracle(slab):
    """The paper's 30 x 65 x 65 nm box in FP32 against the FP64 oracle: every
    force and potential, the energy, and the grids q^k and u^k below the top
    (the per-level transfer path that large boxes take), at the 1e-4
    relative RMS bound of the single-precision form."""
    msmx = m()
    w, (eo, fo, po, st_o) = slab
    n = w.n
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=n)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    e, f, p = ctx.energy_forces(x)
    torch.cuda.synchronize()
    ctx.check()
    shapes = ctx.grid_shape()
    assert len(shapes) == 8 == len(st_o["q_grid"])
    assert rel_rms(f.double().cpu().numpy(), fo) < 1e-4
    assert rel_rms(p.double().cpu().numpy(), po) < 1e-4
    assert e.item() == pytest.approx(eo, rel=1e-5)
    st = ctx.stages(n)
    assert rel_rms(st["u_short"].cpu().numpy(), st_o["u_short"]) < 1e-5
    assert rel_rms(st["f_short"].cpu().numpy(), st_o["f_short"]) < 1e-5
    # every grid below the top at the single-precision bound. The top grid
    # (6 x 8 x 8 nodes) holds the residual of charges that cancel almost
    # exactly (the box is neutral), so its single-precision rounding is large
    # relative to its own values; its FP64 values are checked to rounding in
    # the next test, and its contribution is inside u^0 and the outputs above.
    for k in range(len(shapes)):
        assert tuple(st["q_grid"][k].shape) == st_o["q_grid"][k].shape, k
        if k == len(shapes) - 1:
            continue
        assert grid_rel_rms(st["q_grid"][k], st_o["q_grid"][k]) < 1e-4, k
        assert grid_rel_rms(st["ucut_grid"][k], st_o["ucut_grid"][k]) < 1e-4, k
        assert grid_rel_rms(st["u_grid"][k], st_o["u_grid"][k]) < 1e-4, k
    # level-0 grid charges keep the atoms' total charge and dipole (quadratic reproduction of the basis)
    q0 = st["q_grid"][0].cpu().numpy()
    org, dim = shapes[0]
    ax = [w.lo[d] + w.h * (org[d] + np.arange(dim[d])) for d in range(3)]
    assert abs(q0.sum() - w.q.sum()) < 1e-4 * np.abs(q0).sum()
    dip_grid = np.array([(q0.sum(axis=(0, 1)) * ax[0]).sum(), (q0.sum(axis=(0, 2)) * ax[1]).sum(),
                         (q0.sum(axis=(1, 2)) * ax[2]).sum()])
    dip_atoms = (w.q[:, None] * w.xyz).sum(0)
    scale = (np.abs(w.q)[:, None] * np.abs(w.xyz)).sum(0)
    assert np.all(np.abs(dip_grid - dip_atoms) < 1e-5 * scale)


@pytest.mark.timeout(1200)
def test_water_slab_12675000_fp64_against_oracle(slab):
    """The same box in FP64: outputs and every grid of the eight levels equal
    the oracle's to rounding, so the full-size chain (binning, pair sum,
    anterpolation, per-level restriction, lattice cutoff, top level,
    prolongation, interpolation) matches the algorithm step by step."""
    msmx = m()
    w, (eo, fo, po, st_o) = slab
    n = w.n
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp64", max_atoms=n)
    e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(np.float64), device="cuda"))
    torch.cuda.synchronize()
    ctx.check()
    assert e.item() == pytest.approx(eo, rel=1e-11)
    assert max_rel(f.cpu().numpy(), fo) < 1e-10
    assert max_rel(p.cpu().numpy(), po) < 1e-10
    st = ctx.stages(n)
    assert max_rel(st["u_short"].cpu().numpy(), st_o["u_short"]) < 1e-11
    assert max_rel(st["f_short"].cpu().numpy(), st_o["f_short"]) < 1e-11
    for k in range(8):
        assert max_rel(st["q_grid"][k].cpu().numpy(), st_o["q_grid"][k]) < 1e-11, k
        assert max_rel(st["ucut_grid"][k].cpu().numpy(), st_o["ucut_grid"][k]) < 1e-11, k
        assert max_rel(st["u_grid"][k].cpu().numpy(), st_o["u_grid"][k]) < 1e-11, k
