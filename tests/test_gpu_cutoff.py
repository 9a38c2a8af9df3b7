"""Parity of the simple cutoff method (Section 5: the coarse propagator the
paper proposes for parareal) and of Wolf summation (its refinement, also
Section 5) on the GPU with the FP64 oracle.

The cutoff is a discontinuity: a pair whose distance is within rounding of
the cutoff may be counted on one side and not on the other. Atoms in such a
pair are left out of the per-atom comparisons (there are few, and the tests
assert that), and the energy tolerance allows for their terms.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import named, rigid_water_velocities, water_box, water_model_arrays

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
KE = 138.935458


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def msmx():
    import paper_1309_1889_amd as m
    return m


def rel_rms(x, ref):
    return float(np.sqrt(((np.asarray(x, np.float64) - ref) ** 2).sum() / (ref ** 2).sum()))


def band(precision):
    """Relative half-width of the band around the cutoff inside which the
    kernel's rounded r^2 < a^2 test and the oracle's may disagree."""
    return 1e-6 if precision == "fp32" else 1e-9


def ambiguous_pairs(xyz, rc, rel):
    """Pairs whose distance lies within rel * rc of the cutoff."""
    from scipy.spatial import cKDTree
    t = cKDTree(xyz)
    pairs = t.query_pairs(rc * (1 + rel), output_type="ndarray")
    if len(pairs) == 0:
        return pairs
    d = np.linalg.norm(xyz[pairs[:, 0]] - xyz[pairs[:, 1]], axis=1)
    return pairs[d > rc * (1 - rel)]


def box(n_mol, side, seed):
    per = int(math.ceil(n_mol ** (1 / 3)))
    return water_box(n_mol, (per,) * 3, (side,) * 3, seed=seed)


@pytest.mark.parametrize("precision,rc,h", [("fp64", 1.2, 0.25), ("fp64", 0.8, 0.5), ("fp32", 1.2, 0.25),
                                            ("fp32", 0.8, 0.5), ("fp32", 1.0, 0.3)])
def test_cutoff_matches_oracle(precision, rc, h):
    w = box(1500, 3.6, seed=51)
    dt = np.float32 if precision == "fp32" else np.float64
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx = msmx().MsmContext(rc, h, w.lo, w.hi, precision=precision, method="cutoff", max_atoms=w.n)
    e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert ctx.grid_shape() == []     # no grids for the cutoff method
    eo, fo, po = oracle.cutoff(w.xyz, w.q, rc)
    amb = ambiguous_pairs(w.xyz, rc, band(precision))
    assert len(amb) <= 0.005 * w.n
    keep = np.setdiff1d(np.arange(w.n), amb.ravel())
    f = f.double().cpu().numpy()
    p = p.double().cpu().numpy()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert rel_rms(f[keep], fo[keep]) < tol
    assert rel_rms(p[keep], po[keep]) < tol
    slack = sum(KE * abs(w.q[i] * w.q[j]) / rc for i, j in amb)
    assert abs(e.item() - eo) <= tol * abs(eo) + slack


def test_cutoff_beyond_the_box_is_exact_coulomb():
    """Below the cutoff the method is Coulomb's law: with a cutoff longer than
    any distance in the box every pair counts and the result is exact Coulomb
    (the brute-force pair sum)."""
    w = box(200, 1.8, seed=52)
    ctx = msmx().MsmContext(4.0, 0.5, w.lo, w.hi, precision="fp64", method="cutoff", max_atoms=w.n)
    e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(np.float64), device="cuda"))
    torch.cuda.synchronize()
    ec, fc, pc = oracle.coulomb(w.xyz, w.q)
    assert e.item() == pytest.approx(ec, rel=1e-12)
    assert rel_rms(f.cpu().numpy(), fc) < 1e-12
    assert rel_rms(p.cpu().numpy(), pc) < 1e-12


def test_cutoff_batched_equals_separate_bitwise():
    m = msmx()
    ws = [box(n, s, seed) for n, s, seed in [(300, 2.1, 61), (700, 2.8, 62), (150, 1.7, 63)]]
    lo = np.zeros(3)
    hi = np.full(3, max(float((w.hi - w.lo).max()) for w in ws))
    offs = np.cumsum([0] + [w.n for w in ws])
    doms = np.array([np.concatenate([w.lo, w.hi]) for w in ws])
    big = m.MsmContext(1.0, 0.3, lo, hi, precision="fp32", method="cutoff", max_atoms=int(offs[-1]), max_systems=3)
    x = torch.tensor(np.concatenate([w.xyzq(np.float32) for w in ws]), device="cuda")
    e, f, p = big.energy_forces(x, offs, doms)
    torch.cuda.synchronize()
    for k, w in enumerate(ws):
        one = m.MsmContext(1.0, 0.3, w.lo, w.hi, precision="fp32", method="cutoff", max_atoms=w.n)
        e1, f1, p1 = one.energy_forces(torch.tensor(w.xyzq(np.float32), device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(e[k:k + 1], e1)
        assert torch.equal(f[offs[k]:offs[k + 1]], f1)
        assert torch.equal(p[offs[k]:offs[k + 1]], p1)


def test_cutoff_water_99999_sampled_against_oracle():
    """The 99,999-atom water box in FP32 with the coarse propagator's cutoff
    (1.2 nm on 0.25 nm cells, the launch the parareal benchmark uses), 256
    sampled atoms checked one by one against the direct oracle loop."""
    w = named("water_99999").as_dtype(np.float32)
    rc = 1.2
    ctx = msmx().MsmContext(rc, 0.25, w.lo, w.hi, precision="fp32", method="cutoff", max_atoms=w.n)
    e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(np.float32), device="cuda"))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    rng = np.random.default_rng(71)
    sel = np.sort(rng.choice(w.n, 256, replace=False))
    amb = ambiguous_pairs(w.xyz, rc, band("fp32"))
    sel = np.setdiff1d(sel, amb.ravel())
    assert len(sel) >= 250
    fo, po = oracle.cutoff_subset(w.xyz, w.q, rc, sel)
    assert rel_rms(f.double().cpu().numpy()[sel], fo) < 1e-5
    assert rel_rms(p.double().cpu().numpy()[sel], po) < 1e-5
    # the energy is one half of sum q phi over all atoms (checked on the GPU's own outputs)
    pe = float((w.q * p.double().cpu().numpy()).sum()) * 0.5
    assert e.item() == pytest.approx(pe, rel=1e-6)


# ---------------------------------------------------------------------------
# dynamics with the cutoff method as the coarse propagator
# ---------------------------------------------------------------------------
def small_water(n_mol, side, seed, margin=0.6):
    per = int(math.ceil(n_mol ** (1 / 3)))
    w = water_box(n_mol, (per,) * 3, (side,) * 3, seed=seed, margin=margin)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=seed + 1)
    return w, mass, molid, lj, tri, v


def model_ctx(w, a, h, precision, mass, molid, lj, tri, method, max_atoms=None, max_systems=1):
    c = msmx().MsmContext(a, h, w.lo, w.hi, precision=precision, ke=KE, max_atoms=max_atoms or w.n,
                          max_systems=max_systems, method=method)
    c.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                 torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
    return c


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cutoff_model_forces_match_oracle(precision):
    w, mass, molid, lj, tri, v = small_water(300, 3.0, seed=13)
    dt = np.float32 if precision == "fp32" else np.float64
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx = model_ctx(w, 0.9, 0.3, precision, mass, molid, lj, tri, "cutoff")
    e, f, _ = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    p = oracle.OracleParams(0.9, 0.3, tuple(w.lo), tuple(w.hi), 0, KE, method=oracle.METHOD_CUTOFF)
    eo, fo = oracle.md_forces(p, oracle.OracleModel(mass, molid, lj, True, tri), w.xyz, w.q)
    amb = ambiguous_pairs(w.xyz, 0.9, band(precision))
    keep = np.setdiff1d(np.arange(w.n), amb.ravel())
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert rel_rms(f.double().cpu().numpy()[keep], fo[keep]) < tol
    slack = sum(KE * abs(w.q[i] * w.q[j]) / 0.9 + 1.0 for i, j in amb)
    assert abs(e.item() - eo) <= tol * abs(eo) + slack


def _parareal_inputs(S):
    w, mass, molid, lj, tri, v = small_water(125, 1.55, seed=21)
    q = torch.tensor(w.q, dtype=torch.float64, device="cuda")
    invm = torch.tensor(1.0 / mass, dtype=torch.float64, device="cuda")
    s0 = torch.tensor(np.concatenate([w.xyz, v], 1), dtype=torch.float64, device="cuda").contiguous()
    fine = model_ctx(w, 0.9, 0.25, "fp64", mass, molid, lj, tri, "msm", max_atoms=S * w.n, max_systems=S)
    coarse = model_ctx(w, 0.9, 0.45, "fp64", mass, molid, lj, tri, "cutoff")
    return w, mass, molid, lj, tri, v, q, invm, s0, fine, coarse


def test_parareal_with_cutoff_coarse_is_exact_after_k_iterations():
    S, sf, dtf, sg, dtg = 4, 3, 0.001, 3, 0.001
    w, mass, molid, lj, tri, v, q, invm, s0, fine, coarse = _parareal_inputs(S)
    m = msmx()
    ref = model_ctx(w, 0.9, 0.25, "fp64", mass, molid, lj, tri, "msm")
    serial = [s0.clone()]
    for _ in range(S):
        cur = serial[-1]
        x = torch.cat([cur[:, :3], q[:, None]], 1).contiguous()
        vv = torch.cat([cur[:, 3:], invm[:, None]], 1).contiguous()
        ref.vv_run(x, vv, sf, dtf, energies=False)
        serial.append(torch.cat([x[:, :3], vv[:, :3]], 1))
    torch.cuda.synchronize()
    for K in (1, 2):
        lam, rep, rc = m.parareal(fine, coarse, q, invm, s0, nslices=S, kmax=K, tol=0.0, steps_f=sf, dt_f=dtf,
                                  steps_g=sg, dt_g=dtg)
        torch.cuda.synchronize()
        assert rep["iterations"] == K and rc == 1
        for n in range(K + 1):
            assert torch.equal(lam[n], serial[n]), (K, n)


def test_parareal_with_cutoff_coarse_matches_oracle():
    S, sf, dtf, sg, dtg = 4, 3, 0.001, 3, 0.001
    w, mass, molid, lj, tri, v, q, invm, s0, fine, coarse = _parareal_inputs(S)
    lam, rep, rc = msmx().parareal(fine, coarse, q, invm, s0, nslices=S, kmax=2, tol=0.0, steps_f=sf, dt_f=dtf,
                                   steps_g=sg, dt_g=dtg)
    torch.cuda.synchronize()
    pf = oracle.OracleParams(0.9, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    pg = oracle.OracleParams(0.9, 0.45, tuple(w.lo), tuple(w.hi), 0, KE, method=oracle.METHOD_CUTOFF)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    lo_, it, res, rco = oracle.parareal(pf, pg, model, w.xyz, v, w.q, S, sf, dtf, sg, dtg, 2, 0.0)
    assert it == rep["iterations"] == 2
    got = lam.cpu().numpy()
    assert np.abs(got[..., :3] - lo_[..., :3]).max() < 1e-9
    assert np.abs(got[..., 3:] - lo_[..., 3:]).max() < 1e-6
    np.testing.assert_allclose(rep["residual"], res, rtol=1e-5, atol=1e-12)


# ---------------------------------------------------------------------------
# Wolf summation (Section 5's refinement of the simple cutoff)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision,rc,h,alpha", [("fp64", 1.2, 0.25, 2.0), ("fp64", 0.9, 0.3, 3.5),
                                                  ("fp32", 1.2, 0.25, 2.0), ("fp32", 0.9, 0.45, 3.5)])
def test_wolf_matches_oracle(precision, rc, h, alpha):
    w = box(1500, 3.6, seed=53)
    dt = np.float32 if precision == "fp32" else np.float64
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx = msmx().MsmContext(rc, h, w.lo, w.hi, precision=precision, method="wolf", alpha=alpha, max_atoms=w.n)
    e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
    torch.cuda.synchronize()
    assert ctx.status() == 0
    eo, fo, po = oracle.wolf(w.xyz, w.q, rc, alpha)
    # the Wolf potential vanishes at the cutoff, so only the (small) force
    # jump of pairs within rounding of it is ambiguous
    amb = ambiguous_pairs(w.xyz, rc, band(precision))
    keep = np.setdiff1d(np.arange(w.n), amb.ravel())
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert rel_rms(f.double().cpu().numpy()[keep], fo[keep]) < tol
    assert rel_rms(p.double().cpu().numpy(), po) < tol
    assert e.item() == pytest.approx(eo, rel=tol)


def test_wolf_model_forces_match_oracle():
    w, mass, molid, lj, tri, v = small_water(300, 3.0, seed=14)
    c = msmx().MsmContext(0.9, 0.3, w.lo, w.hi, precision="fp64", ke=KE, max_atoms=w.n, method="wolf", alpha=3.0)
    c.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                 torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
    e, f, _ = c.energy_forces(torch.tensor(w.xyzq(np.float64), device="cuda"))
    torch.cuda.synchronize()
    p = oracle.OracleParams(0.9, 0.3, tuple(w.lo), tuple(w.hi), 0, KE, method=oracle.METHOD_WOLF, alpha=3.0)
    eo, fo = oracle.md_forces(p, oracle.OracleModel(mass, molid, lj, True, tri), w.xyz, w.q)
    amb = ambiguous_pairs(w.xyz, 0.9, band("fp64"))
    keep = np.setdiff1d(np.arange(w.n), amb.ravel())
    assert rel_rms(f.cpu().numpy()[keep], fo[keep]) < 1e-11
    assert e.item() == pytest.approx(eo, rel=1e-11)


def test_parareal_with_wolf_coarse_matches_oracle_and_is_exact():
    S, sf, dtf, sg, dtg = 4, 3, 0.001, 3, 0.001
    w, mass, molid, lj, tri, v = small_water(125, 1.55, seed=21)
    q = torch.tensor(w.q, dtype=torch.float64, device="cuda")
    invm = torch.tensor(1.0 / mass, dtype=torch.float64, device="cuda")
    s0 = torch.tensor(np.concatenate([w.xyz, v], 1), dtype=torch.float64, device="cuda").contiguous()
    fine = model_ctx(w, 0.9, 0.25, "fp64", mass, molid, lj, tri, "msm", max_atoms=S * w.n, max_systems=S)
    coarse = msmx().MsmContext(0.9, 0.45, w.lo, w.hi, precision="fp64", ke=KE, max_atoms=w.n, method="wolf",
                               alpha=3.0)
    coarse.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                      torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
    lam, rep, rc = msmx().parareal(fine, coarse, q, invm, s0, nslices=S, kmax=2, tol=0.0, steps_f=sf, dt_f=dtf,
                                   steps_g=sg, dt_g=dtg)
    torch.cuda.synchronize()
    pf = oracle.OracleParams(0.9, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    pg = oracle.OracleParams(0.9, 0.45, tuple(w.lo), tuple(w.hi), 0, KE, method=oracle.METHOD_WOLF, alpha=3.0)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    lo_, it, res, rco = oracle.parareal(pf, pg, model, w.xyz, v, w.q, S, sf, dtf, sg, dtg, 2, 0.0)
    assert it == rep["iterations"] == 2
    got = lam.cpu().numpy()
    assert np.abs(got[..., :3] - lo_[..., :3]).max() < 1e-9
    assert np.abs(got[..., 3:] - lo_[..., 3:]).max() < 1e-6
    # slices 0..2 equal the serial fine trajectory bitwise
    ref = model_ctx(w, 0.9, 0.25, "fp64", mass, molid, lj, tri, "msm")
    cur = s0.clone()
    for n in range(1, 3):
        x = torch.cat([cur[:, :3], q[:, None]], 1).contiguous()
        vv = torch.cat([cur[:, 3:], invm[:, None]], 1).contiguous()
        ref.vv_run(x, vv, sf, dtf, energies=False)
        cur = torch.cat([x[:, :3], vv[:, :3]], 1)
        torch.cuda.synchronize()
        assert torch.equal(lam[n], cur), n
