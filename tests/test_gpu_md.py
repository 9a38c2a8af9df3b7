"""Dynamics on the GPU against the FP64 oracle: forces of the molecular model
(MSM Coulomb with exclusions, Lennard-Jones), velocity Verlet with RATTLE,
batched systems, and parareal (Section 4), including its defining property:
after k iterations slices 0..k equal the serial fine trajectory bitwise."""
import math

import numpy as np
import pytest

import oracle
from workloads import rigid_water_velocities, water_box, water_model_arrays

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


def small_water(n_mol, side, seed, margin=0.6):
    per = int(math.ceil(n_mol ** (1 / 3)))
    w = water_box(n_mol, (per,) * 3, (side,) * 3, seed=seed, margin=margin)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=seed + 1)
    return w, mass, molid, lj, tri, v


def make_ctx(w, a, h, precision, mass, molid, lj, tri, max_atoms=None, max_systems=1, rigid=True, lo=None, hi=None):
    m = msmx()
    ctx = m.MsmContext(a, h, w.lo if lo is None else lo, w.hi if hi is None else hi, precision=precision, ke=KE,
                       max_atoms=max_atoms or w.n, max_systems=max_systems)
    ctx.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                   torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=rigid, tri=tri)
    return ctx


def state_tensors(xyz, v, q, mass):
    """Integrator state: FP64 in both precisions (the forces follow the context)."""
    x = torch.tensor(np.concatenate([xyz, q[:, None]], 1), dtype=torch.float64, device="cuda").contiguous()
    vv = torch.tensor(np.concatenate([v, 1.0 / mass[:, None]], 1), dtype=torch.float64, device="cuda").contiguous()
    return x, vv


def rel_rms(x, ref):
    return float(np.sqrt(((np.asarray(x) - ref) ** 2).sum() / (ref ** 2).sum()))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_model_forces_match_oracle(precision):
    w, mass, molid, lj, tri, v = small_water(300, 3.0, seed=11)
    dt = np.float32 if precision == "fp32" else np.float64
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx = make_ctx(w, 1.0, 0.25, precision, mass, molid, lj, tri)
    p = oracle.OracleParams(1.0, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    eo, fo = oracle.md_forces(p, oracle.OracleModel(mass, molid, lj, True, tri), w.xyz, w.q)
    tol = 1e-11 if precision == "fp64" else 1e-4
    # the excluded intramolecular terms nearly cancel the full Coulomb energy,
    # so the energy is compared on the scale of the terms that cancel
    scale = abs(oracle.msm(p, w.xyz, w.q)[0])
    # cluster forms of 8, 16 and 32 atoms, shared streams; the broadcast form;
    # the pair search in cells of edge h/2
    forms = ((2, 1), (3, 1), (5, 1), (6, 1), (7, 1), (9, 1), (8, 1), (2, 2), (5, 2))
    if precision == "fp32":
        forms += ((10, 1), (10, 2))   # each pair once (Newton's third law)
    for pw, pc in forms:
        ctx.set_tuning(pair_waves=pw, pair_cell=pc)
        e, f, _ = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
        torch.cuda.synchronize()
        assert ctx.status() == 0
        assert rel_rms(f.double().cpu().numpy(), fo) < tol, (pw, pc)
        assert abs(e.item() - eo) < tol * scale, (pw, pc)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", ["hydrogen_sites", "two_oxygen_types"])
def test_model_forces_general_lennard_jones_match_oracle(precision, variant):
    """Lennard-Jones parameters that the one-type pair kernel cannot take:
    sites on the hydrogens too (three per molecule, two types), or two oxygen
    types (one site per molecule). The general kernel reads each atom's
    parameters and molecule; both against the oracle."""
    w, mass, molid, lj, tri, v = small_water(300, 3.0, seed=14)
    lj = lj.copy()
    if variant == "hydrogen_sites":
        lj[1::3] = (0.12, 0.06)
        lj[2::3] = (0.12, 0.06)
    else:
        lj[0::6, 0] *= 1.08
        lj[0::6, 1] *= 0.7
    dt = np.float32 if precision == "fp32" else np.float64
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx = make_ctx(w, 1.0, 0.25, precision, mass, molid, lj, tri)
    p = oracle.OracleParams(1.0, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    eo, fo = oracle.md_forces(p, oracle.OracleModel(mass, molid, lj, True, tri), w.xyz, w.q)
    tol = 1e-11 if precision == "fp64" else 1e-4
    scale = abs(oracle.msm(p, w.xyz, w.q)[0])
    for pw in (2, 5):
        ctx.set_tuning(pair_waves=pw)
        e, f, _ = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
        torch.cuda.synchronize()
        assert ctx.status() == 0
        assert rel_rms(f.double().cpu().numpy(), fo) < tol, pw
        assert abs(e.item() - eo) < tol * scale, pw


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_velocity_verlet_matches_oracle(precision):
    w, mass, molid, lj, tri, v = small_water(216, 1.86, seed=3)
    xyz, vel = w.xyz, v
    ctx = make_ctx(w, 1.0, 0.25, precision, mass, molid, lj, tri)
    x, vv = state_tensors(xyz, vel, w.q, mass)
    ep, ek = ctx.vv_run(x, vv, 10, 0.001)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    p = oracle.OracleParams(1.0, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    xo, vo, epo, eko = oracle.vv(p, model, xyz, vel, w.q, 0.001, 10)
    xg = x[:, :3].cpu().numpy()
    vg = vv[:, :3].cpu().numpy()
    if precision == "fp64":
        assert np.abs(xg - xo).max() < 1e-9
        assert rel_rms(vg, vo) < 1e-7
        assert ep.item() == pytest.approx(epo, rel=1e-8)
        assert ek.item() == pytest.approx(eko, rel=1e-8)
    else:
        assert np.abs(xg - xo).max() < 2e-4
        assert rel_rms(vg, vo) < 2e-3
        assert ek.item() == pytest.approx(eko, rel=2e-3)
    # the rigid geometry holds to the FP64 constraint tolerance in both precisions
    d = xg.reshape(-1, 3, 3)
    lim = 1e-9
    for (a, b), L in zip([(0, 1), (0, 2), (1, 2)], tri):
        assert np.abs(np.linalg.norm(d[:, a] - d[:, b], axis=1) - L).max() < lim
    # RATTLE's velocity stage solves its three linear conditions exactly: no
    # relative velocity along any bond beyond rounding (the tolerance would
    # allow 1e-10 of the bond length squared per ps)
    vgm = vg.reshape(-1, 3, 3)
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        r = d[:, a] - d[:, b]
        w = vgm[:, a] - vgm[:, b]
        along = np.abs((r * w).sum(1)) / (np.linalg.norm(r, axis=1) * np.linalg.norm(w, axis=1) + 1e-300)
        assert along.max() < 1e-11, (a, b, along.max())


def test_uneven_batch_vv_equals_separate_bitwise():
    systems = [small_water(n, s, seed) for n, s, seed in [(64, 1.3, 1), (125, 1.6, 2), (27, 0.95, 3)]]
    lo = np.full(3, -0.6)
    hi = lo + max(float((s[0].hi - s[0].lo).max()) for s in systems)
    sizes = [s[0].n for s in systems]
    offs = np.cumsum([0] + sizes)
    mass = np.concatenate([s[1] for s in systems])
    molid = np.concatenate([s[2] + 1000 * k for k, s in enumerate(systems)]).astype(np.int32)
    lj = np.concatenate([s[3] for s in systems])
    tri = systems[0][4]
    doms = np.array([np.concatenate([s[0].lo, s[0].hi]) for s in systems])
    big = make_ctx(systems[0][0], 0.9, 0.25, "fp32", mass, molid, lj, tri, max_atoms=int(offs[-1]), max_systems=3,
                   lo=lo, hi=hi)
    xs, vs = zip(*[state_tensors(s[0].xyz, s[5], s[0].q, s[1]) for s in systems])
    x = torch.cat(xs).contiguous()
    v = torch.cat(vs).contiguous()
    ep, ek = big.vv_run(x, v, 5, 0.002, offsets=offs, domains=doms)
    torch.cuda.synchronize()
    assert big.status() == 0
    for k, s in enumerate(systems):
        one = make_ctx(s[0], 0.9, 0.25, "fp32", s[1], s[2], s[3], tri)
        x1, v1 = state_tensors(s[0].xyz, s[5], s[0].q, s[1])
        ep1, ek1 = one.vv_run(x1, v1, 5, 0.002)
        torch.cuda.synchronize()
        assert torch.equal(x[offs[k]:offs[k + 1]], x1)
        assert torch.equal(v[offs[k]:offs[k + 1]], v1)
        assert torch.equal(ep[k:k + 1], ep1) and torch.equal(ek[k:k + 1], ek1)


def _parareal_setup(precision, S):
    w, mass, molid, lj, tri, v = small_water(125, 1.55, seed=21)
    xyz, vel = w.xyz, v
    fine = make_ctx(w, 0.9, 0.25, precision, mass, molid, lj, tri, max_atoms=S * w.n, max_systems=S)
    coarse = make_ctx(w, 0.7, 0.5, precision, mass, molid, lj, tri)
    q = torch.tensor(w.q, dtype=torch.float64, device="cuda")
    invm = torch.tensor(1.0 / mass, dtype=torch.float64, device="cuda")
    s0 = torch.tensor(np.concatenate([xyz, vel], 1), dtype=torch.float64, device="cuda").contiguous()
    return w, mass, molid, lj, tri, xyz, vel, fine, coarse, q, invm, s0


def _serial(ctx, s0, q, invm, S, steps, dt):
    """Serial propagation slice by slice from the FP64 slice states."""
    out = [s0.clone()]
    for _ in range(S):
        cur = out[-1]
        x = torch.cat([cur[:, :3], q[:, None]], 1).contiguous()
        v = torch.cat([cur[:, 3:], invm[:, None]], 1).contiguous()
        ctx.vv_run(x, v, steps, dt, energies=False)
        out.append(torch.cat([x[:, :3], v[:, :3]], 1))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_parareal_exact_after_k_iterations(precision):
    S, sf, dtf, sg, dtg = 5, 3, 0.001, 1, 0.003
    w, mass, molid, lj, tri, xyz, vel, fine, coarse, q, invm, s0 = _parareal_setup(precision, S)
    m = msmx()
    # serial references on single-system contexts with the same parameters
    ref_f = make_ctx(w, 0.9, 0.25, precision, mass, molid, lj, tri)
    serial_f = _serial(ref_f, s0, q, invm, S, sf, dtf)
    serial_g = _serial(coarse, s0, q, invm, S, sg, dtg)
    lam0, rep0, _ = m.parareal(fine, coarse, q, invm, s0, nslices=S, kmax=0, tol=0.0, steps_f=sf, dt_f=dtf,
                               steps_g=sg, dt_g=dtg)
    torch.cuda.synchronize()
    for n in range(S + 1):
        assert torch.equal(lam0[n], serial_g[n]), n
    for K in (1, 3, S):
        lam, rep, rc = m.parareal(fine, coarse, q, invm, s0, nslices=S, kmax=K, tol=0.0, steps_f=sf, dt_f=dtf,
                                  steps_g=sg, dt_g=dtg)
        torch.cuda.synchronize()
        assert rep["iterations"] == K
        for n in range(K + 1):
            assert torch.equal(lam[n], serial_f[n]), (K, n)
        if K == S:
            assert rc == 0 and rep["converged"]
        else:
            assert rc == 1
            assert not torch.equal(lam[S], serial_f[S])


def test_parareal_fp64_matches_oracle():
    S, sf, dtf, sg, dtg = 4, 3, 0.001, 1, 0.003
    w, mass, molid, lj, tri, xyz, vel, fine, coarse, q, invm, s0 = _parareal_setup("fp64", S)
    m = msmx()
    lam, rep, rc = m.parareal(fine, coarse, q, invm, s0, nslices=S, kmax=2, tol=0.0, steps_f=sf, dt_f=dtf,
                              steps_g=sg, dt_g=dtg)
    torch.cuda.synchronize()
    pf = oracle.OracleParams(0.9, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    pg = oracle.OracleParams(0.7, 0.5, tuple(w.lo), tuple(w.hi), 0, KE)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    lo_, it, res, rco = oracle.parareal(pf, pg, model, xyz, vel, w.q, S, sf, dtf, sg, dtg, 2, 0.0)
    assert it == rep["iterations"] == 2
    got = lam.cpu().numpy()
    assert np.abs(got[..., :3] - lo_[..., :3]).max() < 1e-9
    assert np.abs(got[..., 3:] - lo_[..., 3:]).max() < 1e-6
    np.testing.assert_allclose(rep["residual"], res, rtol=1e-5, atol=1e-12)


def test_parareal_reports_domain_exit():
    S = 2
    w, mass, molid, lj, tri, xyz, vel, fine, coarse, q, invm, s0 = _parareal_setup("fp64", S)
    m = msmx()
    fast = s0.clone()
    fast[:, 3:] += 500.0      # every atom leaves the domain within the first slice
    with pytest.raises(m.MsmError) as ei:
        m.parareal(fine, coarse, q, invm, fast, nslices=S, kmax=1, tol=0.0, steps_f=2, dt_f=0.002, steps_g=1,
                   dt_g=0.004)
    assert ei.value.code == -2


# ---------------------------------------------------------------------------
# multiple time steps (impulse r-RESPA: grid part slow, short-range part fast)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mts_matches_oracle(precision):
    w, mass, molid, lj, tri, v = small_water(216, 1.86, seed=3)
    ctx = make_ctx(w, 1.0, 0.25, precision, mass, molid, lj, tri)
    x, vv = state_tensors(w.xyz, v, w.q, mass)
    ep, ek = ctx.vv_mts_run(x, vv, 5, 2, 0.002)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    p = oracle.OracleParams(1.0, 0.25, tuple(w.lo), tuple(w.hi), 0, KE)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    xo, vo, epo, eko = oracle.vv_mts(p, model, w.xyz, v, w.q, 0.002, 2, 5)
    xg = x[:, :3].cpu().numpy()
    vg = vv[:, :3].cpu().numpy()
    if precision == "fp64":
        assert np.abs(xg - xo).max() < 1e-9
        assert rel_rms(vg, vo) < 1e-7
        assert ep.item() == pytest.approx(epo, rel=1e-8)
        assert ek.item() == pytest.approx(eko, rel=1e-8)
    else:
        assert np.abs(xg - xo).max() < 2e-4
        assert rel_rms(vg, vo) < 2e-3
        assert ek.item() == pytest.approx(eko, rel=2e-3)
    d = xg.reshape(-1, 3, 3)
    for (a_, b_), L in zip([(0, 1), (0, 2), (1, 2)], tri):
        assert np.abs(np.linalg.norm(d[:, a_] - d[:, b_], axis=1) - L).max() < 1e-9


def test_mts_with_one_inner_step_is_velocity_verlet():
    w, mass, molid, lj, tri, v = small_water(125, 1.55, seed=9)
    ctx = make_ctx(w, 0.9, 0.25, "fp64", mass, molid, lj, tri)
    x1, v1 = state_tensors(w.xyz, v, w.q, mass)
    x2, v2 = state_tensors(w.xyz, v, w.q, mass)
    ep1, ek1 = ctx.vv_run(x1, v1, 6, 0.001)
    ep2, ek2 = ctx.vv_mts_run(x2, v2, 6, 1, 0.001)
    torch.cuda.synchronize()
    assert (x1 - x2).abs().max().item() < 1e-10
    assert (v1 - v2).abs().max().item() < 1e-8
    assert ep2.item() == pytest.approx(ep1.item(), rel=1e-10)


def test_mts_is_for_msm_contexts_only():
    w, mass, molid, lj, tri, v = small_water(27, 0.95, seed=10)
    c = msmx().MsmContext(0.9, 0.25, w.lo, w.hi, precision="fp64", max_atoms=w.n, method="cutoff")
    c.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                 torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
    x, vv = state_tensors(w.xyz, v, w.q, mass)
    with pytest.raises(msmx().MsmError) as ei:
        c.vv_mts_run(x, vv, 1, 2, 0.002)
    assert ei.value.code == -6


def test_constraint_failure_is_a_status_not_a_hang():
    """A tolerance below FP64 resolution cannot be met: every RATTLE loop
    stops at its cap and the step reports MSM_ERR_CONSTRAINT (-7) through the
    status word. A non-finite position stops the loops at once and reports
    MSM_ERR_NONFINITE (-3). Both are ordinary status checks."""
    m = msmx()
    w, mass, molid, lj, tri, v = small_water(60, 1.6, seed=17)
    ctx = m.MsmContext(1.0, 0.25, w.lo, w.hi, precision="fp64", ke=KE, max_atoms=w.n)
    ctx.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                   torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri, tol=1e-30)
    x, vv = state_tensors(w.xyz, v, w.q, mass)
    ctx.vv_run(x, vv, 1, 0.002, energies=False)
    torch.cuda.synchronize()
    assert ctx.status() == -7
    assert ctx.status() == 0          # cleared after reading
    ok = m.MsmContext(1.0, 0.25, w.lo, w.hi, precision="fp64", ke=KE, max_atoms=w.n)
    ok.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                  torch.tensor(lj, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
    x, vv = state_tensors(w.xyz, v, w.q, mass)
    ok.vv_run(x, vv, 2, 0.002, energies=False)
    torch.cuda.synchronize()
    assert ok.status() == 0
    vv[4, 0] = float("nan")
    ok.vv_run(x, vv, 1, 0.002, energies=False)
    torch.cuda.synchronize()
    assert ok.status() == -3


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_binding_after_an_evaluation_rebuilds_the_model_plan(precision):
    """A context that has evaluated without a model and is then bound (and
    rebound with the Lennard-Jones parameters of the hydrogens switched on)
    gives the bits of a fresh context bound the same way: the plan of the
    Lennard-Jones atoms follows the model."""
    m = msmx()
    w, mass, molid, lj, tri, v = small_water(300, 3.0, seed=21)
    dt = np.float32 if precision == "fp32" else np.float64
    x = torch.tensor(w.xyzq(dt), device="cuda")
    ctx = m.MsmContext(1.0, 0.25, w.lo, w.hi, precision=precision, ke=KE, max_atoms=w.n)
    ctx.energy_forces(x)
    lj_all = lj.copy()
    lj_all[1::3] = lj_all[2::3] = (0.1, 0.2)   # hydrogens with Lennard-Jones too
    for table in (lj, lj_all):
        ctx.bind_model(len(mass), torch.tensor(molid, dtype=torch.int32, device="cuda"),
                       torch.tensor(table, dtype=torch.float64, device="cuda"), rigid=True, tri=tri)
        got = ctx.energy_forces(x)
        fresh = make_ctx(w, 1.0, 0.25, precision, mass, molid, table, tri)
        ref = fresh.energy_forces(x)
        torch.cuda.synchronize()
        assert ctx.status() == 0 and fresh.status() == 0
        for a, b in zip(got, ref):
            assert torch.equal(a, b)


def test_molecule_size_limit():
    """Molecules of more than 1024 atoms are refused at binding."""
    m = msmx()
    n = 2048
    ctx = m.MsmContext(1.0, 0.25, np.zeros(3), np.full(3, 4.0), precision="fp32", ke=KE, max_atoms=n)
    molid = torch.zeros(n, dtype=torch.int32, device="cuda")
    molid[1025:] = 1
    with pytest.raises(m.MsmError):
        ctx.bind_model(n, molid, None)
    molid[1024:] = 1
    ctx.bind_model(n, molid, None)   # two molecules of 1024 atoms
