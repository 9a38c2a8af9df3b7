"""Parity of the HIP multilevel summation path with the FP64 CPU oracle.

Both sides get the same seeded inputs (single-precision runs hand the oracle
the float-rounded values promoted to double). The FP64 path must agree with
the oracle to rounding (per stage and in the outputs); the FP32 path to the
1e-4 relative force RMS bound stated for the single-precision form. Batched
evaluation must reproduce per-system evaluation bitwise, and repeated calls
must be bitwise identical.
"""
import numpy as np
import pytest

import oracle
from workloads import named, uniform_pm, uniform_pm_box, water_box

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    import paper_1309_1889_amd as m
    return m


def rel_rms(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))


def max_rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def run_gpu(w, precision, ke=138.935458, levels=None, max_systems=1, smoothing=2, basis=3):
    m = _lib()
    dt = np.float32 if precision == "fp32" else np.float64
    ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, levels=w.levels if levels is None else levels,
                       precision=precision, ke=ke, max_atoms=max(w.n, 1), max_systems=max_systems,
                       smoothing=smoothing, basis=basis)
    xyzq = torch.tensor(w.xyzq(dt), device="cuda")
    e, f, p = ctx.energy_forces(xyzq)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    return ctx, float(e[0].item()), f.double().cpu().numpy(), p.double().cpu().numpy()


def run_oracle(w, ke=138.935458, levels=None, stages=False, smoothing=0, basis=0):
    p = oracle.OracleParams(w.a, w.h, tuple(w.lo), tuple(w.hi), w.levels if levels is None else levels, ke,
                            smoothing=smoothing, basis=basis)
    return oracle.msm(p, w.xyz, w.q, stages=stages)


# ---------------------------------------------------------------------------
def test_fp64_matches_oracle_per_stage_charges_2000():
    w = named("charges_2000")
    ctx, e, f, p = run_gpu(w, "fp64")
    eo, fo, po, st = run_oracle(w, stages=True)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    g = ctx.stages(w.n)
    assert max_rel(g["u_short"].cpu().numpy(), st["u_short"]) < 1e-12
    assert max_rel(g["f_short"].cpu().numpy(), st["f_short"]) < 1e-12
    shapes = ctx.grid_shape()
    assert len(shapes) == len(st["q_grid"]) == 3
    for k in range(len(shapes)):
        assert tuple(g["q_grid"][k].shape) == st["q_grid"][k].shape
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-12, k
        assert max_rel(g["ucut_grid"][k].cpu().numpy(), st["ucut_grid"][k]) < 1e-12, k
        assert max_rel(g["u_grid"][k].cpu().numpy(), st["u_grid"][k]) < 1e-12, k


@pytest.mark.parametrize("h,two_pass", [(0.25, False), (0.5, True)])
def test_anterpolation_forms_match_oracle_per_stage(h, two_pass):
    """Anterpolation runs as LDS tiles up to 2 atoms per cell on average and
    as per-cell partial charges above; both against the oracle's scatter, on
    the grid charges q^k and the outputs."""
    w = water_box(1500, (12, 12, 12), (3.6, 3.6, 3.6), seed=23, a=0.8, h=h)
    ctx, e, f, p = run_gpu(w, "fp64")
    ncells = 1
    for d in range(3):
        nc = int(np.floor((w.hi[d] - w.lo[d]) / h)) + 1
        ncells *= (nc + 3) // 4 * 4
    assert (w.n > 2 * ncells) == two_pass
    eo, fo, po, st = run_oracle(w, stages=True)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    g = ctx.stages(w.n)
    for k in range(len(st["q_grid"])):
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-12, k


@pytest.mark.parametrize("box", ["water_2400", "water_99999"])
def test_fp32_grid_charges_match_oracle(box):
    """The single-precision anterpolation (one-axis weights staged with each
    atom) against the oracle's scatter on every level's grid charges, to
    single-precision rounding relative to the largest grid charge: a node
    adds about a hundred products of three weights and a charge of either
    sign, so rounding reaches a few 1e-6 of the largest value; a wrong weight
    or node would be off by 1e-2 or more."""
    w = (water_box(800, (10, 10, 10), (3.1, 3.1, 3.1), seed=29) if box == "water_2400"
         else named("water_99999")).as_dtype(np.float32)
    ctx, e, f, p = run_gpu(w, "fp32")
    eo, fo, po, st = run_oracle(w, stages=True)
    g = ctx.stages(w.n)
    for k in range(len(st["q_grid"])):
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-5, k
    assert rel_rms(f, fo) < 1e-5
    assert rel_rms(p, po) < 1e-5


# the composite transfers hold a level-0 xy plane of at most this many nodes in
# LDS; larger planes restrict and prolong one level at a time
PLANE_CAP = 6144


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_level_transfers_match_oracle_per_stage(precision):
    """A flat 22 x 22 x 1.5 nm domain: its level-0 xy plane (92 x 92 nodes)
    exceeds the composite transfers' LDS plane, so restriction and
    prolongation run one level at a time (the path of every large box). FP64:
    every q^k, u^{k,cutoff} and u^k of the six grids and the outputs against
    the oracle at rounding level; FP32: the outputs at the single-precision
    bound."""
    w = uniform_pm_box(2000, (22.0, 22.0, 1.5), seed=31)
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    ctx, e, f, p = run_gpu(w, precision)
    shapes = ctx.grid_shape()
    org, dim = shapes[0]
    assert dim[0] * dim[1] > PLANE_CAP and len(shapes) == 6
    if precision == "fp32":
        eo, fo, po = run_oracle(w)
        assert rel_rms(f, fo) < 1e-4
        assert rel_rms(p, po) < 1e-4
        assert e == pytest.approx(eo, rel=1e-4)
        return
    eo, fo, po, st = run_oracle(w, stages=True)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    g = ctx.stages(w.n)
    assert len(st["q_grid"]) == len(shapes)
    for k in range(len(shapes)):
        assert tuple(g["q_grid"][k].shape) == st["q_grid"][k].shape, k
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-12, k
        assert max_rel(g["ucut_grid"][k].cpu().numpy(), st["ucut_grid"][k]) < 1e-12, k
        assert max_rel(g["u_grid"][k].cpu().numpy(), st["u_grid"][k]) < 1e-12, k


def test_anterpolation_global_gather_matches_oracle():
    """A sparse 6 nm box with 2,500 of its 3,000 charges in one 1 nm cube: the
    tile whose 11 x 11 x 7-cell region holds the dense spot has more atoms than
    its LDS stages (2,048), so its nodes gather from global memory, while the
    box as a whole stays below 2 atoms per cell (the tiled form). q^k and the
    outputs against the oracle's scatter at rounding level."""
    w = uniform_pm_box(3000, (6.0, 6.0, 6.0), seed=32, cluster=(2500, (2.5, 2.5, 2.5), 1.0))
    ncells = 1
    for d in range(3):
        nc = int(np.floor((w.hi[d] - w.lo[d]) / w.h)) + 1
        ncells *= (nc + 3) // 4 * 4
    assert w.n <= 2 * ncells   # the tiled form, not the two-pass cell form
    ctx, e, f, p = run_gpu(w, "fp64")
    eo, fo, po, st = run_oracle(w, stages=True)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    g = ctx.stages(w.n)
    for k in range(len(st["q_grid"])):
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-12, k


@pytest.mark.parametrize("m", [1, 2, 3])
def test_smoothing_orders_match_oracle_per_stage(m):
    """gamma of order m (degree 2m) in the pair kernel, the stencil weights,
    the top level and the self term, against the oracle's own gamma_m."""
    w = water_box(700, (13, 13, 13), (4.1, 4.1, 4.1), seed=24)
    ctx, e, f, p = run_gpu(w, "fp64", smoothing=m)
    eo, fo, po, st = run_oracle(w, stages=True, smoothing=m)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    g = ctx.stages(w.n)
    assert max_rel(g["u_short"].cpu().numpy(), st["u_short"]) < 1e-12
    assert max_rel(g["f_short"].cpu().numpy(), st["f_short"]) < 1e-12
    for k in range(len(st["ucut_grid"])):
        assert max_rel(g["ucut_grid"][k].cpu().numpy(), st["ucut_grid"][k]) < 1e-12, k


@pytest.mark.parametrize("m", [1, 3])
def test_smoothing_orders_fp32(m):
    w = water_box(700, (13, 13, 13), (4.1, 4.1, 4.1), seed=25).as_dtype(np.float32)
    _, e, f, p = run_gpu(w, "fp32", smoothing=m)
    eo, fo, po = run_oracle(w, smoothing=m)
    assert rel_rms(f, fo) < 1e-4
    assert rel_rms(p, po) < 1e-4
    assert e == pytest.approx(eo, rel=1e-4)


@pytest.mark.parametrize("m,h", [(2, 0.25), (3, 0.25), (3, 0.5)])
def test_quintic_basis_matches_oracle_per_stage(m, h):
    """The degree-5 nodal basis in anterpolation (tiles at h = 0.25, cell
    partials at h = 0.5), restriction, prolongation and interpolation, on
    every grid and the outputs, against the oracle."""
    w = water_box(1500, (12, 12, 12), (3.6, 3.6, 3.6), seed=26, a=0.8, h=h)
    ctx, e, f, p = run_gpu(w, "fp64", smoothing=m, basis=5)
    eo, fo, po, st = run_oracle(w, stages=True, smoothing=m, basis=5)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11
    shapes = ctx.grid_shape()
    g = ctx.stages(w.n)
    assert len(shapes) == len(st["q_grid"])
    # the quintic restriction adds 7^3 terms per node (the cubic 5^3), in
    # separable passes on the GPU and as one 3-D sum in the oracle, over grids
    # of cancelling charges: rounding relative to the largest value reaches
    # ~1.5e-12 on the coarse levels, so the grids are held to 1e-11
    for k in range(len(shapes)):
        assert tuple(g["q_grid"][k].shape) == st["q_grid"][k].shape, k
        assert max_rel(g["q_grid"][k].cpu().numpy(), st["q_grid"][k]) < 1e-11, k
        assert max_rel(g["u_grid"][k].cpu().numpy(), st["u_grid"][k]) < 1e-11, k


def test_quintic_basis_fp32_and_batched():
    m = _lib()
    ws = [water_box(700, (13, 13, 13), (4.1, 4.1, 4.1), seed=27), water_box(300, (10, 10, 10), (3.1, 3.1, 3.1),
                                                                            seed=28)]
    w = ws[0].as_dtype(np.float32)
    _, e, f, p = run_gpu(w, "fp32", smoothing=3, basis=5)
    eo, fo, po = run_oracle(w, smoothing=3, basis=5)
    assert rel_rms(f, fo) < 1e-4
    assert rel_rms(p, po) < 1e-4
    # two systems in one call equal each alone, bitwise
    hi = np.maximum(ws[0].hi - ws[0].lo, ws[1].hi - ws[1].lo)
    big = m.MsmContext(0.9, 0.25, np.zeros(3), hi, precision="fp32", max_atoms=ws[0].n + ws[1].n, max_systems=2,
                       smoothing=3, basis=5)
    x = torch.tensor(np.concatenate([v.xyzq(np.float32) for v in ws]), device="cuda")
    offs = [0, ws[0].n, ws[0].n + ws[1].n]
    doms = np.array([np.concatenate([v.lo, v.hi]) for v in ws])
    eb, fb, pb = big.energy_forces(x, offs, doms)
    torch.cuda.synchronize()
    for k, v in enumerate(ws):
        one = m.MsmContext(0.9, 0.25, v.lo, v.hi, precision="fp32", max_atoms=v.n, smoothing=3, basis=5)
        e1, f1, p1 = one.energy_forces(torch.tensor(v.xyzq(np.float32), device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(eb[k:k + 1], e1)
        assert torch.equal(fb[offs[k]:offs[k + 1]], f1)


def test_smoothing_order_out_of_range_is_rejected():
    m = _lib()
    with pytest.raises(m.MsmError) as ei:
        m.MsmContext(1.2, 0.25, (0, 0, 0), (3, 3, 3), precision="fp64", max_atoms=10, smoothing=4)
    assert ei.value.code == -6
    with pytest.raises(m.MsmError) as ei:
        m.MsmContext(1.2, 0.25, (0, 0, 0), (3, 3, 3), precision="fp64", max_atoms=10, basis=4)
    assert ei.value.code == -6


def test_grid_shapes_agree_with_oracle():
    m = _lib()
    for w in [named("charges_2000"), water_box(500, (12, 12, 12), (3.7, 3.7, 3.7), seed=3)]:
        ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp64", max_atoms=w.n)
        p = oracle.OracleParams.of(w)
        shapes = ctx.grid_shape()
        assert len(shapes) == oracle.levels(p)
        for k, s in enumerate(shapes):
            assert s == oracle.grid_shape(p, k)


def test_fp32_matches_oracle_charges_2000():
    w = named("charges_2000").as_dtype(np.float32)
    _, e, f, p = run_gpu(w, "fp32")
    eo, fo, po = run_oracle(w)
    assert rel_rms(f, fo) < 1e-4
    assert rel_rms(p, po) < 1e-4
    assert e == pytest.approx(eo, rel=1e-4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_water_small_matches_oracle(precision):
    w = water_box(700, (13, 13, 13), (4.1, 4.1, 4.1), seed=21)
    if precision == "fp32":
        w = w.as_dtype(np.float32)
    _, e, f, p = run_gpu(w, precision)
    eo, fo, po = run_oracle(w)
    tol = 1e-11 if precision == "fp64" else 1e-4
    assert rel_rms(f, fo) < tol
    assert rel_rms(p, po) < tol
    assert e == pytest.approx(eo, rel=tol)


@pytest.mark.parametrize("pw", [2, 3, 5, 6, 7, 9, 10])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cluster_pair_forms_match_oracle(pw, precision):
    """Each cluster form of the short-range sum (8-atom clusters, one or two
    per wave, or sharing a workgroup's stream, or each pair once with
    Newton's third law; 16- and 32-atom clusters) against the oracle, on a
    water box whose last 64-atom group is partly empty (999 atoms) and on
    uniform charges with the coarse cells of h = 0.5. The Newton form is
    single precision only: a double precision context refuses it."""
    m = _lib()
    dt = np.float32 if precision == "fp32" else np.float64
    tol = 1e-11 if precision == "fp64" else 1e-4
    for w in (water_box(1001 // 3, (7, 7, 7), (3.3, 3.3, 3.3), seed=31),
              uniform_pm(777, 3.4, seed=32, a=0.8, h=0.5)):
        if precision == "fp32":
            w = w.as_dtype(np.float32)
        ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, levels=w.levels, precision=precision, max_atoms=w.n)
        if pw == 10 and precision == "fp64":
            with pytest.raises(m.MsmError):
                ctx.set_tuning(pair_waves=pw)
            continue
        ctx.set_tuning(pair_waves=pw)
        e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
        torch.cuda.synchronize()
        assert ctx.status() == 0
        eo, fo, po = run_oracle(w)
        assert rel_rms(f.double().cpu().numpy(), fo) < tol, w.n
        assert rel_rms(p.double().cpu().numpy(), po) < tol, w.n
        assert float(e[0].item()) == pytest.approx(eo, rel=tol)


@pytest.mark.parametrize("pc", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pair_cells_finer_than_h_match_oracle(pc, precision):
    """The pair search in cells of edge h/2 and h/3 (a second binning of the
    atoms, the sums permuted back) against the oracle, with the 8- and
    16-atom cluster forms, on a water box and on uniform charges at the
    coarse h = 0.5 with a = 0.8 (the coarse propagator's grid); the model
    exclusions and Lennard-Jones applied on top; and a batch of two systems
    equal to the systems alone, bitwise."""
    m = _lib()
    dt = np.float32 if precision == "fp32" else np.float64
    tol = 1e-11 if precision == "fp64" else 1e-4
    for w in (water_box(1001 // 3, (7, 7, 7), (3.3, 3.3, 3.3), seed=31),
              uniform_pm(777, 3.4, seed=32, a=0.8, h=0.5)):
        if precision == "fp32":
            w = w.as_dtype(np.float32)
        ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, levels=w.levels, precision=precision, max_atoms=w.n)
        eo, fo, po = run_oracle(w)
        for pw in (2, 5):
            ctx.set_tuning(pair_waves=pw, pair_cell=pc)
            assert ctx.tuning()["pair_cell"] == pc
            e, f, p = ctx.energy_forces(torch.tensor(w.xyzq(dt), device="cuda"))
            torch.cuda.synchronize()
            assert ctx.status() == 0
            assert rel_rms(f.double().cpu().numpy(), fo) < tol, (w.n, pw)
            assert rel_rms(p.double().cpu().numpy(), po) < tol, (w.n, pw)
            assert float(e[0].item()) == pytest.approx(eo, rel=tol)
    parts = [water_box(n, (p_,) * 3, (s_,) * 3, seed=40 + n) for n, p_, s_ in ((700, 9, 3.0), (433, 8, 2.6))]
    offs = [0, 3 * 700, 3 * 700 + 3 * 433]
    doms = [list(q.lo) + list(q.hi) for q in parts]
    big = m.MsmContext(1.2, 0.25, parts[0].lo, parts[0].hi, precision=precision, max_atoms=offs[-1], max_systems=2)
    big.set_tuning(pair_cell=pc)
    x = torch.tensor(np.concatenate([q.xyzq(dt) for q in parts]), device="cuda")
    eb, fb, pb = big.energy_forces(x, offs, doms)
    for s_, q in enumerate(parts):
        one = m.MsmContext(1.2, 0.25, q.lo, q.hi, precision=precision, max_atoms=q.n)
        one.set_tuning(pair_cell=pc)
        e1, f1, p1 = one.energy_forces(torch.tensor(q.xyzq(dt), device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(eb[s_:s_ + 1], e1) and torch.equal(fb[offs[s_]:offs[s_ + 1]], f1)
        assert torch.equal(pb[offs[s_]:offs[s_ + 1]], p1)
    with pytest.raises(m.MsmError):
        big.set_tuning(pair_cell=4)


@pytest.mark.parametrize("a,h,levels", [(0.8, 0.5, 0), (1.2, 0.25, 1), (1.2, 0.25, 2), (0.6, 0.2, 0),
                                        (1.0, 0.35, 0), (0.3, 0.25, 0), (1.3, 0.25, 0), (1.4, 0.25, 0)])
def test_fp64_parameter_variants(a, h, levels):
    w = uniform_pm(500, 3.3, seed=5, a=a, h=h, levels=levels)
    _, e, f, p = run_gpu(w, "fp64")
    eo, fo, po = run_oracle(w)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11


@pytest.mark.parametrize("a,h", [(0.3, 0.25), (0.8, 0.5), (1.4, 0.25)])
def test_fp32_parameter_variants(a, h):
    # stencil reach 2, 3 and 11: the smallest and largest shapes of the tiled stencil
    w = uniform_pm(600, 3.3, seed=6, a=a, h=h).as_dtype(np.float32)
    _, e, f, p = run_gpu(w, "fp32")
    eo, fo, po = run_oracle(w)
    assert rel_rms(f, fo) < 1e-4
    assert rel_rms(p, po) < 1e-4


def test_non_cubic_domain_and_boundary_atoms():
    rng = np.random.default_rng(12)
    lo, hi = np.array([-0.3, 0.1, 1.0]), np.array([2.9, 4.6, 2.7])
    xyz = rng.uniform(lo, hi, (400, 3))
    xyz[0] = lo                     # on the lower corner
    xyz[1] = hi                     # on the upper corner
    xyz[2] = [hi[0], lo[1], 1.75]   # on faces
    xyz[3] = lo + 0.25 * np.array([3, 5, 2])   # on a level-0 node
    q = rng.standard_normal(400)
    from workloads import Workload
    w = Workload("box", xyz, q, lo, hi, a=0.9, h=0.25)
    _, e, f, p = run_gpu(w, "fp64")
    eo, fo, po = run_oracle(w)
    assert e == pytest.approx(eo, rel=1e-12)
    assert max_rel(f, fo) < 1e-11
    assert max_rel(p, po) < 1e-11


@pytest.mark.parametrize("n_spread,h", [(300, 0.25), (1200, 0.6)])
def test_crowded_cell(n_spread, h):
    # 300 atoms inside one 0.2 nm cube (a single cell) plus more spread out:
    # the per-cell ordering takes its heapsort branch, in the one-thread-per-
    # cell form (few atoms per cell on average) and the one-wave-per-cell form
    rng = np.random.default_rng(17)
    xyz = np.concatenate([rng.uniform(1.02, 1.22, (300, 3)), rng.uniform(0.0, 3.0, (n_spread, 3))])
    q = rng.standard_normal(300 + n_spread) * 0.1
    from workloads import Workload
    w = Workload("crowded", xyz, q, np.zeros(3), np.full(3, 3.0), a=0.8, h=h)
    nb = (int(np.floor(3.0 / h)) + 1 + 3) // 4 * 4
    assert (w.n > 2 * nb ** 3) == (h > 0.5)
    _, e, f, p = run_gpu(w, "fp64")
    eo, fo, po = run_oracle(w)
    assert e == pytest.approx(eo, rel=1e-11)
    assert max_rel(f, fo) < 1e-10
    assert max_rel(p, po) < 1e-10


def test_single_atom_and_pair():
    from workloads import Workload
    for xyz, q in [(np.array([[1.1, 0.7, 1.9]]), np.array([1.5])),
                   (np.array([[1.1, 0.7, 1.9], [1.3, 0.9, 1.2]]), np.array([1.0, -2.0]))]:
        w = Workload("tiny", xyz, q, np.zeros(3), np.full(3, 2.5), a=0.8, h=0.25)
        _, e, f, p = run_gpu(w, "fp64")
        eo, fo, po = run_oracle(w)
        assert e == pytest.approx(eo, rel=1e-12, abs=1e-12)
        np.testing.assert_allclose(f, fo, rtol=1e-11, atol=1e-11 * max(1.0, np.abs(fo).max()))


@pytest.mark.parametrize("precision,pw", [("fp64", 2), ("fp32", 2), ("fp32", 10)])
def test_batched_equals_separate_bitwise(precision, pw):
    """A batch of systems (one of them empty) gives each system the bits it
    gets alone, with the default pair form and with the Newton form, whose
    fixed-point sums do not depend on the order of their terms."""
    m = _lib()
    dt = np.float32 if precision == "fp32" else np.float64
    systems = [water_box(300, (10, 10, 10), (3.0, 3.0, 3.0), seed=31),
               uniform_pm(0, 2.0, seed=1),
               water_box(900, (14, 14, 14), (4.4, 4.4, 4.4), seed=32),
               uniform_pm(777, 3.5, seed=33)]
    big = np.max([s.hi - s.lo for s in systems], axis=0)
    lo0 = np.zeros(3)
    ntot = sum(s.n for s in systems)
    ctx = m.MsmContext(1.2, 0.25, lo0, lo0 + big, precision=precision, max_atoms=ntot, max_systems=4)
    ctx.set_tuning(pair_waves=pw)
    offs = np.cumsum([0] + [s.n for s in systems])
    doms = np.array([np.concatenate([s.lo, s.hi]) for s in systems])
    xyzq = torch.tensor(np.concatenate([s.xyzq(dt) for s in systems]), device="cuda")
    e, f, p = ctx.energy_forces(xyzq, offs, doms)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for s, sysw in enumerate(systems):
        if sysw.n == 0:
            assert e[s].item() == 0.0
            continue
        one = m.MsmContext(1.2, 0.25, sysw.lo, sysw.hi, precision=precision, max_atoms=sysw.n)
        one.set_tuning(pair_waves=pw)
        x1 = torch.tensor(sysw.xyzq(dt), device="cuda")
        e1, f1, p1 = one.energy_forces(x1)
        torch.cuda.synchronize()
        assert torch.equal(e[s:s + 1], e1)
        assert torch.equal(f[offs[s]:offs[s + 1]], f1)
        assert torch.equal(p[offs[s]:offs[s + 1]], p1)
        if precision == "fp64":
            eo, fo, _ = run_oracle(sysw)
            assert e1.item() == pytest.approx(eo, rel=1e-12)


def test_deep_anterpolation_tiles_same_bits():
    """Single precision batches whose level-0 grids hold enough tiles use
    anterpolation tiles 8 node layers deep instead of 4 (fewer staged halo
    atoms per node); each node's sum is kept per cell layer and added in layer
    order, so both depths give the same bits. Eight water boxes in 12 nm
    domains (343 deep tiles each, 2,744 together) go through one batched call
    (deep tiles) and one call each (a single grid of 343 deep tiles keeps the
    shallow ones); the outputs must agree bitwise, and one system matches the
    oracle."""
    m = _lib()
    parts = [water_box(200 + 40 * i, (10, 10, 10), (3.0, 3.0, 3.0), seed=70 + i, margin=4.5).as_dtype(np.float32)
             for i in range(8)]
    big = np.max([q.hi - q.lo for q in parts], axis=0)
    offs = np.cumsum([0] + [q.n for q in parts])
    doms = np.array([np.concatenate([q.lo, q.hi]) for q in parts])
    ctx = m.MsmContext(1.2, 0.25, np.zeros(3), big, precision="fp32", max_atoms=int(offs[-1]), max_systems=8)
    x = torch.tensor(np.concatenate([q.xyzq(np.float32) for q in parts]), device="cuda")
    eb, fb, pb = [t.clone() for t in ctx.energy_forces(x, offs, doms)]
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for s_, q in enumerate(parts):
        one = m.MsmContext(1.2, 0.25, q.lo, q.hi, precision="fp32", max_atoms=q.n)
        e1, f1, p1 = one.energy_forces(torch.tensor(q.xyzq(np.float32), device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(eb[s_:s_ + 1], e1), s_
        assert torch.equal(fb[offs[s_]:offs[s_ + 1]], f1), s_
        assert torch.equal(pb[offs[s_]:offs[s_ + 1]], p1), s_
        if s_ == 0:
            eo, fo, po = run_oracle(q)
            assert rel_rms(f1.double().cpu().numpy(), fo) < 1e-4
            assert rel_rms(p1.double().cpu().numpy(), po) < 1e-4
            assert float(e1.item()) == pytest.approx(eo, rel=1e-5)


def test_repeat_is_bitwise_deterministic():
    m = _lib()
    w = water_box(2000, (19, 19, 19), (5.8, 5.8, 5.8), seed=41)
    ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=w.n)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    r1 = [t.clone() for t in ctx.energy_forces(x)]
    r2 = ctx.energy_forces(x)
    torch.cuda.synchronize()
    for a_, b_ in zip(r1, r2):
        assert torch.equal(a_, b_)
    # a permutation of the input only permutes the outputs (within rounding)
    perm = torch.randperm(w.n, generator=torch.Generator().manual_seed(0)).cuda()
    e3, f3, p3 = ctx.energy_forces(x[perm].contiguous())
    torch.cuda.synchronize()
    assert e3.item() == pytest.approx(r1[0].item(), rel=1e-6)
    assert rel_rms(f3.cpu().numpy(), r1[1][perm].cpu().numpy()) < 1e-6


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_forces_only_evaluation_gives_the_same_forces(precision):
    """An evaluation asked for forces alone skips the short-range potential
    sums; its forces are those of the full evaluation, bit for bit, also with
    a molecular model bound."""
    m = _lib()
    w = water_box(2000, (19, 19, 19), (5.8, 5.8, 5.8), seed=43)
    dt = np.float32 if precision == "fp32" else np.float64
    x = torch.tensor(w.xyzq(dt), device="cuda")
    cases = [(False, None), (True, None)]
    if precision == "fp32":
        cases += [(False, 10), (True, 10)]   # and each pair once (Newton's third law)
    for model, pw in cases:
        ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, precision=precision, max_atoms=w.n)
        if pw is not None:
            ctx.set_tuning(pair_waves=pw)
        if model:
            from workloads import water_model_arrays
            mass, molid, lj, tri = water_model_arrays(w.n)
            ctx.bind_model(w.n, torch.tensor(molid, dtype=torch.int32, device="cuda"),
                           torch.tensor(lj, device="cuda"), rigid=True, tri=tri)
        _, f_full, _ = ctx.energy_forces(x)
        _, f_only, _ = ctx.energy_forces(x, want=("forces",))
        torch.cuda.synchronize()
        assert ctx.status() == 0
        assert torch.equal(f_full, f_only), (model, pw)


def test_status_reports_domain_and_nonfinite():
    m = _lib()
    w = uniform_pm(100, 2.0, seed=2)
    ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=200)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    x[5, 1] = 2.6
    ctx.energy_forces(x)
    assert ctx.status() == -2
    x[5, 1] = float("nan")
    ctx.energy_forces(x)
    assert ctx.status() == -3
    assert ctx.status() == 0          # cleared after reading
    x2 = torch.zeros((300, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(m.MsmError) as ei:
        ctx.energy_forces(x2)
    assert ei.value.code == -4


def test_water_99999_fp32_matches_oracle():
    """The benchmark workload at full size: every atom against the oracle."""
    w = named("water_99999").as_dtype(np.float32)
    _, e, f, p = run_gpu(w, "fp32")
    eo, fo, po = run_oracle(w)
    assert rel_rms(f, fo) < 1e-4
    assert rel_rms(p, po) < 1e-4
    assert e == pytest.approx(eo, rel=1e-5)


def test_newton_form_water_99999_matches_oracle():
    """The pair form that evaluates each pair once (Newton's third law, its
    candidate's share in fixed point) on the benchmark workload: every atom
    against the oracle, within single precision rounding of the form that
    evaluates each pair from both sides, and the same bits when repeated."""
    m = _lib()
    w = named("water_99999").as_dtype(np.float32)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    ctx = m.MsmContext(w.a, w.h, w.lo, w.hi, levels=w.levels, precision="fp32", max_atoms=w.n)
    e2, f2, p2 = [t.clone() for t in ctx.energy_forces(x)]
    ctx.set_tuning(pair_waves=10)
    e, f, p = [t.clone() for t in ctx.energy_forces(x)]
    er, fr, pr = ctx.energy_forces(x)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    assert torch.equal(e, er) and torch.equal(f, fr) and torch.equal(p, pr)
    assert rel_rms(f.double().cpu().numpy(), f2.double().cpu().numpy()) < 1e-6
    assert rel_rms(p.double().cpu().numpy(), p2.double().cpu().numpy()) < 1e-6
    eo, fo, po = run_oracle(w)
    assert rel_rms(f.double().cpu().numpy(), fo) < 1e-4
    assert rel_rms(p.double().cpu().numpy(), po) < 1e-4
    assert float(e[0].item()) == pytest.approx(eo, rel=1e-5)


def test_water_99999_fp64_matches_oracle():
    w = named("water_99999")
    _, e, f, p = run_gpu(w, "fp64")
    eo, fo, po = run_oracle(w)
    assert rel_rms(f, fo) < 1e-10
    assert e == pytest.approx(eo, rel=1e-11)
