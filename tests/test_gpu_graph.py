"""Captured HIP graphs: replays must reproduce eager evaluation bitwise,
with the inputs changed in place between replays, interleaved with eager
work and synchronisations, and after the batch shape changes."""
import math

import numpy as np
import pytest

from workloads import rigid_water_velocities, water_box, water_model_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_graph_replays_match_eager_bitwise():
    import paper_1309_1889_amd as msmx
    w = water_box(2000, (19, 19, 19), (5.8, 5.8, 5.8), seed=41)
    eager = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=2 * w.n, max_systems=2)
    graph = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=2 * w.n, max_systems=2)
    graph.set_graphs(True)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    rng = np.random.default_rng(3)
    outs = [torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty((w.n, 3), device="cuda"),
            torch.empty(w.n, device="cuda")]
    for rep in range(6):
        # change the input in place: same pointers, new data
        x[:, :3] += torch.tensor(rng.uniform(-0.003, 0.003, (w.n, 3)), dtype=torch.float32, device="cuda")
        graph.energy_forces(x, energy=outs[0], forces=outs[1], potentials=outs[2])
        e0, f0, p0 = eager.energy_forces(x)
        torch.cuda.synchronize()
        assert graph.status() == 0
        assert torch.equal(outs[0], e0) and torch.equal(outs[1], f0) and torch.equal(outs[2], p0), rep
    # a new batch shape is captured again
    x2 = torch.cat([x, x]).contiguous()
    offs = [0, w.n, 2 * w.n]
    for rep in range(3):
        eg, fg, pg = graph.energy_forces(x2, offs)
        ee, fe, pe = eager.energy_forces(x2, offs)
        torch.cuda.synchronize()
        assert torch.equal(eg, ee) and torch.equal(fg, fe) and torch.equal(pg, pe)


def test_graph_velocity_verlet_matches_eager():
    import paper_1309_1889_amd as msmx
    n_mol = 125
    per = int(math.ceil(n_mol ** (1 / 3)))
    w = water_box(n_mol, (per,) * 3, (1.6,) * 3, seed=5, margin=0.6)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=6)
    ctxs = []
    for graphs in (False, True):
        c = msmx.MsmContext(0.9, 0.25, w.lo, w.hi, precision="fp64", max_atoms=w.n)
        c.bind_model(w.n, torch.tensor(molid, dtype=torch.int32, device="cuda"),
                     torch.tensor(lj, device="cuda"), rigid=True, tri=tri)
        c.set_graphs(graphs)
        ctxs.append(c)
    states = []
    for c in ctxs:
        x = torch.tensor(np.concatenate([w.xyz, w.q[:, None]], 1), device="cuda").contiguous()
        vv = torch.tensor(np.concatenate([v, 1.0 / mass[:, None]], 1), device="cuda").contiguous()
        ep, ek = c.vv_run(x, vv, 8, 0.002)
        ep2, ek2 = c.vv_run(x, vv, 8, 0.002)
        torch.cuda.synchronize()
        states.append((x, vv, ep2, ek2))
    for a, b in zip(states[0], states[1]):
        assert torch.equal(a, b)


def test_autotune_and_tunings_agree():
    import paper_1309_1889_amd as msmx
    w = water_box(3000, (21, 21, 21), (6.6, 6.6, 6.6), seed=8)
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=w.n)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    ref = [t.clone() for t in ctx.energy_forces(x)]
    chosen = ctx.autotune(x, reps=3)
    assert chosen["pair_waves"] in (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 16) and chosen["stencil_threads"] in (256, 1024)
    assert chosen["pair_cell"] in (1, 2, 3)
    assert ctx.tuning() == chosen
    for pw in (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 16):
        for st in (256, 1024):
            ctx.set_tuning(pw, st, pair_cell=1 if pw != 2 else 2)
            e, f, p = ctx.energy_forces(x)
            e2, f2, p2 = ctx.energy_forces(x)
            torch.cuda.synchronize()
            assert torch.equal(f, f2) and torch.equal(e, e2)       # each configuration is deterministic
            rel = float(((f - ref[1]) ** 2).sum().sqrt() / (ref[1] ** 2).sum().sqrt())
            assert rel < 1e-5, (pw, st, rel)
            assert e.item() == pytest.approx(ref[0].item(), rel=1e-6)
    with pytest.raises(msmx.MsmError):
        ctx.set_tuning(11, 256)
    with pytest.raises(msmx.MsmError):
        ctx.set_tuning(pair_cell=0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_concurrent_stages_change_no_bit(precision):
    """The short-range sum on the context's second stream, beside the grid
    stages, gives the same bits as every stage in turn, eagerly and in graph
    replays (each replay checked, with eager work between replays), for
    every pair kernel form."""
    import paper_1309_1889_amd as msmx
    w = water_box(3000, (21, 21, 21), (6.6, 6.6, 6.6), seed=12)
    dt = np.float32 if precision == "fp32" else np.float64
    x = torch.tensor(w.xyzq(dt), device="cuda")
    seq = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision=precision, max_atoms=w.n)
    conc = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision=precision, max_atoms=w.n)
    seq.set_tuning(concurrent=0)
    assert conc.tuning()["concurrent"] == 1
    forms = ((1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (7, 1), (8, 1), (9, 1), (2, 2), (5, 2))
    if precision == "fp32":
        forms += ((10, 1), (10, 2))
    for pw, pc in forms:
        seq.set_tuning(pair_waves=pw, pair_cell=pc)
        conc.set_tuning(pair_waves=pw, pair_cell=pc)
        ref = seq.energy_forces(x)
        for graphs in (False, True):
            conc.set_graphs(graphs)
            for rep in range(3):
                got = conc.energy_forces(x)
                again = seq.energy_forces(x)       # eager work between replays
                torch.cuda.synchronize()
                for a, b, c in zip(got, ref, again):
                    assert torch.equal(a, b) and torch.equal(b, c), (pw, pc, graphs, rep)
        conc.set_graphs(False)
    assert seq.status() == 0 and conc.status() == 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_two_clusters_per_wave_same_bits(precision):
    """Two clusters sharing one candidate stream in a wave, and the clusters
    of a group or half group sharing one stream in a workgroup, keep, for
    each cluster, the candidates of its own box in the same order, so the
    sums are the one-cluster form's bit for bit; systems whose last group is
    partly empty included."""
    import paper_1309_1889_amd as msmx
    dt = np.float32 if precision == "fp32" else np.float64
    parts = [water_box(n, (p,) * 3, (s,) * 3, seed=20 + n) for n, p, s in ((1000, 10, 3.2), (733, 10, 3.0))]
    w = parts[0]
    x = torch.tensor(np.concatenate([p.xyzq(dt) for p in parts]), device="cuda")
    offs = [0, parts[0].n, parts[0].n + parts[1].n]
    doms = [list(p.lo) + list(p.hi) for p in parts]
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision=precision, max_atoms=offs[-1], max_systems=2)
    got = {}
    for pw in (2, 3, 7, 9):
        ctx.set_tuning(pair_waves=pw)
        got[pw] = [t.clone() for t in ctx.energy_forces(x, offs, doms)]
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for pw in (3, 7, 9):
        for a, b in zip(got[2], got[pw]):
            assert torch.equal(a, b), pw


def test_shared_stream_forms_same_bits_large():
    """The workgroup-shared candidate streams at 99,999 atoms, where a batch
    of pieces spans more stream positions than the position table holds (so
    the search path of the table runs) and the stream takes several batches
    and rounds: the sums are the one-cluster form's bit for bit."""
    import paper_1309_1889_amd as msmx
    from workloads import named
    w = named("water_99999").as_dtype(np.float32)
    x = torch.tensor(w.xyzq(np.float32), device="cuda")
    ctx = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=w.n)
    got = {}
    for pw in (2, 7, 9):
        ctx.set_tuning(pair_waves=pw)
        got[pw] = [t.clone() for t in ctx.energy_forces(x)]
    torch.cuda.synchronize()
    assert ctx.status() == 0
    for pw in (7, 9):
        for a, b in zip(got[2], got[pw]):
            assert torch.equal(a, b), pw
