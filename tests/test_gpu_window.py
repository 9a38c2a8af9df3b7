"""Parareal with a sliding computational window (Section 4) on the GPU:
exact states only (tolerance 0) give the serial fine trajectory bitwise, a
window as wide as the run repeats parareal_run's iterates, the pipelined
schedule (fine batches overlapping the coarse sweep on another stream) gives
the same bits as the plain one, a checkpoint resumes bitwise, and FP64 runs
follow the oracle's window state by state."""
import math

import numpy as np
import pytest

import oracle
from workloads import rigid_water_velocities, water_box, water_model_arrays

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KE = 138.935458
SF, DTF, SG, DTG = 3, 0.001, 1, 0.003


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def msmx():
    import paper_1309_1889_amd as m
    return m


class Case:
    """125 rigid waters; fine MSM a 0.9 h 0.25 (3 x 1 fs), coarse MSM a 0.7 h 0.5 (1 x 3 fs)."""

    def __init__(self, precision, width, fine_stream=None):
        m = msmx()
        per = int(math.ceil(125 ** (1 / 3)))
        self.w = water_box(125, (per,) * 3, (1.55,) * 3, seed=21, margin=0.6)
        self.mass, self.molid, self.lj, self.tri = water_model_arrays(self.w.n)
        self.v = rigid_water_velocities(self.w.xyz, 300.0, seed=22)
        n = self.w.n
        self.fine = self._ctx(0.9, 0.25, precision, width * n, width, fine_stream)
        self.coarse = self._ctx(0.7, 0.5, precision, n, 1)
        self.q = torch.tensor(self.w.q, dtype=torch.float64, device="cuda")
        self.invm = torch.tensor(1.0 / self.mass, dtype=torch.float64, device="cuda")
        self.s0 = torch.tensor(np.concatenate([self.w.xyz, self.v], 1), dtype=torch.float64,
                               device="cuda").contiguous()
        self.precision, self.width, self.m = precision, width, m

    def _ctx(self, a, h, precision, max_atoms, max_systems, stream=None):
        ctx = msmx().MsmContext(a, h, self.w.lo, self.w.hi, precision=precision, ke=KE, max_atoms=max_atoms,
                                max_systems=max_systems)
        ctx.bind_model(len(self.mass), torch.tensor(self.molid, dtype=torch.int32, device="cuda"),
                       torch.tensor(self.lj, dtype=torch.float64, device="cuda"), rigid=True, tri=self.tri)
        if stream is not None:
            ctx.set_stream(stream)
        return ctx

    def buffers(self, T):
        lam = torch.zeros((T + 1, self.w.n, 6), dtype=torch.float64, device="cuda")
        lam[0] = self.s0
        ring = torch.zeros((self.width, self.w.n, 6), dtype=torch.float64, device="cuda")
        return lam, ring, self.m.WindowState()

    def run(self, lam, ring, st, tol, **kw):
        rc = self.m.parareal_window(self.fine, self.coarse, self.q, self.invm, lam, ring, st, width=self.width,
                                    tol=tol, steps_f=SF, dt_f=DTF, steps_g=SG, dt_g=DTG, **kw)
        torch.cuda.synchronize()
        return rc

    def serial_fine(self, T):
        ref = self._ctx(0.9, 0.25, self.precision, self.w.n, 1)
        out = [self.s0.clone()]
        for _ in range(T):
            cur = out[-1]
            x = torch.cat([cur[:, :3], self.q[:, None]], 1).contiguous()
            v = torch.cat([cur[:, 3:], self.invm[:, None]], 1).contiguous()
            ref.vv_run(x, v, SF, DTF, energies=False)
            out.append(torch.cat([x[:, :3], v[:, :3]], 1))
        torch.cuda.synchronize()
        return torch.stack(out)


@pytest.mark.parametrize("precision,pipeline", [("fp64", False), ("fp32", False), ("fp32", True)])
def test_window_with_zero_tolerance_is_the_serial_fine_trajectory(precision, pipeline):
    T, W = 7, 3
    c = Case(precision, W, torch.cuda.Stream() if pipeline else None)
    print(f"window tol 0: {precision} pipeline={pipeline} T={T} W={W} n={c.w.n}", flush=True)
    lam, ring, st = c.buffers(T)
    rc = c.run(lam, ring, st, 0.0, pipeline=pipeline, chunk=1)
    assert rc == 0 and st.start == T and st.iterations == T
    assert torch.equal(lam, c.serial_fine(T))
    assert st.coarse_slices == W + sum(min(W, T - b) for b in range(T)) + (T - W)
    if not pipeline:
        assert st.fine_slices == sum(min(W, T - b) for b in range(T))


def test_full_window_iterates_are_parareal_runs():
    T = 5
    c = Case("fp32", T)
    for K in (1, 2, 4):
        print(f"full window vs parareal_run: K={K}", flush=True)
        ref, rep, _ = c.m.parareal(c.fine, c.coarse, c.q, c.invm, c.s0, nslices=T, kmax=K, tol=0.0, steps_f=SF,
                                   dt_f=DTF, steps_g=SG, dt_g=DTG)
        torch.cuda.synchronize()
        lam, ring, st = c.buffers(T)
        c.run(lam, ring, st, 0.0, max_iters=K)
        assert st.iterations == K and st.start == K
        assert torch.equal(lam, ref), K


def _oracle_window(c, T, tol, stops):
    pf = oracle.OracleParams(0.9, 0.25, tuple(c.w.lo), tuple(c.w.hi), 0, KE)
    pg = oracle.OracleParams(0.7, 0.5, tuple(c.w.lo), tuple(c.w.hi), 0, KE)
    model = oracle.OracleModel(c.mass, c.molid, c.lj, True, c.tri, 1e-12)
    lam, ring = oracle.window_buffers(c.w.xyz, c.v, T, c.width)
    st = oracle.WindowState()
    starts = []
    while True:
        rc = oracle.parareal_window(pf, pg, model, lam, ring, c.w.q, st, c.width, SF, DTF, SG, DTG, tol,
                                    max_iters=1)
        starts.append(st.start)
        if rc == 0 or len(starts) >= stops:
            return lam, starts


def test_window_fp64_follows_the_oracle_state_by_state():
    T, W, tol = 8, 4, 3e-4
    c = Case("fp64", W)
    print(f"window fp64 vs oracle: T={T} W={W} tol={tol}", flush=True)
    ref, starts = _oracle_window(c, T, tol, 2 * T)
    # the acceptance decisions do not sit on the tolerance: 1 % either way takes the same ones
    assert _oracle_window(c, T, 0.99 * tol, 2 * T)[1] == starts
    assert _oracle_window(c, T, 1.01 * tol, 2 * T)[1] == starts
    assert len(starts) < T   # some iteration accepted more than the exact state
    lam, ring, st = c.buffers(T)
    got = []
    while True:
        rc = c.run(lam, ring, st, tol, max_iters=1)
        got.append(st.start)
        if rc == 0:
            break
    assert got == starts
    g = lam.cpu().numpy()
    assert np.abs(g[..., :3] - ref[..., :3]).max() < 1e-9
    assert np.abs(g[..., 3:] - ref[..., 3:]).max() < 1e-6


def test_pipelined_run_equals_the_plain_one_bitwise():
    T, W, tol = 10, 4, 3e-4
    plain = Case("fp32", W)
    lam_p, ring_p, st_p = plain.buffers(T)
    print("window plain vs pipelined", flush=True)
    assert plain.run(lam_p, ring_p, st_p, tol) == 0
    for chunk in (1, 2, 0):
        pipe = Case("fp32", W, torch.cuda.Stream())
        lam, ring, st = pipe.buffers(T)
        assert pipe.run(lam, ring, st, tol, pipeline=True, chunk=chunk) == 0
        assert torch.equal(lam, lam_p), chunk
        assert torch.equal(ring, ring_p), chunk
        assert (st.iterations, st.coarse_slices) == (st_p.iterations, st_p.coarse_slices)
        assert st.fine_slices >= st_p.fine_slices


@pytest.mark.parametrize("pipeline", [False, True])
def test_resume_from_a_checkpoint_is_bitwise_the_uninterrupted_run(pipeline):
    T, W, tol = 10, 4, 3e-4
    c = Case("fp32", W, torch.cuda.Stream() if pipeline else None)
    lam_u, ring_u, st_u = c.buffers(T)
    assert c.run(lam_u, ring_u, st_u, tol, pipeline=pipeline) == 0
    for stop in (1, 3):
        print(f"window resume: pipeline={pipeline} stop={stop}", flush=True)
        lam, ring, st = c.buffers(T)
        assert c.run(lam, ring, st, tol, pipeline=pipeline, max_iters=stop) == 1
        # checkpoint to host memory, then resume from fresh device buffers
        saved = (lam.cpu().numpy().copy(), ring.cpu().numpy().copy(), st.copy())
        del lam, ring
        lam2 = torch.tensor(saved[0], device="cuda")
        ring2 = torch.tensor(saved[1], device="cuda")
        st2 = saved[2]
        assert c.run(lam2, ring2, st2, tol, pipeline=pipeline) == 0
        assert torch.equal(lam2, lam_u)
        assert (st2.iterations, st2.coarse_slices) == (st_u.iterations, st_u.coarse_slices)


def test_restart_from_the_window_edge_with_zero_tolerance_is_serial_fine():
    T, W = 6, 3
    c = Case("fp32", W)
    lam, ring, st = c.buffers(T)
    assert c.run(lam, ring, st, 0.0, max_iters=2) == 1
    b = st.start
    lam2, ring2, st2 = c.buffers(T)
    lam2[:b + 1] = lam[:b + 1]
    st2.start = b     # window_valid 0: predicted again from lambda_b
    assert c.run(lam2, ring2, st2, 0.0) == 0
    assert torch.equal(lam2, c.serial_fine(T))


def test_window_reports_domain_exit():
    T, W = 3, 2
    c = Case("fp64", W)
    lam, ring, st = c.buffers(T)
    lam[0, :, 3:] += 500.0    # every atom leaves the domain within the first slice
    with pytest.raises(c.m.MsmError) as ei:
        c.run(lam, ring, st, 0.0, max_iters=1)
    assert ei.value.code == -2


def test_window_argument_checks():
    c = Case("fp32", 2)
    lam, ring, st = c.buffers(4)
    with pytest.raises(ValueError):
        c.m.parareal_window(c.fine, c.coarse, c.q, c.invm, lam, ring[:1].contiguous(), st, width=2, tol=0.0,
                            steps_f=1, dt_f=0.001, steps_g=1, dt_g=0.001)
    # the fine context holds 2 systems: a window of 3 does not fit
    ring3 = torch.zeros((3, c.w.n, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(c.m.MsmError) as ei:
        c.m.parareal_window(c.fine, c.coarse, c.q, c.invm, lam, ring3, st, width=3, tol=0.0, steps_f=1,
                            dt_f=0.001, steps_g=1, dt_g=0.001)
    assert ei.value.code == -4
