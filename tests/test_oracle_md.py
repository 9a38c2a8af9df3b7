"""Pins of the dynamics oracle: velocity Verlet (Section 2) with rigid water,
and the parareal iteration (Section 4).

Pinned against facts that do not come from the oracle: closed-form
Lennard-Jones, exclusions equal to removing Coulomb's law for the excluded
pairs (checked against brute force), constraint lengths, second-order energy
drift of velocity Verlet, and the parareal properties that hold for any
propagators (k iterations reproduce the fine trajectory on the first k
slices; zero iterations give the coarse trajectory).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import rigid_water_velocities, water_box, water_model_arrays

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def small_water(n_mol=64, side=1.24, seed=7, margin=0.6):
    per = int(math.ceil(n_mol ** (1 / 3)))
    w = water_box(n_mol, (per,) * 3, (side,) * 3, seed=seed, margin=margin)
    mass, molid, lj, tri = water_model_arrays(w.n)
    model = oracle.OracleModel(mass, molid, lj, True, tri, 1e-12)
    v = rigid_water_velocities(w.xyz, 300.0, seed=seed + 1)
    return w, model, v


def test_lennard_jones_closed_form():
    lo, hi = (0.0, 0.0, 0.0), (2.0, 2.0, 2.0)
    p = oracle.OracleParams(1.0, 0.25, lo, hi, 0, 138.935458)
    sig, eps, r = 0.3, 0.5, 0.37
    xyz = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]])
    m = oracle.OracleModel(np.ones(2), np.array([0, 1], np.int32), np.array([[sig, eps], [sig, eps]]))
    e, f = oracle.md_forces(p, m, xyz, np.zeros(2))
    u = lambda x: 4 * eps * ((sig / x) ** 12 - (sig / x) ** 6)  # noqa: E731
    assert e == pytest.approx(u(r) - u(1.0), rel=1e-13)
    fx = (u(r + 1e-6) - u(r - 1e-6)) / 2e-6
    assert f[1, 0] == pytest.approx(-fx, rel=1e-7)
    assert f[0, 0] == pytest.approx(fx, rel=1e-7)
    # same molecule: excluded; beyond the cutoff: nothing
    m2 = oracle.OracleModel(np.ones(2), np.array([3, 3], np.int32), np.array([[sig, eps], [sig, eps]]))
    assert oracle.md_forces(p, m2, xyz, np.zeros(2))[0] == 0.0
    far = np.array([[0.2, 0.2, 0.2], [1.4, 0.2, 0.2]])
    assert oracle.md_forces(p, m, far, np.zeros(2))[0] == 0.0


def test_exclusions_remove_coulomb_of_intramolecular_pairs():
    w = water_box(300, (10, 10, 10), (3.0, 3.0, 3.0), seed=5)
    mass, molid, _, _ = water_model_arrays(w.n)
    p = oracle.OracleParams.of(w)
    m = oracle.OracleModel(mass, molid)
    e, f = oracle.md_forces(p, m, w.xyz, w.q)
    e0, f0, _ = oracle.coulomb(w.xyz, w.q)
    # brute force without the intramolecular pairs
    x = w.xyz.reshape(-1, 3, 3)
    qm = w.q.reshape(-1, 3)
    fx = np.zeros_like(x)
    e_in = 0.0
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        d = x[:, a] - x[:, b]
        r = np.linalg.norm(d, axis=1)
        u = 138.935458 * qm[:, a] * qm[:, b] / r
        e_in += u.sum()
        fx[:, a] += (u / r ** 2)[:, None] * d
        fx[:, b] -= (u / r ** 2)[:, None] * d
    e_ref = e0 - e_in
    f_ref = f0 - fx.reshape(-1, 3)
    assert abs(e - e_ref) / abs(e_ref) < 0.01
    assert np.sqrt(((f - f_ref) ** 2).sum() / (f_ref ** 2).sum()) < 0.01


def test_rattle_keeps_bonds_and_vv_drift_is_second_order():
    w, model, v = small_water()
    p = oracle.OracleParams(0.8, 0.25, tuple(w.lo), tuple(w.hi), 0, 138.935458)
    drift = []
    for dt, ns in [(0.002, 20), (0.001, 40)]:
        _, _, ep0, ek0 = oracle.vv(p, model, w.xyz, v, w.q, dt, 0)
        x, vv, ep, ek = oracle.vv(p, model, w.xyz, v, w.q, dt, ns)
        d = x.reshape(-1, 3, 3)
        for (a, b), L in zip([(0, 1), (0, 2), (1, 2)], model.tri):
            assert np.abs(np.linalg.norm(d[:, a] - d[:, b], axis=1) - L).max() < 1e-10
        # velocities along every bond vanish
        vm = vv.reshape(-1, 3, 3)
        for a, b in [(0, 1), (0, 2), (1, 2)]:
            assert np.abs(((vm[:, a] - vm[:, b]) * (d[:, a] - d[:, b])).sum(1)).max() < 1e-8
        drift.append(abs((ep + ek) - (ep0 + ek0)))
    # velocity Verlet: halving dt over the same time cuts the drift about 4x
    assert 2.5 < drift[0] / drift[1] < 6.0


def test_parareal_exact_after_k_iterations_and_coarse_at_zero():
    w, model, v = small_water(n_mol=27, side=0.93, seed=3)
    pf = oracle.OracleParams(0.8, 0.25, tuple(w.lo), tuple(w.hi), 0, 138.935458)
    pg = oracle.OracleParams(0.6, 0.5, tuple(w.lo), tuple(w.hi), 0, 138.935458)
    S, sf, dtf, sg, dtg = 4, 3, 0.001, 1, 0.003
    # serial fine and serial coarse trajectories
    fine = [np.concatenate([w.xyz, v], 1)]
    coarse = [fine[0]]
    for _ in range(S):
        x, vv, _, _ = oracle.vv(pf, model, fine[-1][:, :3], fine[-1][:, 3:], w.q, dtf, sf)
        fine.append(np.concatenate([x, vv], 1))
        x, vv, _, _ = oracle.vv(pg, model, coarse[-1][:, :3], coarse[-1][:, 3:], w.q, dtg, sg)
        coarse.append(np.concatenate([x, vv], 1))
    lam0, it0, _, _ = oracle.parareal(pf, pg, model, w.xyz, v, w.q, S, sf, dtf, sg, dtg, 0, 0.0)
    assert it0 == 0
    for n in range(S + 1):
        assert np.array_equal(lam0[n], coarse[n])
    for K in (1, 2, S):
        lam, it, res, rc = oracle.parareal(pf, pg, model, w.xyz, v, w.q, S, sf, dtf, sg, dtg, K, 0.0)
        assert it == K
        for n in range(K + 1):
            assert np.array_equal(lam[n], fine[n]), (K, n)
        if K < S:
            assert not np.array_equal(lam[S], fine[S])
    assert rc == 0   # K = S is exact, reported as converged
    # the residual shrinks as slices become exact
    lam, it, res, rc = oracle.parareal(pf, pg, model, w.xyz, v, w.q, S, sf, dtf, sg, dtg, S, 1e-30)
    assert res[-1] <= res[0]


def test_cutoff_model_forces_are_cutoff_coulomb_plus_the_same_lennard_jones():
    """With the simple cutoff method (Section 5) the Coulomb part is the cutoff
    sum without intramolecular pairs, and the Lennard-Jones part is the same
    one the MSM model adds."""
    w, model, _ = small_water(64, 1.24, seed=17)
    kw = dict(lo=tuple(w.lo), hi=tuple(w.hi), levels=0, ke=138.935458)
    pc = oracle.OracleParams(0.6, 0.25, method=oracle.METHOD_CUTOFF, **kw)
    pm = oracle.OracleParams(0.6, 0.25, method=oracle.METHOD_MSM, **kw)
    no_lj = oracle.OracleModel(model.mass, model.molid, None, True, model.tri)
    ec0, fc0 = oracle.md_forces(pc, no_lj, w.xyz, w.q)
    e_ref, f_ref, _ = oracle.cutoff(w.xyz, w.q, 0.6, molid=model.molid)
    assert ec0 == pytest.approx(e_ref, rel=1e-13)
    np.testing.assert_allclose(fc0, f_ref, rtol=1e-12, atol=1e-9)
    ec, fc = oracle.md_forces(pc, model, w.xyz, w.q)
    em0, fm0 = oracle.md_forces(pm, no_lj, w.xyz, w.q)
    em, fm = oracle.md_forces(pm, model, w.xyz, w.q)
    assert ec - ec0 == pytest.approx(em - em0, rel=1e-10)
    np.testing.assert_allclose(fc - fc0, fm - fm0, rtol=1e-9, atol=1e-7)


def test_parareal_corrected_states_keep_the_rigid_geometry():
    """The correction of Section 4 adds and subtracts whole states; for rigid
    molecules each corrected state is projected back, so every iterate has
    the bond lengths and no relative velocity along any bond (the
    propagators' own tolerance), however far the coarse propagator is from
    the fine one (here the simple cutoff method against MSM)."""
    w, model, v = small_water(64, 1.24, seed=29)
    kw = dict(lo=tuple(w.lo), hi=tuple(w.hi), levels=0, ke=138.935458)
    pf = oracle.OracleParams(0.6, 0.25, **kw)
    pg = oracle.OracleParams(0.6, 0.25, method=oracle.METHOD_CUTOFF, **kw)
    lam, it, res, rc = oracle.parareal(pf, pg, model, w.xyz, v, w.q, 5, 5, 0.002, 5, 0.002, 1, 0.0)
    assert it == 1
    for n in range(6):
        x = lam[n, :, :3].reshape(-1, 3, 3)
        u = lam[n, :, 3:].reshape(-1, 3, 3)
        for (a, b), L in zip([(0, 1), (0, 2), (1, 2)], model.tri):
            r = x[:, a] - x[:, b]
            assert np.abs(np.linalg.norm(r, axis=1) - L).max() < 1e-9
            assert np.abs((r * (u[:, a] - u[:, b])).sum(1)).max() < 1e-9


# ---------------------------------------------------------------------------
# sliding computational window (Section 4): the first open state is exact after
# every iteration, states that moved less than the tolerance are accepted, and
# the window moves on; its state (lambda, coarse ring, counters) is a checkpoint
# ---------------------------------------------------------------------------
def _window_case():
    w, model, v = small_water(n_mol=27, side=0.93, seed=3)
    pf = oracle.OracleParams(0.8, 0.25, tuple(w.lo), tuple(w.hi), 0, 138.935458)
    pg = oracle.OracleParams(0.6, 0.5, tuple(w.lo), tuple(w.hi), 0, 138.935458)
    return w, model, v, pf, pg, (3, 0.001, 1, 0.003)


def _serial(p, model, w, v, steps, dt, T):
    out = [np.concatenate([w.xyz, v], 1)]
    for _ in range(T):
        x, vv, _, _ = oracle.vv(p, model, out[-1][:, :3], out[-1][:, 3:], w.q, dt, steps)
        out.append(np.concatenate([x, vv], 1))
    return np.stack(out)


@pytest.mark.parametrize("width", [1, 3, 7])
def test_window_with_zero_tolerance_is_the_serial_fine_trajectory(width):
    w, model, v, pf, pg, (sf, dtf, sg, dtg) = _window_case()
    T = 7
    fine = _serial(pf, model, w, v, sf, dtf, T)
    lam, ring = oracle.window_buffers(w.xyz, v, T, width)
    st = oracle.WindowState()
    rc = oracle.parareal_window(pf, pg, model, lam, ring, w.q, st, width, sf, dtf, sg, dtg, 0.0)
    assert rc == 0 and st.start == T
    assert np.array_equal(lam, fine)
    # exact states only: one per iteration, each iteration runs F on the whole window
    assert st.iterations == T
    assert st.fine_slices == sum(min(width, T - b) for b in range(T))


def test_full_window_iterates_are_plain_parareal():
    """A window as wide as the run with tolerance 0 moves by one slice per
    iteration, so after K iterations every state, converged or not, is plain
    parareal's after K iterations."""
    w, model, v, pf, pg, (sf, dtf, sg, dtg) = _window_case()
    T = 5
    for K in (1, 2, 4):
        ref, it, _, _ = oracle.parareal(pf, pg, model, w.xyz, v, w.q, T, sf, dtf, sg, dtg, K, 0.0)
        lam, ring = oracle.window_buffers(w.xyz, v, T, T)
        st = oracle.WindowState()
        rc = oracle.parareal_window(pf, pg, model, lam, ring, w.q, st, T, sf, dtf, sg, dtg, 0.0, max_iters=K)
        assert st.iterations == K and st.start == K
        assert np.array_equal(lam, ref), K


def _tolerance_run(max_iters_first=0):
    w, model, v, pf, pg, (sf, dtf, sg, dtg) = _window_case()
    T, W, tol = 9, 4, 2e-4
    lam, ring = oracle.window_buffers(w.xyz, v, T, W)
    st = oracle.WindowState()
    rc = oracle.parareal_window(pf, pg, model, lam, ring, w.q, st, W, sf, dtf, sg, dtg, tol,
                                max_iters=max_iters_first)
    return (w, model, v, pf, pg, sf, dtf, sg, dtg, T, W, tol), lam, ring, st, rc


def test_window_tolerance_accepts_several_states_per_iteration():
    (w, model, v, pf, pg, sf, dtf, sg, dtg, T, W, tol), lam, ring, st, rc = _tolerance_run()
    assert rc == 0 and st.start == T
    assert st.iterations < T   # some iteration accepted more than the exact state
    fine = _serial(pf, model, w, v, sf, dtf, T)
    coarse = _serial(pg, model, w, v, sg, dtg, T)
    err = np.abs(lam[:, :, :3] - fine[:, :, :3]).max()
    assert err < np.abs(coarse[:, :, :3] - fine[:, :, :3]).max()
    assert np.array_equal(lam[1], fine[1])   # the first state is always exact


def test_window_resume_from_a_checkpoint_is_bitwise_the_uninterrupted_run():
    case, full, _, st_full, _ = _tolerance_run()
    (w, model, v, pf, pg, sf, dtf, sg, dtg, T, W, tol) = case
    for stop in (1, 2, 3):
        _, lam, ring, st, rc = _tolerance_run(stop)
        assert rc == 1 and st.iterations == stop
        # checkpoint: copies of lambda, the ring and the state, then resume
        lam2, ring2, st2 = lam.copy(), ring.copy(), st.copy()
        rc = oracle.parareal_window(pf, pg, model, lam2, ring2, w.q, st2, W, sf, dtf, sg, dtg, tol)
        assert rc == 0
        assert np.array_equal(lam2, full)
        assert (st2.iterations, st2.fine_slices, st2.coarse_slices) == \
            (st_full.iterations, st_full.fine_slices, st_full.coarse_slices)


def test_window_resume_from_the_window_edge_with_zero_tolerance_is_serial_fine():
    """A checkpoint of the final states alone (the window rebuilt by the coarse
    prediction from its edge) still ends on the serial fine trajectory when
    only exact states are accepted."""
    w, model, v, pf, pg, (sf, dtf, sg, dtg) = _window_case()
    T, W = 6, 3
    fine = _serial(pf, model, w, v, sf, dtf, T)
    lam, ring = oracle.window_buffers(w.xyz, v, T, W)
    st = oracle.WindowState()
    assert oracle.parareal_window(pf, pg, model, lam, ring, w.q, st, W, sf, dtf, sg, dtg, 0.0, max_iters=2) == 1
    b = st.start
    lam2, ring2 = oracle.window_buffers(w.xyz, v, T, W)
    lam2[:b + 1] = lam[:b + 1]
    st2 = oracle.WindowState()
    st2.start = b
    assert oracle.parareal_window(pf, pg, model, lam2, ring2, w.q, st2, W, sf, dtf, sg, dtg, 0.0) == 0
    assert np.array_equal(lam2, fine)


# ---------------------------------------------------------------------------
# multiple time steps (Section 5 names them): impulse r-RESPA with the grid
# part of MSM as the slow force
# ---------------------------------------------------------------------------
def test_force_split_adds_up_to_the_model_force():
    w, model, _ = small_water(64, 1.24, seed=7)
    p = oracle.OracleParams(0.6, 0.2, tuple(w.lo), tuple(w.hi), 0)
    e, f = oracle.md_forces(p, model, w.xyz, w.q)
    ef, ff, es, fs = oracle.md_forces_split(p, model, w.xyz, w.q)
    assert ef + es == pytest.approx(e, rel=1e-12)
    np.testing.assert_allclose(ff + fs, f, rtol=0, atol=1e-12 * np.abs(f).max())


def test_mts_with_one_inner_step_is_velocity_verlet():
    w, model, v = small_water(64, 1.24, seed=7)
    p = oracle.OracleParams(0.6, 0.2, tuple(w.lo), tuple(w.hi), 0)
    x1, v1, ep1, ek1 = oracle.vv(p, model, w.xyz, v, w.q, 0.001, 10)
    x2, v2, ep2, ek2 = oracle.vv_mts(p, model, w.xyz, v, w.q, 0.001, 1, 10)
    assert np.abs(x1 - x2).max() < 1e-10
    assert np.abs(v1 - v2).max() < 1e-8
    assert ep2 == pytest.approx(ep1, rel=1e-10)


def test_mts_energy_error_is_second_order_and_shrinks_with_inner_steps():
    w, model, v = small_water(64, 1.24, seed=7)
    p = oracle.OracleParams(0.6, 0.2, tuple(w.lo), tuple(w.hi), 0)

    def drift(dt, n):
        _, _, e0, k0 = oracle.vv_mts(p, model, w.xyz, v, w.q, dt, n, 0)
        x, vv, e1, k1 = oracle.vv_mts(p, model, w.xyz, v, w.q, dt, n, int(round(0.2 / dt)))
        d = x.reshape(-1, 3, 3)
        assert np.abs(np.linalg.norm(d[:, 0] - d[:, 1], axis=1) - model.tri[0]).max() < 1e-9
        return abs((e1 + k1) - (e0 + k0))

    for n in (2, 4):
        ratio = drift(0.004, n) / drift(0.002, n)
        assert 2.5 < ratio < 6.0, (n, ratio)
    assert drift(0.004, 4) < drift(0.004, 2) < drift(0.004, 1)
