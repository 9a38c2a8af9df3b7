"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks a fact that the paper (Section 3 unless stated) or plain
mathematics fixes: closed forms, smoothness conditions, the telescoping of the
kernel splitting, moment preservation, an independent dense evaluation of the
nested interpolation formula, brute-force Coulomb within the method's stated
error bound, finite differences, Newton's third law and grid symmetries. A
plausible mistake in the oracle (a dropped term, a wrong sign, index or
transposition) fails at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import dense
from workloads import uniform_pm, water_box

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def fd(f, x, eps=1e-5):
    return (f(x + eps) - f(x - eps)) / (2 * eps)


def fd2(f, x, eps=1e-4):
    return (f(x + eps) - 2 * f(x) + f(x - eps)) / eps ** 2


# --------------------------------------------------------------------------
# smoothing function gamma (Section 3): even quartic inside, 1/rho outside,
# joined with C2 continuity.
# --------------------------------------------------------------------------
def test_gamma_is_reciprocal_beyond_one(orc):
    for rho in [1.0, 1.3, 2.0, 7.5]:
        assert orc.gamma(rho) == pytest.approx(1.0 / rho, rel=1e-15)


def test_gamma_is_even_quartic_inside(orc):
    # A polynomial in rho^2 of degree 2 is fixed by three samples; every other
    # sample on [0, 1) must lie on it.
    s = np.array([0.0, 0.4, 0.8])
    coef = np.polyfit(s ** 2, orc.gamma(s), 2)
    for rho in np.linspace(0.05, 0.99, 17):
        assert orc.gamma(rho) == pytest.approx(np.polyval(coef, rho ** 2), abs=1e-13)


def test_gamma_c2_join(orc):
    g = lambda x: orc.gamma(x)  # noqa: E731
    left = lambda x: np.polyval(np.polyfit(np.array([0.0, 0.4, 0.8]) ** 2, orc.gamma(np.array([0.0, 0.4, 0.8])), 2), x ** 2)  # noqa: E731
    # value, slope and curvature of the inner polynomial at rho = 1 match 1/rho
    assert left(1.0) == pytest.approx(1.0, abs=1e-12)
    assert fd(left, 1.0) == pytest.approx(-1.0, abs=1e-8)
    assert fd2(left, 1.0) == pytest.approx(2.0, abs=1e-5)
    # and the function itself is C1 across the join
    assert fd(g, 1.0, 1e-6) == pytest.approx(-1.0, abs=1e-6)
    assert orc.dgamma(1.0 - 1e-12) == pytest.approx(orc.dgamma(1.0 + 1e-12), abs=1e-10)


def test_dgamma_matches_finite_difference(orc):
    for rho in [0.1, 0.5, 0.93, 1.2, 3.0]:
        assert orc.dgamma(rho) == pytest.approx(fd(orc.gamma, rho), rel=1e-7, abs=1e-9)


# --------------------------------------------------------------------------
# nodal basis Phi (Section 3; cubic numerical Hermite, p = 3)
# --------------------------------------------------------------------------
def test_phi_interpolates_and_has_support_four(orc):
    for n in range(-4, 5):
        assert orc.Phi(float(n)) == (1.0 if n == 0 else 0.0)
    for t in [-3.5, -2.0, -2.7, 2.0, 2.01, 3.9]:
        assert orc.Phi(t) == 0.0


def test_phi_reproduces_quadratics(orc):
    rng = np.random.default_rng(0)
    for t in rng.uniform(-3, 3, 25):
        ns = np.arange(math.floor(t) - 3, math.floor(t) + 4)
        w = orc.Phi(t - ns)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (w * ns).sum() == pytest.approx(t, abs=1e-13)
        assert (w * ns ** 2).sum() == pytest.approx(t * t, abs=1e-12)
        # it is not cubic-exact: the numerical Hermite slopes are second order
    t = 0.3
    ns = np.arange(-3, 4)
    assert abs((orc.Phi(t - ns) * ns ** 3).sum() - t ** 3) > 1e-3


def test_phi_is_c1_piecewise_cubic(orc):
    # C1 at the knots
    for knot in [-2.0, -1.0, 0.0, 1.0, 2.0]:
        assert orc.dPhi(knot - 1e-9) == pytest.approx(orc.dPhi(knot + 1e-9), abs=1e-7)
    # slopes at the nodes are the central differences of the cardinal data
    assert orc.dPhi(0.0) == pytest.approx(0.0, abs=1e-15)
    assert orc.dPhi(1.0) == pytest.approx(-0.5, abs=1e-12)
    assert orc.dPhi(-1.0) == pytest.approx(0.5, abs=1e-12)
    # cubic on each unit interval: fourth differences vanish
    for left in [-2.0, -1.0, 0.0, 1.0]:
        xs = left + np.linspace(0.1, 0.9, 5)
        assert abs(np.diff(orc.Phi(xs), 4)[0]) < 1e-13
    for t in [-1.7, -0.4, 0.25, 1.5]:
        assert orc.dPhi(t) == pytest.approx(fd(orc.Phi, t), abs=1e-8)


def test_restriction_weights(orc):
    # a fine node at half-integer coarse offset d/2 weighs Phi(d/2)
    w = orc.Phi(np.arange(-3, 4) / 2.0)
    np.testing.assert_allclose(w, [-1 / 16, 0, 9 / 16, 1, 9 / 16, 0, -1 / 16], atol=1e-15)


# --------------------------------------------------------------------------
# kernel splitting (Section 3): 1/r = g* + g^0 + ... + g^{l-1}, telescoping
# --------------------------------------------------------------------------
@pytest.mark.parametrize("l", [1, 2, 3, 5])
def test_splitting_telescopes_to_reciprocal(orc, l):
    a = 1.2
    for r in [0.05, 0.3, 1.1, 1.2, 2.0, 3.7, 9.0, 30.0]:
        total = orc.gstar(r, a) + sum(orc.glevel(r, a, k, l) for k in range(l))
        assert total == pytest.approx(1.0 / r, rel=1e-13)


def test_splitting_supports(orc):
    a, l = 1.2, 4
    for r in [a, 1.5 * a, 3 * a]:
        assert orc.gstar(r, a) == pytest.approx(0.0, abs=1e-15)
    for k in range(l - 1):
        for r in [2 ** (k + 1) * a, 2 ** (k + 1) * a * 1.3]:
            assert orc.glevel(r, a, k, l) == pytest.approx(0.0, abs=1e-15)
        assert abs(orc.glevel(0.5 * 2 ** (k + 1) * a, a, k, l)) > 1e-3
    # beyond the cutoff the level kernels alone give 1/r (the short part is zero)
    for r in [1.25, 2.5, 6.0]:
        assert sum(orc.glevel(r, a, k, l) for k in range(l)) == pytest.approx(1.0 / r, rel=1e-13)


# --------------------------------------------------------------------------
# grids and the whole long-range chain against the dense nested formula
# --------------------------------------------------------------------------
def _tiny(seed=7, n=12, side=1.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, side, (n, 3)), rng.standard_normal(n), np.zeros(3), np.full(3, side)


@pytest.mark.parametrize("a,h,l", [(0.5, 0.25, 3), (0.6, 0.25, 2), (0.45, 0.3, 1)])
def test_fast_oracle_equals_dense_nested_formula(orc, a, h, l):
    xyz, q, lo, hi = _tiny()
    p = orc.OracleParams(a, h, tuple(lo), tuple(hi), l, 1.0)
    e, f, pot, st = orc.msm(p, xyz, q, stages=True)
    ed, phid, us, ul = dense.energy_potential(xyz, q, a, h, lo, hi, l, pad=1)
    assert e == pytest.approx(ed, rel=1e-13)
    np.testing.assert_allclose(st["u_long"], ul, rtol=0, atol=1e-13 * np.abs(ul).max())
    np.testing.assert_allclose(st["u_short"], us, rtol=0, atol=1e-13 * np.abs(us).max())
    np.testing.assert_allclose(pot, phid, rtol=0, atol=1e-13 * np.abs(phid).max())


def test_literal_pair_formula_matches_oracle_pair_energy(orc):
    # two unit charges: U = (g* + I(g_a))(r_12) + the grid self-energy residual of each
    # charge, 1/2 (I(g_a)(r_i, r_i) - gamma(0)/a), which the self term does not cancel exactly
    ri, rj = np.array([0.31, 0.52, 0.77]), np.array([0.95, 0.40, 0.28])
    lo, hi, a, h, l = np.zeros(3), np.full(3, 1.25), 0.5, 0.25, 2
    M = dense.long_range_matrix(np.stack([ri, rj]), a, h, lo, hi, l, pad=1)
    approx = float(dense.g_star(np.array(np.linalg.norm(ri - rj)), a)) + M[0, 1]
    self_res = 0.5 * (M[0, 0] + M[1, 1]) - float(dense.gamma(0.0)) / a
    p = orc.OracleParams(a, h, tuple(lo), tuple(hi), l, 1.0)
    e, _, _ = orc.msm(p, np.stack([ri, rj]), np.array([1.0, 1.0]))
    assert e == pytest.approx(approx + self_res, rel=1e-12)
    assert approx == pytest.approx(1.0 / np.linalg.norm(ri - rj), rel=0.02)
    assert abs(self_res) < 0.05 * float(dense.gamma(0.0)) / a


def test_grid_ranges_rule(orc):
    p = orc.OracleParams(1.2, 0.25, (0, 0, 0), (4, 4, 4), 0, 1.0)
    assert orc.levels(p) == 3     # the paper's three-grid example
    assert orc.grid_shape(p, 0) == ((-1, -1, -1), (20, 20, 20))
    assert orc.grid_shape(p, 1) == ((-2, -2, -2), (13, 13, 13))
    assert orc.grid_shape(p, 2) == ((-2, -2, -2), (9, 9, 9))


def test_grid_moments_preserved(orc):
    w = uniform_pm(300, 3.0, seed=3)
    p = orc.OracleParams(0.9, 0.25, tuple(w.lo), tuple(w.hi), 3, 1.0)
    q = np.random.default_rng(1).standard_normal(w.n)
    _, _, _, st = orc.msm(p, w.xyz, q, stages=True)
    m0 = q.sum()
    m1 = (q[:, None] * w.xyz).sum(0)
    m2 = (q[:, None, None] * w.xyz[:, :, None] * w.xyz[:, None, :]).sum(0)
    for k, grid in enumerate(st["q_grid"]):
        org, dim = orc.grid_shape(p, k)
        hk = 0.25 * 2 ** k
        ax = [w.lo[d] + hk * (org[d] + np.arange(dim[d])) for d in range(3)]
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        pos = np.stack([X, Y, Z], -1).reshape(-1, 3)
        g = grid.reshape(-1)
        assert g.sum() == pytest.approx(m0, abs=1e-11)
        np.testing.assert_allclose((g[:, None] * pos).sum(0), m1, atol=1e-10)
        np.testing.assert_allclose((g[:, None, None] * pos[:, :, None] * pos[:, None, :]).sum(0), m2, atol=1e-9)


def test_atoms_on_nodes(orc):
    # atoms exactly on level-0 nodes put their charge on that node only, and
    # read back exactly that node's potential
    lo, h = np.zeros(3), 0.25
    idx = np.array([[2, 3, 4], [5, 5, 1], [7, 2, 6], [3, 8, 8]])
    xyz = lo + h * idx
    q = np.array([1.0, -2.0, 0.5, 0.75])
    p = orc.OracleParams(0.6, h, (0, 0, 0), (2.25, 2.25, 2.25), 2, 1.0)
    _, _, _, st = orc.msm(p, xyz, q, stages=True)
    org, dim = orc.grid_shape(p, 0)
    g = st["q_grid"][0]
    expect = np.zeros_like(g)
    for (ix, iy, iz), qi in zip(idx, q):
        expect[iz - org[2], iy - org[1], ix - org[0]] += qi
    np.testing.assert_allclose(g, expect, atol=1e-15)
    u0 = st["u_grid"][0]
    for i, (ix, iy, iz) in enumerate(idx):
        assert st["u_long"][i] == pytest.approx(u0[iz - org[2], iy - org[1], ix - org[0]], abs=1e-13)


# --------------------------------------------------------------------------
# accuracy against brute-force Coulomb (Section 3: under 1 % relative error
# in potential for a C2 Taylor smoothing with a cubic Hermite basis)
# --------------------------------------------------------------------------
def _rel_rms(x, ref):
    return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))


def test_msm_within_stated_error_of_bruteforce(orc):
    w = uniform_pm(2000, 4.0, seed=1)
    p = orc.OracleParams.of(w)
    e, f, pot = orc.msm(p, w.xyz, w.q)
    e0, f0, p0 = orc.coulomb(w.xyz, w.q)
    assert _rel_rms(pot, p0) < 0.01
    assert _rel_rms(f, f0) < 0.01
    assert abs(e - e0) / abs(e0) < 0.01
    # a shorter cutoff at the same spacing is less accurate
    p2 = orc.OracleParams(0.8, w.h, tuple(w.lo), tuple(w.hi), 0, p.ke)
    _, f2, pot2 = orc.msm(p2, w.xyz, w.q)
    assert _rel_rms(f2, f0) > _rel_rms(f, f0)
    assert _rel_rms(pot2, p0) > _rel_rms(pot, p0)


def test_water_within_stated_error_of_bruteforce(orc):
    w = water_box(600, (13, 13, 13), (4.0, 4.0, 4.0), seed=11)
    p = orc.OracleParams.of(w)
    e, f, pot = orc.msm(p, w.xyz, w.q)
    e0, f0, p0 = orc.coulomb(w.xyz, w.q)
    assert _rel_rms(f, f0) < 0.01
    assert abs(e - e0) / abs(e0) < 0.01


def test_bruteforce_closed_forms(orc):
    # two charges
    e, f, pot = orc.coulomb(np.array([[0, 0, 0], [0.3, 0.4, 0.0]]), np.array([2.0, -1.5]), ke=1.0)
    assert e == pytest.approx(2.0 * -1.5 / 0.5, rel=1e-15)
    # F_0 = -dU/dr_0 = q0 q1 (r_0 - r_1) / r^3
    np.testing.assert_allclose(f[0], 2.0 * -1.5 * np.array([-0.3, -0.4, 0.0]) / 0.5 ** 3, rtol=1e-14)
    np.testing.assert_allclose(f[0], -f[1], rtol=1e-14)
    # eight unit charges on the corners of a unit cube:
    # 12 edges (r=1), 12 face diagonals (sqrt 2), 4 body diagonals (sqrt 3)
    c = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    e, f, _ = orc.coulomb(c, np.ones(8), ke=1.0)
    assert e == pytest.approx(12 + 12 / math.sqrt(2) + 4 / math.sqrt(3), rel=1e-14)
    np.testing.assert_allclose(f.sum(0), 0, atol=1e-13)


# --------------------------------------------------------------------------
# gradients (Section 2: F = -dU/dr), Newton's third law, symmetries
# --------------------------------------------------------------------------
def test_forces_are_minus_energy_gradient(orc):
    w = uniform_pm(200, 2.5, seed=5)
    p = orc.OracleParams(0.8, 0.25, tuple(w.lo), tuple(w.hi), 0, 1.0)
    _, f, pot = orc.msm(p, w.xyz, w.q)
    delta = 1e-4
    for i in [0, 17, 123]:
        for d in range(3):
            xp = w.xyz.copy()
            xm = w.xyz.copy()
            xp[i, d] += delta
            xm[i, d] -= delta
            ep = orc.msm(p, xp, w.q)[0]
            em = orc.msm(p, xm, w.q)[0]
            g = (ep - em) / (2 * delta)
            assert -g == pytest.approx(f[i, d], rel=2e-6, abs=1e-6 * np.abs(f).max())
    # U is quadratic in the charges: the central difference is exact
    for i in [3, 99]:
        qp = w.q.copy()
        qm = w.q.copy()
        qp[i] += 0.1
        qm[i] -= 0.1
        g = (orc.msm(p, w.xyz, qp)[0] - orc.msm(p, w.xyz, qm)[0]) / 0.2
        assert g == pytest.approx(pot[i], rel=1e-11)


def test_short_range_newton_third_law(orc):
    w = water_box(300, (10, 10, 10), (3.0, 3.0, 3.0), seed=4)
    p = orc.OracleParams.of(w, ke=1.0)
    _, _, _, st = orc.msm(p, w.xyz, w.q, stages=True)
    fs = w.q[:, None] * st["f_short"]
    assert np.abs(fs.sum(0)).max() < 1e-10 * np.abs(fs).max()


def test_translation_by_grid_steps_and_axis_symmetries(orc):
    rng = np.random.default_rng(9)
    xyz = rng.uniform(0.6, 2.4, (60, 3))
    q = rng.standard_normal(60)
    h = 0.25
    p = orc.OracleParams(0.7, h, (0, 0, 0), (3.5, 3.5, 3.5), 3, 1.0)
    e, f, pot = orc.msm(p, xyz, q)
    # shift by whole multiples of the coarsest spacing (4h for three grids)
    sh = np.array([4 * h, 0.0, 4 * h])
    e2, f2, _ = orc.msm(p, xyz + sh, q)
    assert e2 == pytest.approx(e, rel=1e-12)
    np.testing.assert_allclose(f2, f, atol=1e-11 * np.abs(f).max())
    # permute axes
    perm = [2, 0, 1]
    e3, f3, _ = orc.msm(p, xyz[:, perm], q)
    assert e3 == pytest.approx(e, rel=1e-12)
    np.testing.assert_allclose(f3, f[:, perm], atol=1e-11 * np.abs(f).max())
    # reflect x through a coarse node at 3.0 (a multiple of 4h): x -> 3 - x keeps the atoms inside
    xr = xyz.copy()
    xr[:, 0] = 3.0 - xr[:, 0]
    e4, f4, _ = orc.msm(p, xr, q)
    assert e4 == pytest.approx(e, rel=1e-12)
    fr = f.copy()
    fr[:, 0] *= -1
    np.testing.assert_allclose(f4, fr, atol=1e-11 * np.abs(f).max())
    # a half-spacing shift is not a grid symmetry: the approximation changes a little
    e5, _, _ = orc.msm(p, xyz + np.array([h / 2, 0, 0]), q)
    assert e5 != pytest.approx(e, rel=1e-12)
    assert e5 == pytest.approx(e, rel=1e-2)


def test_forces_continuous_across_cutoff_and_grid_planes(orc):
    # Section 3: the method gives continuous forces. Move one charge along x and
    # compare the force just left and right of a grid plane (x = 1.25, on the
    # level-0 lattice) and of the cutoff sphere of a second charge (x = 1.3).
    p = orc.OracleParams(0.6, 0.25, (0, 0, 0), (2.5, 2.5, 2.5), 2, 1.0)
    fixed = np.array([0.7, 1.1, 1.3])

    def force(x):
        return orc.msm(p, np.stack([fixed, [x, 1.1, 1.3]]), np.array([1.0, -1.0]))[1][1]

    scale = np.abs(force(1.2)).max()
    eps = 1e-9
    for xc in (1.25, 1.3):
        jump = np.abs(force(xc + eps) - force(xc - eps)).max()
        assert jump < 1e-6 * scale
    # the finite-difference step used here does resolve a real change in force
    assert np.abs(force(1.3 + 1e-3) - force(1.3 - 1e-3)).max() > 1e3 * 1e-6 * scale


def test_oracle_rejects_bad_inputs(orc):
    p = orc.OracleParams(0.6, 0.25, (0, 0, 0), (1, 1, 1), 0, 1.0)
    with pytest.raises(RuntimeError, match="-2"):
        orc.msm(p, np.array([[0.5, 0.5, 1.2]]), np.array([1.0]))
    with pytest.raises(RuntimeError, match="-3"):
        orc.msm(p, np.array([[0.5, np.nan, 0.5]]), np.array([1.0]))


def test_short_subset_matches_full_short_range(orc):
    # the spot-check routine (direct loop over all atoms) and the cell-list
    # short range of the full evaluation are two loop structures of one sum
    w = water_box(400, (11, 11, 11), (3.4, 3.4, 3.4), seed=8)
    p = orc.OracleParams.of(w, ke=1.0)
    _, _, _, st = orc.msm(p, w.xyz, w.q, stages=True)
    sel = np.array([0, 1, 2, 500, 1199])
    u, f = orc.short_subset(p, w.xyz, w.q, sel)
    np.testing.assert_allclose(u, st["u_short"][sel], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f, st["f_short"][sel], rtol=1e-12, atol=1e-10)


# --------------------------------------------------------------------------
# the simple cutoff method (Section 5: the coarse propagator the paper picks)
# --------------------------------------------------------------------------
def test_cutoff_closed_forms(orc):
    # eight unit charges on the corners of a unit cube, cutoff between the
    # face diagonal (sqrt 2) and the body diagonal (sqrt 3): the 12 edges and
    # 12 face diagonals count, the 4 body diagonals do not
    c = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], dtype=float)
    e, f, pot = orc.cutoff(c, np.ones(8), 1.6, ke=1.0)
    assert e == pytest.approx(12 + 12 / math.sqrt(2), rel=1e-14)
    # every corner sees 3 edges and 3 face diagonals
    np.testing.assert_allclose(pot, 3 + 3 / math.sqrt(2), rtol=1e-14)
    # corner (0,0,0): edge pushes of 1 along -x, -y, -z and face-diagonal
    # pushes of 1/2 along each of its two axes (1/r^2 times the unit vector)
    fe = 1.0 + 2 * (1 / 2) * (1 / math.sqrt(2))
    np.testing.assert_allclose(f[0], [-fe, -fe, -fe], rtol=1e-14)
    # cutoff below the edge length: nothing interacts
    e0, f0, p0 = orc.cutoff(c, np.ones(8), 0.99, ke=1.0)
    assert e0 == 0.0 and not f0.any() and not p0.any()
    # cutoff beyond the diagonal: all 28 pairs
    e3, _, _ = orc.cutoff(c, np.ones(8), 1.75, ke=1.0)
    assert e3 == pytest.approx(12 + 12 / math.sqrt(2) + 4 / math.sqrt(3), rel=1e-14)


def test_cutoff_molecule_exclusion_closed_form(orc):
    # two water-like triples; pairs inside a triple are left out, so the energy
    # is the nine intermolecular terms, here written out one by one
    x = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, 0.1, 0.0],
                  [0.4, 0.0, 0.0], [0.5, 0.0, 0.0], [0.4, 0.1, 0.0]])
    q = np.array([-0.8, 0.4, 0.4, -0.8, 0.4, 0.4])
    mol = np.array([0, 0, 0, 1, 1, 1])
    e, _, pot = orc.cutoff(x, q, 1.0, ke=1.0, molid=mol)
    ref = 0.0
    for i in range(3):
        for j in range(3, 6):
            ref += q[i] * q[j] / np.linalg.norm(x[i] - x[j])
    assert e == pytest.approx(ref, rel=1e-14)
    ref0 = sum(q[j] / np.linalg.norm(x[0] - x[j]) for j in range(3, 6))
    assert pot[0] == pytest.approx(ref0, rel=1e-14)


def test_cutoff_gradients_newton_and_euler(orc):
    w = uniform_pm(300, 3.0, seed=8)
    rc = 0.9
    e, f, pot = orc.cutoff(w.xyz, w.q, rc, ke=1.0)
    # Newton's third law pair by pair: zero net force
    np.testing.assert_allclose(f.sum(0), 0, atol=1e-10 * np.abs(f).max())
    # U = 1/2 sum q phi (bilinear in q)
    assert e == pytest.approx(0.5 * (w.q * pot).sum(), rel=1e-13)
    # F = -dU/dr by central differences, for atoms with no pair within 3 delta of the cutoff
    delta = 1e-5
    d = np.linalg.norm(w.xyz[:, None, :] - w.xyz[None, :, :], axis=-1)
    clear = [i for i in range(w.n) if np.all(np.abs(d[i] - rc) > 3 * delta)]
    for i in clear[:4]:
        for c in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, c] += delta
            xm[i, c] -= delta
            fd = -(orc.cutoff(xp, w.q, rc, ke=1.0)[0] - orc.cutoff(xm, w.q, rc, ke=1.0)[0]) / (2 * delta)
            assert f[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # phi_i = dU/dq_i exactly (U is quadratic in q)
    i = clear[0]
    qp, qm = w.q.copy(), w.q.copy()
    qp[i] += 0.5
    qm[i] -= 0.5
    fd = (orc.cutoff(w.xyz, qp, rc, ke=1.0)[0] - orc.cutoff(w.xyz, qm, rc, ke=1.0)[0]) / 1.0
    assert pot[i] == pytest.approx(fd, rel=1e-12)


def test_cutoff_beyond_the_box_is_exact_coulomb(orc):
    w = uniform_pm(150, 2.0, seed=9)
    ec, fc, pc = orc.coulomb(w.xyz, w.q, ke=1.0)
    e, f, p = orc.cutoff(w.xyz, w.q, 4.0, ke=1.0)
    assert e == pytest.approx(ec, rel=1e-13)
    np.testing.assert_allclose(f, fc, rtol=1e-12, atol=1e-12 * np.abs(fc).max())
    np.testing.assert_allclose(p, pc, rtol=1e-12, atol=1e-12 * np.abs(pc).max())


def test_cutoff_subset_rows_equal_the_full_evaluation(orc):
    w = water_box(300, (7, 7, 7), (2.2, 2.2, 2.2), seed=12)
    mol = np.arange(w.n) // 3
    _, f, p = orc.cutoff(w.xyz, w.q, 0.7, molid=mol)
    sel = np.array([0, 5, 77, w.n - 1])
    fs, ps = orc.cutoff_subset(w.xyz, w.q, 0.7, sel, molid=mol)
    np.testing.assert_array_equal(fs, f[sel])
    np.testing.assert_array_equal(ps, p[sel])


# --------------------------------------------------------------------------
# smoothing functions of other orders (Section 3: gamma of degree 2m; the
# paper selects m = 2 and names the trade-off between order and cost)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [1, 2, 3])
def test_gamma_of_order_m_joins_reciprocal_with_m_derivatives(orc, m):
    # inside, gamma_m is an even polynomial of degree 2m: an exact fit in rho^2
    # of degree m reproduces it, and no lower degree does
    s = np.linspace(0.0, 0.99, 4 * m + 3)
    vals = orc.gamma(s, m)
    coef = np.polyfit(s ** 2, vals, m)
    assert np.abs(np.polyval(coef, s ** 2) - vals).max() < 1e-12
    low = np.polyfit(s ** 2, vals, m - 1)
    assert np.abs(np.polyval(low, s ** 2) - vals).max() > 1e-4
    # as a polynomial in rho its derivatives at rho = 1 equal those of 1/rho,
    # (-1)^j j!, for j = 0 .. m, and the (m+1)-th does not
    poly = np.zeros(2 * m + 1)
    poly[::2] = coef   # highest power first: rho^(2m), rho^(2m-2), ...
    for j in range(m + 2):
        dj = np.polyval(np.polyder(poly, j), 1.0) if j else np.polyval(poly, 1.0)
        if j <= m:
            assert dj == pytest.approx((-1) ** j * math.factorial(j), rel=1e-9), j
        else:
            assert abs(dj - (-1) ** j * math.factorial(j)) > 1e-3
    assert orc.gamma(1.5, m) == pytest.approx(1 / 1.5, rel=1e-15)
    # derivative against central differences
    for rho in [0.2, 0.7, 0.95, 1.3]:
        fd = (orc.gamma(rho + 1e-6, m) - orc.gamma(rho - 1e-6, m)) / 2e-6
        assert orc.dgamma(rho, m) == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_gamma_order_two_is_the_printed_quartic(orc):
    for rho in [0.0, 0.3, 0.77, 0.999]:
        assert orc.gamma(rho, 2) == pytest.approx(15 / 8 - 5 / 4 * rho ** 2 + 3 / 8 * rho ** 4, rel=1e-14)


@pytest.mark.parametrize("m", [1, 3])
def test_splitting_of_order_m_telescopes(orc, m):
    a, l = 1.2, 4
    for r in [0.05, 0.3, 1.1, 2.0, 3.7, 9.0, 30.0]:
        total = orc.gstar(r, a, m) + sum(orc.glevel(r, a, k, l, m) for k in range(l))
        assert total == pytest.approx(1.0 / r, rel=1e-13)
    assert orc.gstar(1.3 * a, a, m) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("m", [1, 3])
def test_fast_oracle_of_order_m_equals_dense_nested_formula(orc, m):
    xyz, q, lo, hi = _tiny()
    p = orc.OracleParams(0.5, 0.25, tuple(lo), tuple(hi), 3, 1.0, smoothing=m)
    e, f, pot = orc.msm(p, xyz, q)
    ed, phid, us, ul = dense.energy_potential(xyz, q, 0.5, 0.25, lo, hi, 3, pad=1, m=m)
    assert e == pytest.approx(ed, rel=1e-13)
    np.testing.assert_allclose(pot, phid, rtol=0, atol=1e-13 * np.abs(phid).max())


@pytest.mark.parametrize("m", [1, 3])
def test_msm_of_order_m_within_stated_error_of_bruteforce(orc, m):
    w = uniform_pm(2000, 4.0, seed=1)
    p = orc.OracleParams.of(w, smoothing=m)
    e, f, pot = orc.msm(p, w.xyz, w.q)
    e0, f0, p0 = orc.coulomb(w.xyz, w.q)
    assert _rel_rms(pot, p0) < 0.01
    assert _rel_rms(f, f0) < 0.01
    assert abs(e - e0) / abs(e0) < 0.01
    # the smoothing order changes the result (the self term gamma_m(0)/a differs)
    e2, _, _ = orc.msm(orc.OracleParams.of(w), w.xyz, w.q)
    assert e != e2


# --------------------------------------------------------------------------
# the quintic nodal basis (Section 3: Phi of degree p; the paper selects p = 3)
# --------------------------------------------------------------------------
def test_quintic_basis_interpolates_and_reproduces_quartics(orc):
    nodes = np.arange(-4, 5).astype(float)
    np.testing.assert_array_equal(orc.Phi(nodes, 5), (nodes == 0).astype(float))
    # support |t| < 3
    for t in [3.0, 3.2, -3.0, -4.1]:
        assert orc.Phi(t, 5) == 0.0
    assert abs(orc.Phi(2.5, 5)) > 1e-3
    n = np.arange(-6, 7).astype(float)
    for x in [0.0, 0.21, 0.5, 0.93]:
        for deg in range(5):
            assert (orc.Phi(x - n, 5) * n ** deg).sum() == pytest.approx(x ** deg, abs=1e-13)
    x = 0.37
    assert abs((orc.Phi(x - n, 5) * n ** 5).sum() - x ** 5) > 1e-3


def test_quintic_basis_is_c2(orc):
    e = 1e-9
    for knot in [-2.0, -1.0, 0.0, 1.0, 2.0, 3.0]:
        assert orc.Phi(knot - e, 5) == pytest.approx(orc.Phi(knot + e, 5), abs=1e-8)
        assert orc.dPhi(knot - e, 5) == pytest.approx(orc.dPhi(knot + e, 5), abs=1e-7)
        # second derivative from one-sided differences of Phi'
        d = 1e-5
        left = (orc.dPhi(knot - e, 5) - orc.dPhi(knot - d, 5)) / (d - e)
        right = (orc.dPhi(knot + d, 5) - orc.dPhi(knot + e, 5)) / (d - e)
        assert left == pytest.approx(right, abs=2e-4)
    # Phi' against central differences
    for t in [-2.7, -1.3, -0.4, 0.2, 1.6, 2.9]:
        fd = (orc.Phi(t + 1e-6, 5) - orc.Phi(t - 1e-6, 5)) / 2e-6
        assert orc.dPhi(t, 5) == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_quintic_restriction_weights_are_six_point_midpoint_interpolation(orc):
    # Phi(d/2) at odd d equals the weights of the degree-5 Lagrange polynomial
    # through the six nodes -2 .. 3 evaluated at 1/2 (computed here from its
    # definition), mirrored
    nodes = np.arange(-2, 4).astype(float)
    lag = []
    for j, xj in enumerate(nodes):
        others = np.delete(nodes, j)
        lag.append(np.prod((0.5 - others) / (xj - others)))
    # node xj sits at distance |0.5 - xj| = |d|/2 from the midpoint
    for xj, wj in zip(nodes, lag):
        d = 2 * (0.5 - xj)
        assert orc.Phi(d / 2, 5) == pytest.approx(wj, abs=1e-15)
    assert sum(orc.Phi(d / 2, 5) for d in range(-6, 7)) == pytest.approx(2.0, abs=1e-14)


def test_quintic_basis_equals_dense_derivation(orc):
    # the C basis uses the quintic Hermite polynomials; the dense one solves
    # the six end conditions of each interval from scratch
    t = np.linspace(-3.4, 3.4, 137)
    np.testing.assert_allclose(orc.Phi(t, 5), dense.Phi(t, 5), atol=1e-14)


def test_quintic_grid_ranges(orc):
    p = orc.OracleParams(1.2, 0.25, (0, 0, 0), (4, 4, 4), 0, 1.0, basis=5)
    # level 0 spans base - 2 .. base + 3 of every atom: [-2, 16 + 3]
    assert orc.grid_shape(p, 0) == ((-2, -2, -2), (22, 22, 22))
    # level 1: ceil((-2 - 5) / 2) = -3 .. floor((19 + 5) / 2) = 12
    assert orc.grid_shape(p, 1) == ((-3, -3, -3), (16, 16, 16))


@pytest.mark.parametrize("m", [2, 3])
def test_fast_oracle_quintic_equals_dense_nested_formula(orc, m):
    xyz, q, lo, hi = _tiny()
    p = orc.OracleParams(0.5, 0.25, tuple(lo), tuple(hi), 3, 1.0, smoothing=m, basis=5)
    e, f, pot = orc.msm(p, xyz, q)
    ed, phid, us, ul = dense.energy_potential(xyz, q, 0.5, 0.25, lo, hi, 3, pad=1, m=m, p=5)
    assert e == pytest.approx(ed, rel=1e-13)
    np.testing.assert_allclose(pot, phid, rtol=0, atol=1e-13 * np.abs(phid).max())


def test_quintic_with_order_three_smoothing_beats_the_cubic_pair(orc):
    w = uniform_pm(2000, 4.0, seed=1)
    e0, f0, p0 = orc.coulomb(w.xyz, w.q)
    e3, f3, q3 = orc.msm(orc.OracleParams.of(w), w.xyz, w.q)
    e5, f5, q5 = orc.msm(orc.OracleParams.of(w, smoothing=3, basis=5), w.xyz, w.q)
    assert _rel_rms(f5, f0) < 0.5 * _rel_rms(f3, f0)
    assert _rel_rms(q5, p0) < 0.5 * _rel_rms(q3, p0)
    assert _rel_rms(f5, f0) < 0.01 and abs(e5 - e0) / abs(e0) < 0.01


# --------------------------------------------------------------------------
# Wolf summation (Section 5: the refined coarse propagator it proposes)
# --------------------------------------------------------------------------
def test_wolf_without_damping_beyond_a_neutral_cluster_is_exact_coulomb(orc):
    # with alpha = 0 the shift and self terms sum to -(sum q)^2 / (2 rc), zero
    # for a neutral system, so with every pair inside rc Wolf is exact Coulomb
    w = uniform_pm(120, 1.0, seed=3)
    assert abs(w.q.sum()) < 1e-12
    e0, f0, p0 = orc.coulomb(w.xyz, w.q, ke=1.0)
    e, f, p = orc.wolf(w.xyz, w.q, 5.0, 0.0, ke=1.0)
    assert e == pytest.approx(e0, rel=1e-13)
    np.testing.assert_allclose(f, f0, rtol=0, atol=1e-12 * np.abs(f0).max())
    np.testing.assert_allclose(p, p0, rtol=0, atol=1e-12 * np.abs(p0).max())
    # with damping the result moves away from it
    e2, _, _ = orc.wolf(w.xyz, w.q, 5.0, 2.0, ke=1.0)
    assert abs(e2 - e0) > 1e-3 * abs(e0)


def test_wolf_energy_is_continuous_where_the_simple_cutoff_jumps(orc):
    # move one charge of a pair across the cutoff sphere: the shifted pair
    # potential vanishes there, the plain cutoff jumps by q q / rc
    rc, alpha = 1.0, 2.5
    q = np.array([1.0, -1.0])
    for r in (rc - 1e-9, rc + 1e-9):
        x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        e, _, _ = orc.wolf(x, q, rc, alpha, ke=1.0)
        ec, _, _ = orc.cutoff(x, q, rc, ke=1.0)
        if r < rc:
            e_in, ec_in = e, ec
        else:
            e_out, ec_out = e, ec
    assert abs(e_in - e_out) < 1e-8
    assert abs(ec_in - ec_out) == pytest.approx(1.0 / rc, rel=1e-6)


def test_wolf_gradients_newton_and_self_term(orc):
    w = uniform_pm(300, 3.0, seed=11)
    rc, alpha = 0.9, 3.0
    e, f, pot = orc.wolf(w.xyz, w.q, rc, alpha, ke=1.0)
    np.testing.assert_allclose(f.sum(0), 0, atol=1e-10 * np.abs(f).max())
    assert e == pytest.approx(0.5 * (w.q * pot).sum(), rel=1e-13)
    delta = 1e-5
    d = np.linalg.norm(w.xyz[:, None, :] - w.xyz[None, :, :], axis=-1)
    clear = [i for i in range(w.n) if np.all(np.abs(d[i] - rc) > 3 * delta)]
    for i in clear[:3]:
        for c in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, c] += delta
            xm[i, c] -= delta
            fd = -(orc.wolf(xp, w.q, rc, alpha, ke=1.0)[0] - orc.wolf(xm, w.q, rc, alpha, ke=1.0)[0]) / (2 * delta)
            assert f[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # phi_i = dU/dq_i exactly (U is quadratic in q), the self term included
    i = clear[0]
    qp, qm = w.q.copy(), w.q.copy()
    qp[i] += 0.5
    qm[i] -= 0.5
    fd = orc.wolf(w.xyz, qp, rc, alpha, ke=1.0)[0] - orc.wolf(w.xyz, qm, rc, alpha, ke=1.0)[0]
    assert pot[i] == pytest.approx(fd, rel=1e-12)
    # an isolated charge sees only the self term: phi = -2 (erfc(alpha rc)/(2 rc) + alpha/sqrt(pi)) q
    e1, _, p1 = orc.wolf(np.zeros((1, 3)), np.array([1.0]), rc, 0.0, ke=1.0)
    assert p1[0] == pytest.approx(-1.0 / rc, rel=1e-14)
    assert e1 == pytest.approx(-0.5 / rc, rel=1e-14)


def test_wolf_model_forces_are_wolf_plus_the_same_lennard_jones():
    import oracle
    w = water_box(64, (4, 4, 4), (1.24, 1.24, 1.24), seed=17, margin=0.6)
    from workloads import water_model_arrays
    mass, molid, lj, tri = water_model_arrays(w.n)
    kw = dict(lo=tuple(w.lo), hi=tuple(w.hi), levels=0, ke=138.935458)
    pw = oracle.OracleParams(0.6, 0.25, method=oracle.METHOD_WOLF, alpha=3.0, **kw)
    pc = oracle.OracleParams(0.6, 0.25, method=oracle.METHOD_CUTOFF, **kw)
    full = oracle.OracleModel(mass, molid, lj, True, tri)
    no_lj = oracle.OracleModel(mass, molid, None, True, tri)
    ew0, fw0 = oracle.md_forces(pw, no_lj, w.xyz, w.q)
    e_ref, f_ref, _ = oracle.wolf(w.xyz, w.q, 0.6, 3.0, molid=molid)
    assert ew0 == pytest.approx(e_ref, rel=1e-13)
    ew, fw = oracle.md_forces(pw, full, w.xyz, w.q)
    ec0, fc0 = oracle.md_forces(pc, no_lj, w.xyz, w.q)
    ec, fc = oracle.md_forces(pc, full, w.xyz, w.q)
    assert ew - ew0 == pytest.approx(ec - ec0, rel=1e-10)
