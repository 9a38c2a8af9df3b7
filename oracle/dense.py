"""Dense-matrix evaluation of the multilevel approximation (test infrastructure).

The paper (Section 3) approximates the reciprocal distance by nested grid
interpolation,

    1/r  ~  g* + I^0(g^0 + I^1(g^1 + ... + I^{l-2}(g^{l-2} + I^{l-1} g^{l-1})...)),

with I^k g(r_i, r_j) = sum_mu sum_nu phi^k_mu(r_i) g(r^k_mu, r^k_nu) phi^k_nu(r_j).
This module writes that formula out as explicit matrices on tiny inputs:
Phi0[i, mu] = phi^0_mu(r_i), R_k[mu, nu] = phi^{k+1}_mu(r^k_nu) and
G_k[mu, nu] = g^k(r^k_mu, r^k_nu), so that the long-range potential is
Phi0 (G_0 + R_0^T (G_1 + R_1^T (...) R_1) R_0) Phi0^T q. The grids are padded
well beyond the nodes any atom can reach, so agreement with the fast oracle
also shows that its truncated grids lose no term.

It is NumPy only and shares no code with the C oracle; its smoothing function
and basis are written in the expanded polynomial form rather than the
Hermite-basis form the C file uses.
"""
from __future__ import annotations

import math

import numpy as np


def gamma(rho, m=2):
    """1/rho for rho >= 1; inside, (rho^2)^(-1/2) expanded about rho^2 = 1 up
    to the (rho^2 - 1)^m term (m = 2: 15/8 - 5/4 rho^2 + 3/8 rho^4)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = rho ** 2 - 1.0
    inner = np.zeros_like(rho)
    for k in range(m + 1):
        inner = inner + math.prod(-0.5 - i for i in range(k)) / math.factorial(k) * u ** k
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        outer = 1.0 / rho
    return np.where(rho >= 1.0, outer, inner)


def _cardinal_hermite(t, order, stencils):
    """Hermite interpolant of the cardinal data c(n) = [n == 0] on each unit
    interval, with node derivatives of orders 1 .. order taken from the given
    central-difference stencils; the interpolating polynomial on [n, n+1] is
    found by solving its 2(order+1) end conditions."""
    t = np.asarray(t, dtype=np.float64)
    deg = 2 * order + 1
    out = np.zeros_like(t)
    n_all = np.floor(t).astype(int)
    for n in np.unique(n_all):
        rows, rhs = [], []
        for end, node in ((0.0, n), (1.0, n + 1)):
            vals = [1.0 if node == 0 else 0.0]
            for st in stencils[:order]:
                vals.append(sum(c * (1.0 if node + off == 0 else 0.0) for off, c in st))
            for d, v in enumerate(vals):
                # d-th derivative of sum_j a_j s^j at s = end
                rows.append([math.perm(j, d) * end ** (j - d) if j >= d else 0.0 for j in range(deg + 1)])
                rhs.append(v)
        coef = np.linalg.solve(np.array(rows), np.array(rhs))
        sel = n_all == n
        s = t[sel] - n
        out[sel] = sum(c * s ** j for j, c in enumerate(coef))
    return out


def Phi(t, p=3):
    """Nodal basis of degree p: p = 3 in closed form; p = 5 from its
    definition (slopes and second derivatives by five-point differences)."""
    if p == 5:
        d1 = ((-2, 1 / 12), (-1, -8 / 12), (1, 8 / 12), (2, -1 / 12))
        d2 = ((-2, -1 / 12), (-1, 16 / 12), (0, -30 / 12), (1, 16 / 12), (2, -1 / 12))
        return _cardinal_hermite(t, 2, (d1, d2))
    s = np.abs(np.asarray(t, dtype=np.float64))
    near = (1.0 - s) * (1.0 + s - 1.5 * s * s)
    far = -0.5 * (s - 1.0) * (2.0 - s) ** 2
    return np.where(s <= 1.0, near, np.where(s < 2.0, far, 0.0))


def g_level(r, a, k, l, m=2):
    ak = a * 2.0 ** k
    if k == l - 1:
        return gamma(r / ak, m) / ak
    return gamma(r / ak, m) / ak - gamma(r / (2 * ak), m) / (2 * ak)


def g_star(r, a, m=2):
    with np.errstate(divide="ignore"):
        return np.where(r < a, 1.0 / r - gamma(r / a, m) / a, 0.0)


def _nodes(lo, h, k, lo_idx, hi_idx):
    """Positions of the level-k nodes with integer indices in [lo_idx, hi_idx] per axis."""
    axes = [lo[d] + (2.0 ** k) * h * np.arange(lo_idx[d], hi_idx[d] + 1) for d in range(3)]
    zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def _basis(points, nodes, spacing, p=3):
    """Matrix B[i, mu] = prod_d Phi((x_i,d - x_mu,d) / spacing)."""
    w = np.ones((points.shape[0], nodes.shape[0]))
    for d in range(3):
        w *= Phi((points[:, d][:, None] - nodes[:, d][None, :]) / spacing, p)
    return w


def _pair_dist(x):
    diff = x[:, None, :] - x[None, :, :]
    return np.sqrt((diff ** 2).sum(axis=-1))


def long_range_matrix(xyz, a, h, lo, hi, levels, pad=2, m=2, p=3):
    """The N x N matrix of the nested grid approximation of g_a = g^0 + ... + g^{l-1}."""
    xyz = np.asarray(xyz, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    S = (p + 1) // 2
    n_lo = np.full(3, -S - pad)
    n_hi = np.floor((hi - lo) / h).astype(int) + S + 1 + pad
    ranges = []
    for k in range(levels):
        ranges.append((n_lo.copy(), n_hi.copy()))
        n_lo = np.floor((n_lo - (2 * S - 1)) / 2.0).astype(int) - pad
        n_hi = np.ceil((n_hi + (2 * S - 1)) / 2.0).astype(int) + pad
    nodes = [_nodes(lo, h, k, *ranges[k]) for k in range(levels)]
    Gs = [g_level(_pair_dist(nodes[k]), a, k, levels, m) for k in range(levels)]
    K = Gs[levels - 1]
    for k in range(levels - 2, -1, -1):
        R = _basis(nodes[k], nodes[k + 1], (2.0 ** (k + 1)) * h, p).T   # R[mu_coarse, nu_fine]
        K = Gs[k] + R.T @ K @ R
    P0 = _basis(xyz, nodes[0], h, p)
    return P0 @ K @ P0.T


def energy_potential(xyz, q, a, h, lo, hi, levels, ke=1.0, pad=2, m=2, p=3):
    """Energy and per-atom potentials of the multilevel approximation, dense,
    with the smoothing function of order m."""
    xyz = np.asarray(xyz, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    M = long_range_matrix(xyz, a, h, lo, hi, levels, pad, m, p)
    r = _pair_dist(xyz)
    np.fill_diagonal(r, np.inf)
    S = g_star(r, a, m)
    np.fill_diagonal(S, 0.0)
    u_short = S @ q
    u_long = M @ q
    phi = ke * (u_short + u_long - q * float(gamma(0.0, m)) / a)
    return 0.5 * float(q @ phi), phi, u_short, u_long


def literal_pair_sum(ri, rj, a, h, lo, hi, levels, pad=2):
    """The nested approximation of 1/|ri - rj| for one pair, as a single number."""
    M = long_range_matrix(np.stack([ri, rj]), a, h, lo, hi, levels, pad)
    r = math.dist(ri, rj)
    return float(g_star(np.array(r), a)) + M[0, 1]
