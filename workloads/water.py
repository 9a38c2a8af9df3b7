"""Seeded generators for point-charge and water-like test systems.

Units: nm, e, amu, ps, kJ/mol. Every generator returns float64 arrays; a
caller that runs in single precision rounds them with ``Workload.as_dtype`` and
hands the rounded values to both sides, so that a comparison measures
arithmetic and not input rounding.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Rigid 3-site water: TIP3P partial charges and geometry (Jorgensen et al. 1983).
Q_O = -0.834
Q_H = 0.417
R_OH = 0.09572          # nm
THETA_HOH = 104.52      # degrees
M_O = 16.0              # amu (as fixed for the parareal workload)
M_H = 1.0
KB_KJ_PER_MOL_K = 8.314462618e-3


@dataclasses.dataclass
class Workload:
    name: str
    xyz: np.ndarray                 # (N, 3) float64
    q: np.ndarray                   # (N,)   float64
    lo: np.ndarray                  # (3,)   domain lower corner
    hi: np.ndarray                  # (3,)   domain upper corner
    a: float = 1.2                  # short-range cutoff (nm)
    h: float = 0.25                 # finest grid spacing (nm)
    levels: int = 0                 # 0: choose from the domain
    molid: np.ndarray | None = None     # (N,) int32, molecule of each atom
    mass: np.ndarray | None = None      # (N,)
    vel: np.ndarray | None = None       # (N, 3)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def as_dtype(self, dtype) -> "Workload":
        """Round positions, charges and velocities to ``dtype`` and back to float64."""
        r = dataclasses.replace(self)
        r.xyz = self.xyz.astype(dtype).astype(np.float64)
        r.q = self.q.astype(dtype).astype(np.float64)
        if self.vel is not None:
            r.vel = self.vel.astype(dtype).astype(np.float64)
        return r

    def xyzq(self, dtype=np.float64) -> np.ndarray:
        out = np.empty((self.n, 4), dtype=dtype)
        out[:, :3] = self.xyz
        out[:, 3] = self.q
        return out


def uniform_pm(n: int = 2000, side: float = 4.0, seed: int = 1,
               a: float = 1.2, h: float = 0.25, levels: int = 0) -> Workload:
    """``n`` points uniform in [0, side)^3 with charges +1, -1, +1, ... (net zero
    for even ``n``); the domain is the cube itself."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, side, size=(n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return Workload(f"charges_{n}", xyz, q, np.zeros(3), np.full(3, side),
                    a=a, h=h, levels=levels)


def uniform_pm_box(n: int, dims, seed: int, a: float = 1.2, h: float = 0.25, levels: int = 0,
                   cluster: tuple | None = None) -> Workload:
    """``n`` points uniform in the box [0, dims) with charges +1, -1, ...; the
    domain is the box. ``cluster = (m, corner, side)`` puts the first ``m``
    points uniformly in the cube of edge ``side`` at ``corner`` instead (a
    dense spot in a sparse box)."""
    rng = np.random.default_rng(seed)
    dims = np.asarray(dims, dtype=np.float64)
    xyz = rng.uniform(0.0, 1.0, size=(n, 3)) * dims
    if cluster is not None:
        m, corner, side = cluster
        xyz[:m] = np.asarray(corner, dtype=np.float64) + rng.uniform(0.0, side, size=(m, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return Workload(f"charges_{n}_box", xyz, q, np.zeros(3), dims.copy(), a=a, h=h, levels=levels)


def _random_rotations(rng, m):
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    quat = rng.standard_normal((m, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    w, x, y, z = quat.T
    rot = np.empty((m, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def water_box(n_mol: int, sites: tuple[int, int, int], box: tuple[float, float, float],
              seed: int, jitter: float = 0.02, margin: float = 0.3,
              a: float = 1.2, h: float = 0.25, levels: int = 0,
              name: str | None = None) -> Workload:
    """``n_mol`` rigid 3-site molecules on a random subset of a jittered lattice.

    The lattice has ``sites`` points per axis spread evenly over ``box``; each
    chosen site holds an oxygen displaced by U(-jitter, jitter) per axis, and
    the two hydrogens follow from a uniformly random rotation of the fixed
    molecular geometry. Atom order is O, H, H per molecule. The domain is the
    box grown by ``margin`` on every side.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = sites
    total = nx * ny * nz
    if n_mol > total:
        raise ValueError("more molecules than lattice sites")
    pick = np.sort(rng.choice(total, size=n_mol, replace=False))
    ix = pick % nx
    iy = (pick // nx) % ny
    iz = pick // (nx * ny)
    sp = np.array(box, dtype=np.float64) / np.array(sites, dtype=np.float64)
    centre = (np.stack([ix, iy, iz], axis=1) + 0.5) * sp
    centre += rng.uniform(-jitter, jitter, size=centre.shape)
    half = math.radians(THETA_HOH) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [R_OH * math.sin(half), R_OH * math.cos(half), 0.0],
                      [-R_OH * math.sin(half), R_OH * math.cos(half), 0.0]])
    rot = _random_rotations(rng, n_mol)
    xyz = centre[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    xyz = xyz.reshape(-1, 3)
    q = np.tile(np.array([Q_O, Q_H, Q_H]), n_mol)
    molid = np.repeat(np.arange(n_mol, dtype=np.int32), 3)
    mass = np.tile(np.array([M_O, M_H, M_H]), n_mol)
    lo = np.full(3, -margin)
    hi = np.array(box, dtype=np.float64) + margin
    return Workload(name or f"water_{3 * n_mol}", xyz, q, lo, hi, a=a, h=h,
                    levels=levels, molid=molid, mass=mass)


def water_box_dims(n_atoms: int, density: float = 100.0, fill: float = 0.93):
    """Cube side and lattice size for ``n_atoms`` water-like atoms at ``density``."""
    n_mol = n_atoms // 3
    side = (n_atoms / density) ** (1.0 / 3.0)
    per_axis = int(math.ceil((n_mol / fill) ** (1.0 / 3.0)))
    return n_mol, (per_axis,) * 3, (side,) * 3


def maxwell_velocities(mass: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Gaussian velocities with variance kT/m per axis, centre-of-mass motion removed."""
    rng = np.random.default_rng(seed)
    kt = KB_KJ_PER_MOL_K * temperature
    v = rng.standard_normal((mass.shape[0], 3)) * np.sqrt(kt / mass)[:, None]
    vcom = (mass[:, None] * v).sum(axis=0) / mass.sum()
    return v - vcom


# Lennard-Jones of the TIP3P oxygen (Jorgensen et al. 1983); hydrogens carry none.
SIGMA_O = 0.315061      # nm
EPS_O = 0.6364          # kJ/mol


def water_model_arrays(n_atoms: int):
    """Per-atom masses, molecule ids and (sigma, epsilon) of n_atoms/3 water
    molecules in O, H, H order, and the three rigid distances O-H1, O-H2, H1-H2."""
    n_mol = n_atoms // 3
    mass = np.tile(np.array([M_O, M_H, M_H]), n_mol)
    molid = np.repeat(np.arange(n_mol, dtype=np.int32), 3)
    lj = np.tile(np.array([[SIGMA_O, EPS_O], [0.0, 0.0], [0.0, 0.0]]), (n_mol, 1))
    hh = 2.0 * R_OH * math.sin(math.radians(THETA_HOH) / 2.0)
    return mass, molid, lj, (R_OH, R_OH, hh)


def rigid_water_velocities(xyz: np.ndarray, temperature: float, seed: int) -> np.ndarray:
    """Velocities of rigid molecules (O, H, H triples): a Gaussian centre-of-mass
    velocity with variance kT/M and a Gaussian angular momentum with covariance
    kT I, so every intramolecular distance is constant to first order. The
    total momentum is removed."""
    rng = np.random.default_rng(seed)
    kt = KB_KJ_PER_MOL_K * temperature
    x = xyz.reshape(-1, 3, 3)
    m = np.array([M_O, M_H, M_H])
    mtot = m.sum()
    com = (m[None, :, None] * x).sum(axis=1) / mtot
    rel = x - com[:, None, :]
    inertia = (m[None, :, None, None] * ((rel ** 2).sum(-1)[..., None, None] * np.eye(3)
                                           - rel[..., :, None] * rel[..., None, :])).sum(axis=1)
    chol = np.linalg.cholesky(kt * inertia)
    ang = np.einsum("mij,mj->mi", chol, rng.standard_normal((x.shape[0], 3)))
    omega = np.linalg.solve(inertia, ang[..., None])[..., 0]
    vcom = rng.standard_normal((x.shape[0], 3)) * math.sqrt(kt / mtot)
    vcom -= vcom.mean(axis=0)
    v = vcom[:, None, :] + np.cross(omega[:, None, :], rel)
    return v.reshape(-1, 3)


def uneven_batch_sizes(count: int = 8, smallest: float = 1.0e4, ratio: float = 20.0):
    """Atom counts growing geometrically from ``smallest`` by ``ratio`` overall,
    each a multiple of 3: 9,999 ... 200,001 for the defaults."""
    out = []
    for s in range(count):
        n = smallest * ratio ** (s / (count - 1))
        out.append(3 * int(round(n / 3.0)))
    return out


def named(name: str, **kw) -> Workload:
    """The standard workloads, by a name that says what they are."""
    if name == "charges_2000":
        return uniform_pm(2000, 4.0, seed=kw.get("seed", 1))
    if name == "water_99999":
        return water_box(33333, (33, 33, 33), (10.0, 10.0, 10.0), seed=kw.get("seed", 2),
                         margin=kw.get("margin", 0.3), name=name)
    if name == "water_999999":
        return water_box(333333, (70, 70, 70), (21.5, 21.5, 21.5), seed=kw.get("seed", 3),
                         margin=kw.get("margin", 0.3), name=name)
    if name == "water_12675000":
        return water_box(4225000, (97, 210, 210), (30.0, 65.0, 65.0), seed=kw.get("seed", 5),
                         margin=kw.get("margin", 0.3), name=name)
    raise KeyError(name)
