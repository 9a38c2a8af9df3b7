"""ctypes bindings of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import threading

import numpy as np

from . import build as _build

MAXLEV = 16
_lock = threading.Lock()
_lib = None

_dp = C.POINTER(C.c_double)


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("h", C.c_double), ("levels", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("ke", C.c_double), ("method", C.c_int),
                ("smoothing", C.c_int), ("basis", C.c_int), ("alpha", C.c_double)]


METHOD_MSM = 0
METHOD_CUTOFF = 1
METHOD_WOLF = 2


class _Stages(C.Structure):
    _fields_ = [("u_short", _dp), ("f_short", _dp),
                ("q_grid", _dp * MAXLEV), ("ucut_grid", _dp * MAXLEV), ("u_grid", _dp * MAXLEV),
                ("u_long", _dp), ("g_long", _dp)]


@dataclasses.dataclass
class OracleParams:
    a: float
    h: float
    lo: tuple
    hi: tuple
    levels: int = 0
    ke: float = 138.935458
    method: int = METHOD_MSM    # METHOD_CUTOFF: the simple cutoff method at a (dynamics oracle)
    smoothing: int = 0          # order m of gamma (degree 2m); 0 = 2
    basis: int = 0              # degree p of Phi: 3 (0 = 3) or 5
    alpha: float = 0.0          # Wolf damping (1/nm), METHOD_WOLF only

    def c(self) -> _Params:
        p = _Params()
        p.a, p.h, p.levels, p.ke = float(self.a), float(self.h), int(self.levels), float(self.ke)
        p.method = int(self.method)
        p.smoothing = int(self.smoothing)
        p.basis = int(self.basis)
        p.alpha = float(self.alpha)
        for d in range(3):
            p.lo[d] = float(self.lo[d])
            p.hi[d] = float(self.hi[d])
        return p

    @classmethod
    def of(cls, w, ke: float = 138.935458, smoothing: int = 0, basis: int = 0) -> "OracleParams":
        return cls(w.a, w.h, tuple(w.lo), tuple(w.hi), w.levels, ke, smoothing=smoothing, basis=basis)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = _build.compile_oracle(force=False)
            L = C.CDLL(path)
            for name in ("orc_gamma", "orc_dgamma", "orc_Phi", "orc_dPhi"):
                getattr(L, name).restype = C.c_double
                getattr(L, name).argtypes = [C.c_double]
            for name in ("orc_Phi_p", "orc_dPhi_p"):
                getattr(L, name).restype = C.c_double
                getattr(L, name).argtypes = [C.c_double, C.c_int]
            for name in ("orc_gamma_m", "orc_dgamma_m"):
                getattr(L, name).restype = C.c_double
                getattr(L, name).argtypes = [C.c_double, C.c_int]
            L.orc_gstar_m.restype = C.c_double
            L.orc_gstar_m.argtypes = [C.c_double, C.c_double, C.c_int]
            L.orc_glevel_m.restype = C.c_double
            L.orc_glevel_m.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
            L.orc_gstar.restype = C.c_double
            L.orc_gstar.argtypes = [C.c_double, C.c_double]
            L.orc_glevel.restype = C.c_double
            L.orc_glevel.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
            L.orc_levels.restype = C.c_int
            L.orc_levels.argtypes = [C.POINTER(_Params)]
            L.orc_grid_shape.restype = C.c_int
            L.orc_grid_shape.argtypes = [C.POINTER(_Params), C.c_int, C.c_int * 3, C.c_int * 3]
            L.orc_msm.restype = C.c_int
            L.orc_msm.argtypes = [C.POINTER(_Params), C.c_int64, _dp, _dp, _dp, _dp, _dp,
                                  C.POINTER(_Stages)]
            L.orc_coulomb.restype = C.c_int
            L.orc_threads.restype = C.c_int
            L.orc_threads.argtypes = []
            L.orc_set_threads.restype = None
            L.orc_set_threads.argtypes = [C.c_int]
            L.orc_coulomb.argtypes = [C.c_int64, _dp, _dp, C.c_double, _dp, _dp, _dp]
            L.orc_cutoff.restype = C.c_int
            L.orc_cutoff.argtypes = [C.c_int64, _dp, _dp, C.POINTER(C.c_int32), C.c_double, C.c_double, _dp, _dp,
                                     _dp]
            L.orc_wolf.restype = C.c_int
            L.orc_wolf.argtypes = [C.c_int64, _dp, _dp, C.POINTER(C.c_int32), C.c_double, C.c_double, C.c_double,
                                   _dp, _dp, _dp]
            L.orc_cutoff_subset.restype = C.c_int
            L.orc_cutoff_subset.argtypes = [C.c_int64, _dp, _dp, C.POINTER(C.c_int32), C.c_double, C.c_double,
                                            C.c_int64, C.POINTER(C.c_int64), _dp, _dp]
            _lib = L
        return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _vec(f):
    def g(x):
        if np.isscalar(x):
            return f(float(x))
        return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))
    return g


def gamma(rho, m: int = 2):
    """Smoothing function of order m (degree 2m); m = 2 is the paper's."""
    return _vec(lambda x: lib().orc_gamma_m(x, int(m)))(rho)


def dgamma(rho, m: int = 2):
    return _vec(lambda x: lib().orc_dgamma_m(x, int(m)))(rho)
def Phi(t, p: int = 3):
    """Nodal basis of degree p (3: the paper's cubic Hermite; 5: quintic)."""
    return _vec(lambda x: lib().orc_Phi_p(x, int(p)))(t)


def dPhi(t, p: int = 3):
    return _vec(lambda x: lib().orc_dPhi_p(x, int(p)))(t)


def gstar(r, a, m: int = 2):
    return _vec(lambda x: lib().orc_gstar_m(x, float(a), int(m)))(r)


def glevel(r, a, k, l, m: int = 2):
    return _vec(lambda x: lib().orc_glevel_m(x, float(a), int(k), int(l), int(m)))(r)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Use n OpenMP threads in the oracle's parallel loops from now on."""
    lib().orc_set_threads(int(n))


def levels(p: OracleParams) -> int:
    cp = p.c()
    return lib().orc_levels(C.byref(cp))


def grid_shape(p: OracleParams, level: int):
    cp = p.c()
    org = (C.c_int * 3)()
    dim = (C.c_int * 3)()
    if lib().orc_grid_shape(C.byref(cp), level, org, dim) != 0:
        raise ValueError("bad level")
    return tuple(org), tuple(dim)


def msm(p: OracleParams, xyz, q, stages: bool = False):
    """Energy, forces (n,3) and potentials (n,) of the MSM approximation; with
    ``stages`` also a dict of the intermediate results of every step."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = xyz.shape[0]
    e = np.zeros(1)
    f = np.zeros((n, 3))
    pot = np.zeros(n)
    cp = p.c()
    st = None
    out = {}
    if stages:
        l = levels(p)
        st = _Stages()
        out["u_short"] = np.zeros(n)
        out["f_short"] = np.zeros((n, 3))
        out["u_long"] = np.zeros(n)
        out["g_long"] = np.zeros((n, 3))
        st.u_short, st.f_short = _ptr(out["u_short"]), _ptr(out["f_short"])
        st.u_long, st.g_long = _ptr(out["u_long"]), _ptr(out["g_long"])
        for key in ("q_grid", "ucut_grid", "u_grid"):
            out[key] = []
        for k in range(l):
            _, dim = grid_shape(p, k)
            shape = (dim[2], dim[1], dim[0])
            for key in ("q_grid", "ucut_grid", "u_grid"):
                arr = np.zeros(shape)
                out[key].append(arr)
                getattr(st, key)[k] = _ptr(arr)
    rc = lib().orc_msm(C.byref(cp), n, _ptr(xyz), _ptr(q), _ptr(e), _ptr(f), _ptr(pot),
                       C.byref(st) if st is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle msm failed with code {rc}")
    if stages:
        return float(e[0]), f, pot, out
    return float(e[0]), f, pot


def short_subset(p: OracleParams, xyz, q, sel):
    """u_short and the short-range force bracket of the atoms in ``sel``, each
    by a direct loop over all atoms (spot checks of very large systems)."""
    L = lib()
    if not getattr(L, "_subset_ready", False):
        L.orc_short_subset.restype = C.c_int
        L.orc_short_subset.argtypes = [C.POINTER(_Params), C.c_int64, _dp, _dp, C.c_int64, C.POINTER(C.c_int64),
                                       _dp, _dp]
        L._subset_ready = True
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    u = np.zeros(sel.shape[0])
    f = np.zeros((sel.shape[0], 3))
    cp = p.c()
    rc = L.orc_short_subset(C.byref(cp), xyz.shape[0], _ptr(xyz), _ptr(q), sel.shape[0],
                            sel.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(u), _ptr(f))
    if rc != 0:
        raise RuntimeError(f"oracle short_subset failed with code {rc}")
    return u, f


def coulomb(xyz, q, ke: float = 138.935458):
    """Exact Coulomb energy, forces and potentials by the direct pair sum."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = xyz.shape[0]
    e = np.zeros(1)
    f = np.zeros((n, 3))
    pot = np.zeros(n)
    rc = lib().orc_coulomb(n, _ptr(xyz), _ptr(q), float(ke), _ptr(e), _ptr(f), _ptr(pot))
    if rc != 0:
        raise RuntimeError(f"oracle coulomb failed with code {rc}")
    return float(e[0]), f, pot


def cutoff(xyz, q, rc, ke: float = 138.935458, molid=None):
    """Simple cutoff method (Section 5): energy, forces and potentials of
    Coulomb's law over the pairs closer than ``rc`` (pairs of equal ``molid``
    left out), by the direct pair loop."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = xyz.shape[0]
    mol = None if molid is None else np.ascontiguousarray(molid, dtype=np.int32)
    e = np.zeros(1)
    f = np.zeros((n, 3))
    pot = np.zeros(n)
    rc_ = lib().orc_cutoff(n, _ptr(xyz), _ptr(q), None if mol is None else mol.ctypes.data_as(C.POINTER(C.c_int32)),
                           float(rc), float(ke), _ptr(e), _ptr(f), _ptr(pot))
    if rc_ != 0:
        raise RuntimeError(f"oracle cutoff failed with code {rc_}")
    return float(e[0]), f, pot


def wolf(xyz, q, rc, alpha, ke: float = 138.935458, molid=None):
    """Wolf summation (Section 5): damped, shifted Coulomb below ``rc`` with
    damping ``alpha`` and the self term; energy, forces and potentials."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    n = xyz.shape[0]
    mol = None if molid is None else np.ascontiguousarray(molid, dtype=np.int32)
    e = np.zeros(1)
    f = np.zeros((n, 3))
    pot = np.zeros(n)
    rc_ = lib().orc_wolf(n, _ptr(xyz), _ptr(q), None if mol is None else mol.ctypes.data_as(C.POINTER(C.c_int32)),
                         float(rc), float(alpha), float(ke), _ptr(e), _ptr(f), _ptr(pot))
    if rc_ != 0:
        raise RuntimeError(f"oracle wolf failed with code {rc_}")
    return float(e[0]), f, pot


def cutoff_subset(xyz, q, rc, sel, ke: float = 138.935458, molid=None):
    """Forces (len(sel), 3) and potentials of ``cutoff`` for the atoms in
    ``sel``, each by a direct loop over all atoms."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    mol = None if molid is None else np.ascontiguousarray(molid, dtype=np.int32)
    f = np.zeros((sel.shape[0], 3))
    pot = np.zeros(sel.shape[0])
    rc_ = lib().orc_cutoff_subset(xyz.shape[0], _ptr(xyz), _ptr(q),
                                  None if mol is None else mol.ctypes.data_as(C.POINTER(C.c_int32)), float(rc),
                                  float(ke), sel.shape[0], sel.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(f),
                                  _ptr(pot))
    if rc_ != 0:
        raise RuntimeError(f"oracle cutoff_subset failed with code {rc_}")
    return f, pot


# ---------------------------------------------------------------------------
# dynamics (md_oracle.c)
# ---------------------------------------------------------------------------
_ip = C.POINTER(C.c_int32)


class _Model(C.Structure):
    _fields_ = [("mass", _dp), ("molid", _ip), ("lj", _dp), ("rigid", C.c_int),
                ("tri", C.c_double * 3), ("tol", C.c_double)]


@dataclasses.dataclass
class OracleModel:
    """Molecular model of a dynamics run (see md_oracle.h)."""
    mass: np.ndarray
    molid: np.ndarray | None = None
    lj: np.ndarray | None = None
    rigid: bool = False
    tri: tuple = (0.0, 0.0, 0.0)
    tol: float = 1e-10

    def c(self):
        m = _Model()
        self._keep = [np.ascontiguousarray(self.mass, dtype=np.float64)]
        m.mass = _ptr(self._keep[0])
        if self.molid is not None:
            self._keep.append(np.ascontiguousarray(self.molid, dtype=np.int32))
            m.molid = self._keep[-1].ctypes.data_as(_ip)
        if self.lj is not None:
            self._keep.append(np.ascontiguousarray(self.lj, dtype=np.float64))
            m.lj = _ptr(self._keep[-1])
        m.rigid = 1 if self.rigid else 0
        for d in range(3):
            m.tri[d] = float(self.tri[d])
        m.tol = float(self.tol)
        return m


class WindowState(C.Structure):
    """Resumable state of a sliding-window parareal run (zeros: a new run)."""
    _fields_ = [("start", C.c_int), ("window_valid", C.c_int), ("iterations", C.c_int),
                ("last_accepted", C.c_int), ("fine_slices", C.c_int64), ("coarse_slices", C.c_int64),
                ("last_change", C.c_double)]

    def copy(self):
        c = WindowState()
        C.memmove(C.byref(c), C.byref(self), C.sizeof(WindowState))
        return c


def _md_lib():
    L = lib()
    if not getattr(L, "_md_ready", False):
        L.orc_md_forces.restype = C.c_int
        L.orc_md_forces.argtypes = [C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_vv.restype = C.c_int
        L.orc_vv.argtypes = [C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp, _dp, _dp, C.c_double, C.c_int,
                             _dp, _dp]
        L.orc_parareal.restype = C.c_int
        L.orc_parareal.argtypes = [C.POINTER(_Params), C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp, _dp,
                                   C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int, C.c_double, _dp,
                                   C.POINTER(C.c_int), _dp]
        L.orc_md_forces_split.restype = C.c_int
        L.orc_md_forces_split.argtypes = [C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp, _dp, _dp, _dp,
                                          _dp, _dp]
        L.orc_vv_mts.restype = C.c_int
        L.orc_vv_mts.argtypes = [C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp, _dp, _dp, C.c_double,
                                 C.c_int, C.c_int, _dp, _dp]
        L.orc_parareal_window.restype = C.c_int
        L.orc_parareal_window.argtypes = [C.POINTER(_Params), C.POINTER(_Params), C.POINTER(_Model), C.c_int64, _dp,
                                          C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_double,
                                          C.c_int, _dp, _dp, C.POINTER(WindowState)]
        L._md_ready = True
    return L


def md_forces(p: OracleParams, model: OracleModel, xyz, q):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.zeros_like(xyz)
    e = np.zeros(1)
    cp, cm = p.c(), model.c()
    rc = _md_lib().orc_md_forces(C.byref(cp), C.byref(cm), xyz.shape[0], _ptr(xyz), _ptr(q), _ptr(e), _ptr(f))
    if rc != 0:
        raise RuntimeError(f"oracle md_forces failed with code {rc}")
    return float(e[0]), f


def md_forces_split(p: OracleParams, model: OracleModel, xyz, q):
    """(e_fast, f_fast, e_slow, f_slow): the multiple-time-step split of the
    MSM model force (fast: short-range pairs and Lennard-Jones; slow: grid)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ff, fs = np.zeros_like(xyz), np.zeros_like(xyz)
    ef, es = np.zeros(1), np.zeros(1)
    cp, cm = p.c(), model.c()
    rc = _md_lib().orc_md_forces_split(C.byref(cp), C.byref(cm), xyz.shape[0], _ptr(xyz), _ptr(q), _ptr(ef),
                                       _ptr(ff), _ptr(es), _ptr(fs))
    if rc != 0:
        raise RuntimeError(f"oracle md_forces_split failed with code {rc}")
    return float(ef[0]), ff, float(es[0]), fs


def vv_mts(p: OracleParams, model: OracleModel, xyz, v, q, dt, ninner, nouter):
    """nouter multiple-time-step steps of dt with ninner fast steps each;
    returns new (xyz, v, epot, ekin)."""
    x = np.array(xyz, dtype=np.float64).reshape(-1, 3)
    vv_ = np.array(v, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ep, ek = np.zeros(1), np.zeros(1)
    cp, cm = p.c(), model.c()
    rc = _md_lib().orc_vv_mts(C.byref(cp), C.byref(cm), x.shape[0], _ptr(x), _ptr(vv_), _ptr(q), float(dt),
                              int(ninner), int(nouter), _ptr(ep), _ptr(ek))
    if rc != 0:
        raise RuntimeError(f"oracle vv_mts failed with code {rc}")
    return x, vv_, float(ep[0]), float(ek[0])


def vv(p: OracleParams, model: OracleModel, xyz, v, q, dt, nsteps):
    """Run nsteps of velocity Verlet; returns new (xyz, v, epot, ekin)."""
    x = np.array(xyz, dtype=np.float64).reshape(-1, 3)
    vv_ = np.array(v, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ep, ek = np.zeros(1), np.zeros(1)
    cp, cm = p.c(), model.c()
    rc = _md_lib().orc_vv(C.byref(cp), C.byref(cm), x.shape[0], _ptr(x), _ptr(vv_), _ptr(q), float(dt),
                          int(nsteps), _ptr(ep), _ptr(ek))
    if rc != 0:
        raise RuntimeError(f"oracle vv failed with code {rc}")
    return x, vv_, float(ep[0]), float(ek[0])


def parareal(pf: OracleParams, pg: OracleParams, model: OracleModel, xyz, v, q, nslices, steps_f, dt_f,
             steps_g, dt_g, kmax, tol):
    """Returns (lambda[(nslices+1), n, 6], iterations, residual per iteration, return code)."""
    x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    state = np.ascontiguousarray(np.concatenate([x, np.asarray(v, dtype=np.float64).reshape(-1, 3)], axis=1))
    q = np.ascontiguousarray(q, dtype=np.float64)
    lam = np.zeros((nslices + 1, n, 6))
    iters = C.c_int(0)
    resid = np.zeros(max(kmax, 1))
    cf, cg, cm = pf.c(), pg.c(), model.c()
    rc = _md_lib().orc_parareal(C.byref(cf), C.byref(cg), C.byref(cm), n, _ptr(q), _ptr(state), int(nslices),
                                int(steps_f), float(dt_f), int(steps_g), float(dt_g), int(kmax), float(tol),
                                _ptr(lam), C.byref(iters), _ptr(resid))
    if rc < 0:
        raise RuntimeError(f"oracle parareal failed with code {rc}")
    return lam, iters.value, resid[:iters.value], rc


def window_buffers(xyz, v, nslices, width):
    """lambda[(nslices+1), n, 6] holding the initial state in slice 0, and a zero
    coarse ring[width, n, 6], for a new sliding-window run."""
    x = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    lam = np.zeros((nslices + 1, x.shape[0], 6))
    lam[0, :, :3] = x
    lam[0, :, 3:] = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    return lam, np.zeros((width, x.shape[0], 6))


def parareal_window(pf: OracleParams, pg: OracleParams, model: OracleModel, lam, ring, q, state: WindowState,
                    width, steps_f, dt_f, steps_g, dt_g, tol, max_iters=0):
    """Sliding-window parareal in place on lam and ring (float64, C order) and
    state; returns 0 when every slice is final, 1 when stopped by max_iters."""
    assert lam.dtype == np.float64 and lam.flags.c_contiguous and lam.shape[2] == 6
    assert ring.dtype == np.float64 and ring.flags.c_contiguous and ring.shape[0] == width
    q = np.ascontiguousarray(q, dtype=np.float64)
    cf, cg, cm = pf.c(), pg.c(), model.c()
    rc = _md_lib().orc_parareal_window(C.byref(cf), C.byref(cg), C.byref(cm), lam.shape[1], _ptr(q),
                                       lam.shape[0] - 1, int(width), int(steps_f), float(dt_f), int(steps_g),
                                       float(dt_g), float(tol), int(max_iters), _ptr(lam), _ptr(ring),
                                       C.byref(state))
    if rc < 0:
        raise RuntimeError(f"oracle parareal_window failed with code {rc}")
    return rc
