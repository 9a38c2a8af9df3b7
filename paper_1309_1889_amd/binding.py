"""ctypes binding of libmsmx.so; argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MSM_FP64 = 0
MSM_FP32 = 1
MAXLEV = 16
STAGES = ("bin", "short", "anterp", "restrict", "cutoff", "top", "prolong", "interp")

_lock = threading.Lock()
_lib = None


class MsmError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})" if what else f"{status_string(code)} ({code})")


class _Model(C.Structure):
    _fields_ = [("period", C.c_int64), ("molid_dev", C.c_void_p), ("lj_dev", C.c_void_p),
                ("rigid_triples", C.c_int), ("tri_len", C.c_double * 3), ("constraint_tol", C.c_double)]


class _PararealParams(C.Structure):
    _fields_ = [("nslices", C.c_int), ("kmax", C.c_int), ("tol", C.c_double), ("steps_f", C.c_int),
                ("dt_f", C.c_double), ("steps_g", C.c_int), ("dt_g", C.c_double)]


class _WindowParams(C.Structure):
    _fields_ = [("nslices", C.c_int), ("width", C.c_int), ("max_iters", C.c_int), ("pipeline", C.c_int),
                ("chunk", C.c_int), ("tol", C.c_double), ("steps_f", C.c_int), ("dt_f", C.c_double),
                ("steps_g", C.c_int), ("dt_g", C.c_double)]


class WindowState(C.Structure):
    """Resumable state of a sliding-window parareal run (parareal_window_state);
    all zeros starts a new run."""
    _fields_ = [("start", C.c_int), ("window_valid", C.c_int), ("iterations", C.c_int),
                ("last_accepted", C.c_int), ("fine_slices", C.c_int64), ("coarse_slices", C.c_int64),
                ("last_change", C.c_double), ("seconds", C.c_double)]

    def copy(self):
        c = WindowState()
        C.memmove(C.byref(c), C.byref(self), C.sizeof(WindowState))
        return c


class _PararealReport(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("residual", C.c_double * 64),
                ("seconds", C.c_double)]


class _Tuning(C.Structure):
    _fields_ = [("pair_waves", C.c_int), ("stencil_threads", C.c_int), ("concurrent", C.c_int),
                ("pair_cell", C.c_int)]


def _tuning_dict(t):
    return {"pair_waves": t.pair_waves, "stencil_threads": t.stencil_threads, "concurrent": t.concurrent,
            "pair_cell": t.pair_cell}


METHODS = {"msm": 0, "cutoff": 1, "wolf": 2}


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("h", C.c_double), ("levels", C.c_int), ("precision", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("coulomb_k", C.c_double),
                ("max_atoms", C.c_int64), ("max_systems", C.c_int), ("method", C.c_int),
                ("smoothing", C.c_int), ("basis", C.c_int), ("alpha", C.c_double)]


def lib_path() -> str:
    return os.path.join(HERE, "libmsmx.so")


def lib():
    """Load libmsmx.so; raises if it is not built (there is no fallback)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = lib_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run `python -m paper_1309_1889_amd.build`")
        L = C.CDLL(path)
        vp = C.c_void_p
        L.msm_setup.argtypes = [C.POINTER(_Params), vp, C.POINTER(vp)]
        L.msm_setup.restype = C.c_int
        L.msm_destroy.argtypes = [vp]
        L.msm_destroy.restype = None
        L.msm_set_stream.argtypes = [vp, vp]
        L.msm_set_stream.restype = C.c_int
        L.msm_energy_forces.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double), vp, vp, vp, vp]
        L.msm_energy_forces.restype = C.c_int
        L.msm_get_status.argtypes = [vp]
        L.msm_get_status.restype = C.c_int
        L.msm_status_string.argtypes = [C.c_int]
        L.msm_status_string.restype = C.c_char_p
        L.msm_grid_shape.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.msm_grid_shape.restype = C.c_int
        L.msm_debug_stages.argtypes = [vp, C.c_int, vp, vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]
        L.msm_debug_stages.restype = C.c_int
        L.msm_enable_stage_timing.argtypes = [vp, C.c_int]
        L.msm_enable_stage_timing.restype = C.c_int
        L.msm_stage_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
        L.msm_stage_timing.restype = C.c_int
        L.msm_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.msm_get_tuning.restype = C.c_int
        L.msm_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
        L.msm_set_tuning.restype = C.c_int
        L.msm_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double), vp, C.c_int,
                                   C.POINTER(_Tuning)]
        L.msm_autotune.restype = C.c_int
        L.msm_set_graphs.argtypes = [vp, C.c_int]
        L.msm_set_graphs.restype = C.c_int
        L.msm_md_bind.argtypes = [vp, C.POINTER(_Model)]
        L.msm_md_bind.restype = C.c_int
        L.msm_vv_run.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double), vp, vp, C.c_int,
                                 C.c_double, vp, vp]
        L.msm_vv_run.restype = C.c_int
        L.msm_vv_mts_run.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double), vp, vp, C.c_int,
                                     C.c_int, C.c_double, vp, vp]
        L.msm_vv_mts_run.restype = C.c_int
        L.msm_energy_forces_noalloc.argtypes = [C.POINTER(_Params), vp, C.c_int64, vp, vp, vp, vp, vp]
        L.msm_energy_forces_noalloc.restype = C.c_int
        L.parareal_run.argtypes = [vp, vp, C.POINTER(_PararealParams), C.c_int64, vp, vp, vp, vp,
                                   C.POINTER(_PararealReport)]
        L.parareal_run.restype = C.c_int
        L.parareal_window_run.argtypes = [vp, vp, C.POINTER(_WindowParams), C.c_int64, vp, vp, vp, vp,
                                          C.POINTER(WindowState)]
        L.parareal_window_run.restype = C.c_int
        _lib = L
        return L


def status_string(code: int) -> str:
    try:
        return lib().msm_status_string(int(code)).decode()
    except ImportError:
        return "status %d" % code


def _check(code: int, what: str):
    if code < 0:
        raise MsmError(code, what)
    return code


def _require(t, name, dtype, device, shape):
    """Raise ValueError unless ``t`` is a contiguous tensor of ``dtype`` on
    ``device`` with exactly ``shape`` (the C side cannot check buffer sizes)."""
    if t is None:
        return
    if t.dtype != dtype or t.device != device or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)} on {device}; "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}"
                         f"{'' if t.is_contiguous() else ' (not contiguous)'}")


def _offsets(offsets, n):
    """Validated int64 system offsets: start at 0, non-decreasing, end at n."""
    offs = np.ascontiguousarray(np.asarray([0, n] if offsets is None else offsets, dtype=np.int64))
    if offs.ndim != 1 or len(offs) < 2 or offs[0] != 0 or offs[-1] != n or np.any(np.diff(offs) < 0):
        raise ValueError(f"offsets must rise from 0 to the number of atoms ({n})")
    return offs


def _domains(domains, nsys):
    if domains is None:
        return None, None
    dom = np.ascontiguousarray(np.asarray(domains, dtype=np.float64))
    if dom.size != nsys * 6:
        raise ValueError(f"domains must hold {nsys} x 6 values")
    dom = dom.reshape(nsys, 6)
    return dom, dom.ctypes.data_as(C.POINTER(C.c_double))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


class MsmContext:
    """A configured MSM evaluator with its workspace on one GPU.

    a, h: cutoff and finest grid spacing (nm); lo, hi: domain corners;
    levels: number of grids (0 = from the domain); precision: "fp32" or
    "fp64"; ke: Coulomb prefactor; max_atoms / max_systems: batch capacity;
    method: "msm", "cutoff" for the simple cutoff method at a (Section 5's
    coarse propagator) or "wolf" for Wolf summation at a with damping alpha
    (1/nm); for both h is only the cell edge of the pair search;
    smoothing: order m of the smoothing function (degree 2m), 1 .. 3;
    basis: degree p of the nodal basis, 3 or 5.
    """

    def __init__(self, a, h, lo, hi, *, levels=0, precision="fp32", ke=138.935458,
                 max_atoms=1 << 20, max_systems=1, stream=None, method="msm", smoothing=2, basis=3, alpha=0.0):
        import torch
        if method not in METHODS:
            raise ValueError(f"method must be one of {sorted(METHODS)}")
        self.method = method
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        p = _Params()
        p.a, p.h, p.levels = float(a), float(h), int(levels)
        p.precision = MSM_FP32 if precision == "fp32" else MSM_FP64
        for d in range(3):
            p.lo[d] = float(lo[d])
            p.hi[d] = float(hi[d])
        p.coulomb_k = float(ke)
        p.max_atoms = int(max_atoms)
        p.max_systems = int(max_systems)
        p.method = METHODS[method]
        p.smoothing = int(smoothing)
        p.basis = int(basis)
        p.alpha = float(alpha)
        self.smoothing, self.basis = int(smoothing), int(basis)
        self.params = p
        self.a, self.h, self.ke = float(a), float(h), float(ke)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.max_atoms, self.max_systems = int(max_atoms), int(max_systems)
        handle = C.c_void_p()
        _check(lib().msm_setup(C.byref(p), _stream_handle(stream), C.byref(handle)), "msm_setup")
        self._h = handle

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().msm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(lib().msm_set_stream(self._h, _stream_handle(stream)), "msm_set_stream")

    def status(self) -> int:
        return lib().msm_get_status(self._h)

    def check(self):
        code = self.status()
        if code != 0:
            raise MsmError(code, "device status")

    def tuning(self):
        t = _Tuning()
        _check(lib().msm_get_tuning(self._h, C.byref(t)), "msm_get_tuning")
        return _tuning_dict(t)

    def set_tuning(self, pair_waves=None, stencil_threads=None, concurrent=None, pair_cell=None):
        """Set the launch configuration (msm_set_tuning); None keeps a field."""
        cur = self.tuning()
        t = _Tuning(int(cur["pair_waves"] if pair_waves is None else pair_waves),
                    int(cur["stencil_threads"] if stencil_threads is None else stencil_threads),
                    int(cur["concurrent"] if concurrent is None else concurrent),
                    int(cur["pair_cell"] if pair_cell is None else pair_cell))
        _check(lib().msm_set_tuning(self._h, C.byref(t)), "msm_set_tuning")

    def autotune(self, xyzq, offsets=None, domains=None, reps=5):
        """Pick the fastest launch configuration on this batch (msm_autotune)."""
        self._check_xyzq(xyzq)
        n = xyzq.shape[0]
        offs = _offsets(offsets, n)
        nsys = len(offs) - 1
        dom, dom_p = _domains(domains, nsys)
        t = _Tuning()
        _check(lib().msm_autotune(self._h, nsys, offs.ctypes.data_as(C.POINTER(C.c_int64)), dom_p,
                                  C.c_void_p(xyzq.data_ptr()), int(reps), C.byref(t)), "msm_autotune")
        return _tuning_dict(t)

    def set_graphs(self, enable=True):
        """Replay captured HIP graphs for repeated evaluations (msm_set_graphs)."""
        _check(lib().msm_set_graphs(self._h, 1 if enable else 0), "msm_set_graphs")

    def enable_stage_timing(self, enable=True):
        _check(lib().msm_enable_stage_timing(self._h, 1 if enable else 0), "msm_enable_stage_timing")

    def stage_timing(self, reset=False):
        """Summed milliseconds per stage and the number of timed evaluations."""
        ms = (C.c_double * len(STAGES))()
        n = C.c_int64()
        _check(lib().msm_stage_timing(self._h, ms, C.byref(n), 1 if reset else 0), "msm_stage_timing")
        return dict(zip(STAGES, list(ms))), int(n.value)

    def grid_shape(self, domain=None):
        org = (C.c_int * (3 * MAXLEV))()
        dim = (C.c_int * (3 * MAXLEV))()
        dom = None
        if domain is not None:
            dom = (C.c_double * 6)(*[float(v) for v in domain])
        n = _check(lib().msm_grid_shape(self._h, dom, org, dim), "msm_grid_shape")
        return [(tuple(org[3 * k:3 * k + 3]), tuple(dim[3 * k:3 * k + 3])) for k in range(n)]

    # ------------------------------------------------------------------
    def _check_xyzq(self, xyzq):
        if xyzq.dtype != self.dtype or not xyzq.is_cuda or not xyzq.is_contiguous() or xyzq.dim() != 2 \
                or xyzq.shape[1] != 4:
            raise ValueError("xyzq must be a contiguous (N, 4) device tensor of the context's precision")

    def energy_forces(self, xyzq, offsets=None, domains=None, *, energy=None, forces=None, potentials=None,
                      want=("energy", "forces", "potentials")):
        """Evaluate nsys systems packed in ``xyzq`` (N x 4, contiguous, on the
        context's GPU, in its precision). ``offsets`` (nsys+1 ints) splits the
        atoms into systems (default: one system); ``domains`` (nsys x 6) gives
        per-system domains. Output tensors are allocated unless passed in;
        passed-in ones must be contiguous, on xyzq's device, of shape (nsys,)
        float64, (N, 3) and (N,) in the context's precision.
        Returns (energy[nsys] float64, forces[N,3], potentials[N])."""
        import torch
        self._check_xyzq(xyzq)
        n = xyzq.shape[0]
        offs = _offsets(offsets, n)
        nsys = len(offs) - 1
        dev = xyzq.device
        _require(energy, "energy", torch.float64, dev, (nsys,))
        _require(forces, "forces", self.dtype, dev, (n, 3))
        _require(potentials, "potentials", self.dtype, dev, (n,))
        if energy is None and "energy" in want:
            energy = torch.empty(nsys, dtype=torch.float64, device=dev)
        if forces is None and "forces" in want:
            forces = torch.empty((n, 3), dtype=self.dtype, device=dev)
        if potentials is None and "potentials" in want:
            potentials = torch.empty(n, dtype=self.dtype, device=dev)
        dom, dom_p = _domains(domains, nsys)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        rc = lib().msm_energy_forces(self._h, nsys, offs.ctypes.data_as(C.POINTER(C.c_int64)), dom_p,
                                     ptr(xyzq), ptr(energy), ptr(forces), ptr(potentials))
        _check(rc, "msm_energy_forces")
        self._last_offsets = offs.copy()
        return energy, forces, potentials

    def debug_stages(self, sys=0, domain=None):
        """Intermediate results of the last evaluation of system ``sys``
        (float64 device tensors, caller atom order)."""
        import torch
        shapes = self.grid_shape(domain)
        dev = torch.device("cuda", torch.cuda.current_device())
        # number of atoms of that system is not stored here; the caller slices
        out = {"q_grid": [], "ucut_grid": [], "u_grid": []}
        ptrs = {}
        for key in out:
            arr = (C.c_void_p * len(shapes))()
            for k, (_, dim) in enumerate(shapes):
                t = torch.zeros((dim[2], dim[1], dim[0]), dtype=torch.float64, device=dev)
                out[key].append(t)
                arr[k] = t.data_ptr()
            ptrs[key] = arr
        return out, ptrs

    def stages(self, n_sys_atoms, sys=0, domain=None):
        """Intermediate results (msm_debug_stages) of system ``sys`` of the
        last energy_forces call; ``n_sys_atoms`` must be that system's size."""
        import torch
        last = getattr(self, "_last_offsets", None)
        if last is None or not 0 <= sys < len(last) - 1:
            raise ValueError("stages: no evaluation of that system yet")
        if int(n_sys_atoms) != int(last[sys + 1] - last[sys]):
            raise ValueError(f"stages: system {sys} has {int(last[sys + 1] - last[sys])} atoms, "
                             f"not {n_sys_atoms}")
        out, ptrs = self.debug_stages(sys, domain)
        dev = out["q_grid"][0].device
        us = torch.zeros(n_sys_atoms, dtype=torch.float64, device=dev)
        fs = torch.zeros((n_sys_atoms, 3), dtype=torch.float64, device=dev)
        _check(lib().msm_debug_stages(self._h, sys, C.c_void_p(us.data_ptr()), C.c_void_p(fs.data_ptr()),
                                      ptrs["q_grid"], ptrs["ucut_grid"], ptrs["u_grid"]), "msm_debug_stages")
        torch.cuda.synchronize()
        out["u_short"] = us
        out["f_short"] = fs
        return out

    # ------------------------------------------------------------------
    # dynamics
    # ------------------------------------------------------------------
    def bind_model(self, period, molid=None, lj=None, rigid=False, tri=(0.0, 0.0, 0.0), tol=0.0):
        """Bind a molecular model (see msm_md_model): ``molid`` int32 and ``lj``
        float64 (period, 2) device tensors, or None."""
        import torch
        if molid is not None:
            _require(molid, "molid", torch.int32, molid.device, (int(period),))
            if not molid.is_cuda:
                raise ValueError("molid must be a device tensor")
        if lj is not None:
            _require(lj, "lj", torch.float64, lj.device, (int(period), 2))
            if not lj.is_cuda:
                raise ValueError("lj must be a device tensor")
        m = _Model()
        m.period = int(period)
        m.molid_dev = None if molid is None else molid.data_ptr()
        m.lj_dev = None if lj is None else lj.data_ptr()
        m.rigid_triples = 1 if rigid else 0
        for d in range(3):
            m.tri_len[d] = float(tri[d])
        m.constraint_tol = float(tol)
        self._model_refs = (molid, lj)
        _check(lib().msm_md_bind(self._h, C.byref(m)), "msm_md_bind")

    def vv_run(self, xyzq, vel, nsteps, dt, offsets=None, domains=None, energies=True):
        """Velocity Verlet in place on xyzq (N, 4) and vel (N, 4: v, 1/m),
        both float64 device tensors whatever the context's precision.
        Returns (epot, ekin) float64 tensors of length nsys, or None."""
        import torch
        for t in (xyzq, vel):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 \
                    or t.shape[1] != 4:
                raise ValueError("vv_run expects contiguous float64 (N, 4) device tensors")
        n = xyzq.shape[0]
        if vel.shape[0] != n or vel.device != xyzq.device:
            raise ValueError("xyzq and vel differ in length or device")
        offs = _offsets(offsets, n)
        nsys = len(offs) - 1
        dom, dom_p = _domains(domains, nsys)
        ep = ek = None
        if energies:
            ep = torch.empty(nsys, dtype=torch.float64, device=xyzq.device)
            ek = torch.empty(nsys, dtype=torch.float64, device=xyzq.device)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        _check(lib().msm_vv_run(self._h, nsys, offs.ctypes.data_as(C.POINTER(C.c_int64)), dom_p, ptr(xyzq),
                                ptr(vel), int(nsteps), float(dt), ptr(ep), ptr(ek)), "msm_vv_run")
        return ep, ek

    def vv_mts_run(self, xyzq, vel, nouter, ninner, dt, offsets=None, domains=None, energies=True):
        """Multiple-time-step velocity Verlet in place (see msm_vv_mts_run):
        nouter steps of dt, each with ninner short-range steps of dt/ninner.
        Same tensors as vv_run. Returns (epot, ekin) or None."""
        import torch
        for t in (xyzq, vel):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 \
                    or t.shape[1] != 4:
                raise ValueError("vv_mts_run expects contiguous float64 (N, 4) device tensors")
        n = xyzq.shape[0]
        if vel.shape[0] != n or vel.device != xyzq.device:
            raise ValueError("xyzq and vel differ in length or device")
        offs = _offsets(offsets, n)
        nsys = len(offs) - 1
        dom, dom_p = _domains(domains, nsys)
        ep = ek = None
        if energies:
            ep = torch.empty(nsys, dtype=torch.float64, device=xyzq.device)
            ek = torch.empty(nsys, dtype=torch.float64, device=xyzq.device)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        _check(lib().msm_vv_mts_run(self._h, nsys, offs.ctypes.data_as(C.POINTER(C.c_int64)), dom_p, ptr(xyzq),
                                    ptr(vel), int(nouter), int(ninner), float(dt), ptr(ep), ptr(ek)),
               "msm_vv_mts_run")
        return ep, ek


def _params(a, h, lo, hi, levels, precision, ke, max_atoms, max_systems, method, smoothing, basis, alpha):
    if method not in METHODS:
        raise ValueError(f"method must be one of {sorted(METHODS)}")
    if precision not in ("fp32", "fp64"):
        raise ValueError("precision must be 'fp32' or 'fp64'")
    p = _Params()
    p.a, p.h, p.levels = float(a), float(h), int(levels)
    p.precision = MSM_FP32 if precision == "fp32" else MSM_FP64
    for d in range(3):
        p.lo[d] = float(lo[d])
        p.hi[d] = float(hi[d])
    p.coulomb_k = float(ke)
    p.max_atoms = int(max_atoms)
    p.max_systems = int(max_systems)
    p.method = METHODS[method]
    p.smoothing = int(smoothing)
    p.basis = int(basis)
    p.alpha = float(alpha)
    return p


def energy_forces_noalloc(xyzq, a, h, lo, hi, *, levels=0, precision="fp32", ke=138.935458, method="msm",
                          smoothing=2, basis=3, alpha=0.0, energy=None, forces=None, potentials=None,
                          status=None, stream=None):
    """One evaluation of one system without a context and without device
    allocation in the library (msm_energy_forces_noalloc). Output tensors are
    allocated here unless passed in; ``status`` (one int32 on the device)
    receives the status code of the evaluation. Returns (energy[1], forces,
    potentials, status)."""
    import torch
    dtype = torch.float32 if precision == "fp32" else torch.float64
    if xyzq.dtype != dtype or not xyzq.is_cuda or not xyzq.is_contiguous() or xyzq.dim() != 2 \
            or xyzq.shape[1] != 4:
        raise ValueError("xyzq must be a contiguous (N, 4) device tensor of the given precision")
    n, dev = xyzq.shape[0], xyzq.device
    _require(energy, "energy", torch.float64, dev, (1,))
    _require(forces, "forces", dtype, dev, (n, 3))
    _require(potentials, "potentials", dtype, dev, (n,))
    _require(status, "status", torch.int32, dev, (1,))
    if energy is None:
        energy = torch.empty(1, dtype=torch.float64, device=dev)
    if forces is None:
        forces = torch.empty((n, 3), dtype=dtype, device=dev)
    if potentials is None:
        potentials = torch.empty(n, dtype=dtype, device=dev)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
    p = _params(a, h, lo, hi, levels, precision, ke, n, 1, method, smoothing, basis, alpha)
    ptr = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    _check(lib().msm_energy_forces_noalloc(C.byref(p), _stream_handle(stream), n, ptr(xyzq), ptr(energy),
                                           ptr(forces), ptr(potentials), ptr(status)),
           "msm_energy_forces_noalloc")
    return energy, forces, potentials, status


def parareal(fine, coarse, charges, invmass, state0, *, nslices, kmax, tol, steps_f, dt_f, steps_g, dt_g,
             lam=None):
    """Parareal over ``nslices`` slices (see parareal_run). ``charges``,
    ``invmass`` (natoms,) and ``state0`` (natoms, 6) are float64 device
    tensors. Returns (lambda[(nslices+1), natoms, 6], report dict, return code)."""
    import torch
    n = state0.shape[0]
    dev = state0.device
    _require(state0, "state0", torch.float64, dev, (n, 6))
    _require(charges, "charges", torch.float64, dev, (n,))
    _require(invmass, "invmass", torch.float64, dev, (n,))
    if lam is None:
        lam = torch.empty((nslices + 1, n, 6), dtype=torch.float64, device=dev)
    _require(lam, "lam", torch.float64, dev, (nslices + 1, n, 6))
    pp = _PararealParams()
    pp.nslices, pp.kmax, pp.tol = int(nslices), int(kmax), float(tol)
    pp.steps_f, pp.dt_f, pp.steps_g, pp.dt_g = int(steps_f), float(dt_f), int(steps_g), float(dt_g)
    rep = _PararealReport()
    rc = lib().parareal_run(fine._h, coarse._h, C.byref(pp), n, C.c_void_p(charges.data_ptr()),
                            C.c_void_p(invmass.data_ptr()), C.c_void_p(state0.data_ptr()),
                            C.c_void_p(lam.data_ptr()), C.byref(rep))
    _check(rc, "parareal_run")
    report = {"iterations": rep.iterations, "converged": bool(rep.converged),
              "residual": list(rep.residual[:min(rep.iterations, 64)]), "seconds": rep.seconds}
    return lam, report, rc


def parareal_window(fine, coarse, charges, invmass, lam, ring, state, *, width, tol, steps_f, dt_f, steps_g,
                    dt_g, max_iters=0, pipeline=False, chunk=0):
    """Sliding-window parareal (see parareal_window_run) in place on ``lam``
    ((nslices+1), natoms, 6; slice 0 holds the initial state), ``ring``
    (width, natoms, 6) and ``state`` (a WindowState). ``charges`` and
    ``invmass`` are (natoms,) float64 device tensors. Returns the return code:
    MSM_OK (0) when every slice is final, 1 when stopped after max_iters."""
    if lam.dim() != 3 or lam.shape[2] != 6:
        raise ValueError("parareal_window: lam must be (nslices + 1, natoms, 6)")
    n, dev, f64 = lam.shape[1], lam.device, _torch_f64()
    _require(lam, "lam", f64, dev, tuple(lam.shape))
    _require(ring, "ring", f64, dev, (width, n, 6))
    _require(charges, "charges", f64, dev, (n,))
    _require(invmass, "invmass", f64, dev, (n,))
    pp = _WindowParams()
    pp.nslices, pp.width, pp.max_iters = lam.shape[0] - 1, int(width), int(max_iters)
    pp.pipeline, pp.chunk, pp.tol = int(bool(pipeline)), int(chunk), float(tol)
    pp.steps_f, pp.dt_f, pp.steps_g, pp.dt_g = int(steps_f), float(dt_f), int(steps_g), float(dt_g)
    rc = lib().parareal_window_run(fine._h, coarse._h, C.byref(pp), n, C.c_void_p(charges.data_ptr()),
                                   C.c_void_p(invmass.data_ptr()), C.c_void_p(lam.data_ptr()),
                                   C.c_void_p(ring.data_ptr()), C.byref(state))
    return _check(rc, "parareal_window_run")


def _torch_f64():
    import torch
    return torch.float64
