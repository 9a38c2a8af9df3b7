"""Benchmark: multilevel summation energy + forces on one MI355X.

A step is one complete evaluation of the method on one batch: binning,
short-range pairs, anterpolation, restriction, lattice cutoff on every level,
top level, prolongation, interpolation, combination and the FP64 energy
reduction. The headline workload is the paper's 30 x 65 x 65 nm box of
12,675,000 water-like atoms (4,225,000 rigid 3-site molecules, TIP3P charges
and geometry, random orientations, about 100 atoms/nm^3; cutoff a = 1.2 nm,
finest spacing h = 0.25 nm, 8 grids), with positions and charges already
resident in HBM.

Prints one JSON line: atom-steps/s of the single-precision path (value), the
double-precision path beside it, the accuracy of both against the FP64 CPU
oracle on the same box, a roofline record of the dominant kernel timed live
with HIP events on the evaluation stream, the oracle's own rate on the host
cores, and secondary records (the 99,999-atom box, batches of parareal slice
states, parareal, dynamics of the large box with energy drift, orders,
multiple time steps, the sliding window).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MSM energy+force atom-steps/s at 1 GPU vs FP64 plain; parareal time-to-solution"
PEAK_FP32_VALU = 157.3    # TFLOP/s, MI355X vector FP32 (packed issue)
PEAK_FP32_UNPACKED = 78.6 # TFLOP/s: one FMA per lane and cycle, 256 CUs x 64 lanes x 2.4 GHz
PEAK_FP64_VALU = 78.6     # TFLOP/s, MI355X vector FP64
PEAK_HBM = 8000.0         # GB/s
# Flops of one unique pair inside the cutoff, counted on the Newton-3 form
# (both atoms updated), FMA = 2, the reciprocal square root = 1:
# d = r_i - r_j (3), r^2 (5), 1/r (1), rho^2 (1), gamma polynomial (4),
# g* (1), u_i and u_j (4), 1/r^3 (2), force bracket polynomial and difference
# (3), q_j b d and q_i b d into F_i and F_j (14).
FLOPS_PER_PAIR = 38


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="water_12675000")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the oracle's single-thread CPU-baseline sample")
    ap.add_argument("--no-small", action="store_true", help="skip the secondary 99,999-atom record")
    ap.add_argument("--equilibrate-ps", type=float, default=1.0,
                    help="velocity-rescaled equilibration before the energy-drift runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-slice and uneven batches")
    ap.add_argument("--no-parareal", action="store_true")
    ap.add_argument("--slices", type=int, default=32)
    ap.add_argument("--no-graphs", action="store_true", help="time eager launches only")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--tuning", default=None,
                    help="pair_waves,stencil_threads,concurrent[,pair_cell] for the headline workload instead of autotuning "
                         "(for profiler runs)")
    ap.add_argument("--no-orders", action="store_true", help="skip the smoothing-order / basis-degree study")
    ap.add_argument("--no-mts", action="store_true", help="skip the multiple-time-step dynamics")
    ap.add_argument("--no-window", action="store_true", help="skip the sliding-window parareal runs")
    ap.add_argument("--no-large", action="store_true", help="skip the 12.7M-atom slab")
    ap.add_argument("--only-fp32", action="store_true",
                    help="time only the single-system FP32 path (for profiler runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the timed steps, copy a tensor of this many MiB 5 times (a plain copy "
                         "kernel of known traffic, to calibrate the memory counters)")
    args = ap.parse_args()
    if args.only_fp32:
        args.no_fp64 = args.no_accuracy = args.no_cpu_baseline = args.no_batched = args.no_parareal = True
        args.no_large = args.no_orders = args.no_mts = args.no_window = args.no_small = True
    return args


def unique_pairs(xyz, a, chunk=1 << 20):
    """Unique atom pairs closer than a, counted exactly on the input (a k-d
    tree, every host thread)."""
    from scipy.spatial import cKDTree
    t = cKDTree(xyz)
    total = 0
    for c0 in range(0, xyz.shape[0], chunk):
        total += int(t.query_ball_point(xyz[c0:c0 + chunk], a, return_length=True, workers=-1).sum())
    return (total - xyz.shape[0]) // 2


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, family, model and
    stepping numbers, and the logical CPUs it lists."""
    fields, ncpu = {}, 0
    try:
        for line in open("/proc/cpuinfo"):
            key = line.split(":", 1)[0].strip()
            if key == "processor":
                ncpu += 1
            elif key in ("model name", "cpu family", "model", "stepping") and key not in fields:
                fields[key] = line.split(":", 1)[1].strip()
    except OSError:
        return None
    if "model name" not in fields:
        return None
    return (f"{fields['model name']} (family {fields.get('cpu family', '?')}, model {fields.get('model', '?')}, "
            f"stepping {fields.get('stepping', '?')}; {ncpu} logical CPUs listed)")


def timed_steps(torch, ctx, xyzq, out, steps, warmup):
    for _ in range(warmup):
        ctx.energy_forces(xyzq, energy=out[0], forces=out[1], potentials=out[2])
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        ctx.energy_forces(xyzq, energy=out[0], forces=out[1], potentials=out[2])
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps   # ms per step


def stage_profile(torch, ctx, xyzq, out, steps):
    ctx.stage_timing(reset=True)
    ctx.enable_stage_timing(True)
    for _ in range(steps):
        ctx.energy_forces(xyzq, energy=out[0], forces=out[1], potentials=out[2])
    ctx.enable_stage_timing(False)
    torch.cuda.synchronize()
    ms, n = ctx.stage_timing(reset=True)
    return {k: v / max(n, 1) for k, v in ms.items()}


def stencil_flops(shapes, taps):
    """2 flops per tap per node on every level below the top, all pairs on the top."""
    sizes = [d[0] * d[1] * d[2] for _, d in shapes]
    return 2.0 * taps * sum(sizes[:-1]) + 2.0 * sizes[-1] ** 2


def sphere_taps(a, h):
    R = int(np.ceil(2 * a / h)) - 1
    o = np.arange(-R, R + 1)
    X, Y, Z = np.meshgrid(o, o, o, indexing="ij")
    return int(((h * np.sqrt(X ** 2 + Y ** 2 + Z ** 2)) < 2 * a).sum())


def traffic_record(kernel_file, kernel_name, workload, form):
    """HBM bytes per launch of the kernel form ``form`` (the pair_waves value
    of the launch configuration) from committed counter summaries, if they
    were taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_name}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1309_1889_amd", "csrc", kernel_file), "rb").read()
    if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    got = rec.get("forms", {}).get(str(form))
    return None if got is None else got.get("bytes_per_launch")


def bench_batched(torch, msmx, states, q, lo, hi, steps, warmup, autotune=True):
    """One evaluation of all parareal slice states at once (the fine
    propagator's batch: the serial-fine states at the start of every slice of
    the parareal workload, each a different configuration), against one of
    them alone; and an uneven batch of 8 water boxes of 9,999 .. 200,001 atoms
    against evaluating them one by one."""
    from workloads import uneven_batch_sizes, water_box, water_box_dims
    dev = torch.device("cuda", 0)
    slices, n = states.shape[0], states.shape[1]
    xyzq = torch.empty((slices * n, 4), dtype=torch.float32, device=dev)
    xyzq.view(slices, n, 4)[:, :, :3] = states.float()
    xyzq.view(slices, n, 4)[:, :, 3] = q.float()[None, :]
    offs = np.arange(slices + 1, dtype=np.int64) * n
    ctx = msmx.MsmContext(1.2, 0.25, lo, hi, precision="fp32", max_atoms=slices * n, max_systems=slices)
    out = (torch.empty(slices, dtype=torch.float64, device=dev),
           torch.empty((slices * n, 3), dtype=torch.float32, device=dev),
           torch.empty(slices * n, dtype=torch.float32, device=dev))

    # the launch configuration is tuned on the batch itself
    tuning = ctx.autotune(xyzq, offs, reps=5) if autotune else ctx.tuning()
    # graph replays throughout, so that host launch costs do not weigh on
    # the small single systems they are compared with
    ctx.set_graphs(True)

    def run():
        ctx.energy_forces(xyzq, offs, energy=out[0], forces=out[1], potentials=out[2])

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    k = max(steps // 10, 3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(k):
        run()
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1) / k
    # the stages in turn (HIP events on the library's stream, eager launches)
    ctx.stage_timing(reset=True)
    ctx.enable_stage_timing(True)
    for _ in range(3):
        run()
    ctx.enable_stage_timing(False)
    torch.cuda.synchronize()
    sms, sn = ctx.stage_timing(reset=True)
    stage_ms = {key: round(v / max(sn, 1), 5) for key, v in sms.items()}
    # slice 0 of the batch against a single-system context with the same
    # launch configuration: identical bits; and its time per atom
    one = msmx.MsmContext(1.2, 0.25, lo, hi, precision="fp32", max_atoms=n)
    one.set_tuning(**tuning)
    one.set_graphs(True)
    x0 = xyzq[:n].contiguous()
    e_1, f_1, _ = one.energy_forces(x0)
    torch.cuda.synchronize()
    same = bool(torch.equal(f_1, out[1][:n]) and torch.equal(e_1, out[0][:1]))
    o1 = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float32, device=dev),
          torch.empty(n, dtype=torch.float32, device=dev))
    ms1 = timed_steps(torch, one, x0, o1, max(steps, 10), warmup)
    one.check()
    spread = float((states - states[:1]).abs().amax(dim=(1, 2)).max().item())
    batched = {"workload": f"{slices} parareal slice states x {n} atoms (serial fine, 20 fs apart), one call",
               "systems": slices, "atoms": slices * n, "ms_per_step": ms, "tuning": tuning,
               "value": slices * n / (ms * 1e-3), "unit": "atom-steps/s",
               "single_system_ms": ms1,
               "speedup_vs_single_system": (slices * n / (ms * 1e-3)) / (n / (ms1 * 1e-3)),
               "largest_position_change_between_states_nm": spread, "launch": "graph replay",
               "slice0_bitwise_equal_to_single": same, "stage_ms": stage_ms,
               "evaluation_over_short_stage": ms / stage_ms["short"] if stage_ms.get("short") else None}

    # uneven batch
    sizes = uneven_batch_sizes()
    ws = []
    for i, na in enumerate(sizes):
        n_mol, sites, box = water_box_dims(na)
        ws.append(water_box(n_mol, sites, box, seed=40 + i, margin=0.3).as_dtype(np.float32))
    big = np.max([x.hi - x.lo for x in ws], axis=0)
    uctx = msmx.MsmContext(1.2, 0.25, np.zeros(3), big, precision="fp32", max_atoms=sum(sizes), max_systems=8)
    uctx.set_graphs(True)
    ux = torch.tensor(np.concatenate([x.xyzq(np.float32) for x in ws]), device=dev)
    uoffs = np.cumsum([0] + sizes)
    udoms = np.array([np.concatenate([x.lo, x.hi]) for x in ws])
    # outputs allocated once: a graph replays only on the pointers it captured
    uout = (torch.empty(8, dtype=torch.float64, device=dev), torch.empty((ux.shape[0], 3), dtype=torch.float32, device=dev),
            torch.empty(ux.shape[0], dtype=torch.float32, device=dev))
    for _ in range(warmup):
        uctx.energy_forces(ux, uoffs, udoms, energy=uout[0], forces=uout[1], potentials=uout[2])
    torch.cuda.synchronize()
    e0.record()
    for _ in range(k):
        uctx.energy_forces(ux, uoffs, udoms, energy=uout[0], forces=uout[1], potentials=uout[2])
    e1.record()
    torch.cuda.synchronize()
    uctx.check()
    ums = e0.elapsed_time(e1) / k
    singles = [msmx.MsmContext(1.2, 0.25, x.lo, x.hi, precision="fp32", max_atoms=x.n) for x in ws]
    for c in singles:
        c.set_graphs(True)
    sx = [torch.tensor(x.xyzq(np.float32), device=dev) for x in ws]
    souts = [(torch.empty(1, dtype=torch.float64, device=dev), torch.empty((x.n, 3), dtype=torch.float32, device=dev),
              torch.empty(x.n, dtype=torch.float32, device=dev)) for x in ws]
    for _ in range(warmup):
        for c, x, o in zip(singles, sx, souts):
            c.energy_forces(x, energy=o[0], forces=o[1], potentials=o[2])
    torch.cuda.synchronize()
    e0.record()
    for _ in range(k):
        for c, x, o in zip(singles, sx, souts):
            c.energy_forces(x, energy=o[0], forces=o[1], potentials=o[2])
    e1.record()
    torch.cuda.synchronize()
    sms = e0.elapsed_time(e1) / k
    uneven = {"sizes": sizes, "atoms": int(sum(sizes)), "launch": "graph replay", "batched_ms": ums, "one_by_one_ms": sms,
              "batched_value": sum(sizes) / (ums * 1e-3), "speedup_batched_vs_one_by_one": sms / ums}
    return batched, uneven


def bench_parareal(torch, msmx, slices, n_atoms=99999):
    """Parareal time-to-solution (Section 4) on the water box: `slices` slices
    of 10 velocity-Verlet steps of 2 fs with the fine MSM (a = 1.2, h = 0.25)
    against serial fine on the same GPU, for the configured coarse propagator
    (one 20 fs step with a = 0.8, h = 0.5), a stable MSM one (10 steps of 2 fs
    with a = 0.8, h = 0.5), the paper's choice, the simple cutoff method at
    1.2 nm with 10 steps of 2 fs, and Wolf summation with the same cutoff."""
    from workloads import rigid_water_velocities, water_box, water_box_dims, water_model_arrays
    dev = torch.device("cuda", 0)
    n_mol, sites, box = water_box_dims(n_atoms)
    # the lattice start heats up and surface molecules evaporate at ~2 nm/ps:
    # a 3 nm margin keeps every atom inside the domain over the 640 fs
    w = water_box(n_mol, sites, box, seed=4, margin=3.0)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=104)
    xyz = w.xyz
    mol_t = torch.tensor(molid, dtype=torch.int32, device=dev)
    lj_t = torch.tensor(lj, dtype=torch.float64, device=dev)

    def ctx(a, h, ma, ms, method="msm", alpha=0.0):
        c = msmx.MsmContext(a, h, w.lo, w.hi, precision="fp32", max_atoms=ma, max_systems=ms, method=method,
                            alpha=alpha)
        c.bind_model(w.n, mol_t, lj_t, rigid=True, tri=tri)
        c.set_graphs(True)
        return c

    fine = ctx(1.2, 0.25, slices * w.n, slices)
    q = torch.tensor(w.q, device=dev)
    invm = torch.tensor(1.0 / mass, device=dev)
    s0 = torch.tensor(np.concatenate([xyz, v], 1), device=dev).contiguous()
    # serial fine on the same GPU: 10 steps per slice, each slice restarting from the stored state
    serial = ctx(1.2, 0.25, w.n, 1)
    x = torch.cat([s0[:, :3], q[:, None]], 1).contiguous()
    vv = torch.cat([s0[:, 3:], invm[:, None]], 1).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(slices):
        serial.vv_run(x, vv, 10, 0.002, energies=False)
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - t0
    serial.check()
    # the state at the start of every slice (for the batched evaluation leg)
    states = torch.empty((slices, w.n, 3), dtype=torch.float64, device=dev)
    xs, vs = torch.cat([s0[:, :3], q[:, None]], 1).contiguous(), vv.clone()
    vs.copy_(torch.cat([s0[:, 3:], invm[:, None]], 1))
    for k in range(slices):
        states[k] = xs[:, :3]
        serial.vv_run(xs, vs, 10, 0.002, energies=False)
    torch.cuda.synchronize()
    assert torch.equal(xs, x)   # the same serial trajectory
    out = {"workload": f"{slices} slices x {w.n} atoms, rigid water at 300 K, fine 10 x 2 fs (a 1.2, h 0.25)",
           "serial_fine_seconds": serial_s}
    # coarse propagators: the configured one (MSM, one 20 fs step), a stable MSM
    # one, the paper's choice, the simple cutoff method at 1.2 nm with the fine
    # step (Section 5), and its refinement, Wolf summation (alpha 2 / nm)
    variants = (("coarse_1x20fs", "msm", 0.8, 0.5, 1, 0.020, "MSM a 0.8, h 0.5"),
                ("coarse_10x2fs", "msm", 0.8, 0.5, 10, 0.002, "MSM a 0.8, h 0.5"),
                ("coarse_cutoff_10x2fs", "cutoff", 1.2, 0.25, 10, 0.002, "simple cutoff 1.2 nm"),
                ("coarse_wolf_10x2fs", "wolf", 1.2, 0.25, 10, 0.002, "Wolf summation 1.2 nm, alpha 2 / nm"))
    for name, method, a, h, sg, dtg, desc in variants:
        coarse = ctx(a, h, w.n, 1, method, alpha=2.0 if method == "wolf" else 0.0)
        # the coarse propagator's launch configuration (incl. its pair cells)
        # tuned on the start state; the fine one keeps the default that the
        # serial reference shares
        rec = {"coarse": f"{sg} x {dtg * 1000:g} fs, {desc}",
               "coarse_tuning": coarse.autotune(x.to(torch.float32).contiguous(), reps=3)}
        # cost of one coarse step against one fine step on one slice
        xg, vg = x.clone(), vv.clone()
        coarse.vv_run(xg, vg, 2, dtg, energies=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        coarse.vv_run(xg, vg, 20, dtg, energies=False)
        torch.cuda.synchronize()
        rec["coarse_step_ms"] = (time.perf_counter() - t1) / 20 * 1e3
        st = coarse.status()     # reads and clears the status word
        if st:
            rec["coarse_alone_22_steps"] = msmx.status_string(st)
        try:
            lam, rep, rc = msmx.parareal(fine, coarse, q, invm, s0, nslices=slices, kmax=slices, tol=1e-4,
                                         steps_f=10, dt_f=0.002, steps_g=sg, dt_g=dtg)
            rec.update({"status": "converged" if rc == 0 else "not converged", "iterations": rep["iterations"],
                        "seconds": rep["seconds"], "residual_nm": [float("%.3g" % r) for r in rep["residual"]],
                        "speedup_vs_serial_fine": serial_s / rep["seconds"]})
            last = lam[slices, :, :3]
            rec["final_max_dev_vs_serial_nm"] = float((last - x[:, :3]).abs().max().item())
        except msmx.MsmError as e:
            rec.update({"status": f"failed: {e}"})
        out[name] = rec
        del coarse
    out["fine_step_ms"] = serial_s / (slices * 10) * 1e3
    return out, (states, q, w.lo, w.hi)


def exact_coulomb_rows(xyz, q, sel, ke=138.935458, chunk=64):
    """Exact Coulomb potentials and forces of the atoms in `sel` (direct FP64
    sums over all atoms, in NumPy): the reference of the order study."""
    pot = np.zeros(len(sel))
    f = np.zeros((len(sel), 3))
    for c0 in range(0, len(sel), chunk):
        idx = sel[c0:c0 + chunk]
        d = xyz[idx][:, None, :] - xyz[None, :, :]
        r2 = (d ** 2).sum(-1)
        r2[np.arange(len(idx)), idx] = np.inf
        rinv = 1.0 / np.sqrt(r2)
        pot[c0:c0 + chunk] = ke * (rinv * q[None, :]).sum(1)
        f[c0:c0 + chunk] = ke * q[idx][:, None] * ((q[None, :] * rinv ** 3)[..., None] * d).sum(1)
    return pot, f


def bench_orders(torch, msmx, w32, steps=20, warmup=3):
    """Accuracy and cost of the smoothing order m and basis degree p (Section
    3 names the trade-off): FP32 evaluation time of the water box and the
    relative force and potential RMS error against exact Coulomb on 256
    sampled atoms."""
    dev = torch.device("cuda", 0)
    n = w32.n
    x = torch.tensor(w32.xyzq(np.float32), device=dev)
    out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.float32, device=dev))
    sel = np.sort(np.random.default_rng(81).choice(n, 256, replace=False))
    pot_ex, f_ex = exact_coulomb_rows(w32.xyz.astype(np.float64), w32.q.astype(np.float64), sel)
    rec = []
    for m, p in ((2, 3), (1, 3), (3, 3), (2, 5), (3, 5)):
        ctx = msmx.MsmContext(w32.a, w32.h, w32.lo, w32.hi, precision="fp32", max_atoms=n, smoothing=m, basis=p)
        ms = timed_steps(torch, ctx, x, out, steps, warmup)
        ctx.check()
        f = out[1].double().cpu().numpy()[sel]
        pt = out[2].double().cpu().numpy()[sel]
        rec.append({"smoothing_m": m, "basis_p": p, "ms_per_eval": ms,
                    "force_rel_rms_vs_exact": float(np.sqrt(((f - f_ex) ** 2).sum() / (f_ex ** 2).sum())),
                    "potential_rel_rms_vs_exact": float(np.sqrt(((pt - pot_ex) ** 2).sum() / (pot_ex ** 2).sum()))})
        del ctx
    return {"workload": f"{n} atoms (water box), a {w32.a} nm, h {w32.h} nm, FP32; error on 256 sampled atoms",
            "variants": rec}


def bench_window(torch, msmx, slices=50, width=5, tol=1e-4, n_atoms=99999):
    """Sliding-window parareal (Section 4's example: a 1 ps run with a 100 fs
    window) on the water box: `slices` slices of 10 velocity-Verlet steps of
    2 fs with the fine MSM (a = 1.2, h = 0.25), a window of `width` slices,
    states accepted below `tol` nm; plain (one fine batch, then the coarse
    sweep) and pipelined (fine batches on their own stream as soon as the
    sweep has produced their states), against serial fine on the same GPU."""
    from workloads import rigid_water_velocities, water_box, water_box_dims, water_model_arrays
    dev = torch.device("cuda", 0)
    n_mol, sites, box = water_box_dims(n_atoms)
    w = water_box(n_mol, sites, box, seed=4, margin=3.0)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=104)
    mol_t = torch.tensor(molid, dtype=torch.int32, device=dev)
    lj_t = torch.tensor(lj, dtype=torch.float64, device=dev)

    def ctx(a, h, ma, ms, method="msm", graphs=True, stream=None):
        c = msmx.MsmContext(a, h, w.lo, w.hi, precision="fp32", max_atoms=ma, max_systems=ms, method=method)
        c.bind_model(w.n, mol_t, lj_t, rigid=True, tri=tri)
        c.set_graphs(graphs)
        if stream is not None:
            c.set_stream(stream)
        return c

    q = torch.tensor(w.q, device=dev)
    invm = torch.tensor(1.0 / mass, device=dev)
    s0 = torch.tensor(np.concatenate([w.xyz, v], 1), device=dev).contiguous()
    serial = ctx(1.2, 0.25, w.n, 1)
    x = torch.cat([s0[:, :3], q[:, None]], 1).contiguous()
    vv = torch.cat([s0[:, 3:], invm[:, None]], 1).contiguous()
    serial.vv_run(x.clone(), vv.clone(), 2, 0.002, energies=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    serial.vv_run(x, vv, 10 * slices, 0.002, energies=False)
    torch.cuda.synchronize()
    serial_s = time.perf_counter() - t0
    serial.check()
    out = {"workload": f"{slices} slices x 10 x 2 fs ({slices * 20} fs), window {width} slices ({width * 20} fs), "
                       f"{w.n} atoms, rigid water at 300 K, fine MSM a 1.2 h 0.25, tolerance {tol:g} nm",
           "serial_fine_seconds": serial_s}
    side = torch.cuda.Stream()
    for name, method, a, h, desc in (("coarse_cutoff_10x2fs", "cutoff", 1.2, 0.25, "simple cutoff 1.2 nm"),
                                     ("coarse_msm_10x2fs", "msm", 0.8, 0.5, "MSM a 0.8, h 0.5")):
        coarse = ctx(a, h, w.n, 1, method)
        rec = {"coarse": f"10 x 2 fs, {desc}",
               "coarse_tuning": coarse.autotune(torch.cat([s0[:, :3], q[:, None]], 1).to(torch.float32).contiguous(),
                                                reps=3)}
        for mode, pipe in (("plain", False), ("pipelined", True)):
            fine = ctx(1.2, 0.25, width * w.n, width, graphs=False, stream=side if pipe else None)
            lam = torch.zeros((slices + 1, w.n, 6), dtype=torch.float64, device=dev)
            lam[0] = s0
            ring = torch.zeros((width, w.n, 6), dtype=torch.float64, device=dev)
            st = msmx.WindowState()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            try:
                msmx.parareal_window(fine, coarse, q, invm, lam, ring, st, width=width, tol=tol, steps_f=10,
                                     dt_f=0.002, steps_g=10, dt_g=0.002, pipeline=pipe)
                secs = time.perf_counter() - t1
                rec[mode] = {"seconds": secs, "iterations": st.iterations, "fine_slice_runs": st.fine_slices,
                             "coarse_slice_runs": st.coarse_slices, "speedup_vs_serial_fine": serial_s / secs,
                             "final_max_dev_vs_serial_nm": float((lam[slices, :, :3] - x[:, :3]).abs().max()),
                             "final_rms_dev_vs_serial_nm": float((lam[slices, :, :3] - x[:, :3]).pow(2).sum(1)
                                                                 .mean().sqrt())}
            except msmx.MsmError as e:
                rec[mode] = {"status": f"failed: {e}"}
            del fine, lam, ring
        out[name] = rec
        del coarse
    return out


KB = 8.314462618e-3   # kJ/(mol K)


def rigid_dof(n_atoms):
    """Degrees of freedom of rigid 3-site molecules with the total momentum removed."""
    return 6 * (n_atoms // 3) - 3


def equilibrate(torch, ctx, x, vel, ps, dt=0.002, temperature=300.0, every=10):
    """Velocity Verlet with the velocities rescaled to `temperature` every
    `every` steps (uniform scaling keeps the rigid constraints), for `ps`
    picoseconds. Returns the temperatures seen before each rescaling."""
    dof = rigid_dof(x.shape[0])
    temps = []
    for _ in range(max(int(round(ps / (dt * every))), 0)):
        _, ek = ctx.vv_run(x, vel, every, dt)
        t = 2.0 * ek.item() / (dof * KB)
        temps.append(t)
        vel[:, :3] *= float(np.sqrt(temperature / t))
    torch.cuda.synchronize()
    return temps


def nve_series(torch, ctx, x, vel, nsteps, dt, chunk):
    """Total energy after every `chunk` steps of plain velocity Verlet."""
    ep, ek = ctx.vv_run(x, vel, 0, dt)
    es, ks = [ep.item() + ek.item()], [ek.item()]
    for _ in range(nsteps // chunk):
        ep, ek = ctx.vv_run(x, vel, chunk, dt)
        es.append(ep.item() + ek.item())
        ks.append(ek.item())
    return np.array(es), np.array(ks)


def drift_record(es, ks, dt, chunk, n_atoms):
    """Drift (slope of a least-squares line through E(t)) per ps and per
    degree of freedom, the RMS fluctuation about that line, and the start and
    end temperatures."""
    dof = rigid_dof(n_atoms)
    t = np.arange(len(es)) * chunk * dt
    slope, icept = np.polyfit(t, es, 1)
    resid = es - (slope * t + icept)
    return {"dt_fs": dt * 1000, "steps": int((len(es) - 1) * chunk), "ps": float(t[-1]),
            "drift_kj_mol_per_ps_per_dof": float(slope / dof),
            "drift_relative_to_kinetic_per_ps": float(slope / ks.mean()),
            "energy_change_relative_to_kinetic": float((es[-1] - es[0]) / ks.mean()),
            "rms_fluctuation_kj_mol_per_dof": float(np.sqrt((resid ** 2).mean()) / dof),
            "temperature_start_k": float(2 * ks[0] / (dof * KB)), "temperature_end_k": float(2 * ks[-1] / (dof * KB))}


def dt_halving(torch, ctx, x, vel, ps, dt, chunk_ps=0.02):
    """The same NVE stretch from the same equilibrated state with dt and
    dt/2: velocity Verlet is second order, so the energy fluctuation (and a
    drift that the integrator causes) should shrink about 4 times."""
    rec = {}
    for name, d in (("dt", dt), ("dt_half", dt / 2)):
        xs, vs = x.clone(), vel.clone()
        steps = int(round(ps / d))
        chunk = max(int(round(chunk_ps / d)), 1)
        es, ks = nve_series(torch, ctx, xs, vs, steps, d, chunk)
        rec[name] = drift_record(es, ks, d, chunk, x.shape[0])
        del xs, vs
    rec["fluctuation_ratio"] = rec["dt"]["rms_fluctuation_kj_mol_per_dof"] / rec["dt_half"]["rms_fluctuation_kj_mol_per_dof"]
    rec["drift_ratio"] = rec["dt"]["drift_kj_mol_per_ps_per_dof"] / rec["dt_half"]["drift_kj_mol_per_ps_per_dof"]
    return rec


def bench_dt_halving(torch, msmx, equilibrate_ps=1.0, ps=0.4):
    """Second order of velocity Verlet on the GPU path: a 2,997-atom rigid
    water box in FP64 (so that the integrator's error, not the rounding of
    single-precision forces, sets the energy fluctuation), equilibrated at
    300 K, then the same NVE stretch with dt = 2 fs and 1 fs."""
    from workloads import rigid_water_velocities, water_box, water_model_arrays
    dev = torch.device("cuda", 0)
    w = water_box(999, (10, 10, 10), (3.1, 3.1, 3.1), seed=61, margin=1.5)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=62)
    c = msmx.MsmContext(1.0, 0.25, w.lo, w.hi, precision="fp64", max_atoms=w.n)
    c.bind_model(w.n, torch.tensor(molid, dtype=torch.int32, device=dev), torch.tensor(lj, device=dev), rigid=True,
                 tri=tri)
    c.set_graphs(True)
    x = torch.tensor(np.concatenate([w.xyz, w.q[:, None]], 1), device=dev).contiguous()
    vel = torch.tensor(np.concatenate([v, 1.0 / mass[:, None]], 1), device=dev).contiguous()
    temps = equilibrate(torch, c, x, vel, equilibrate_ps, 0.002)
    rec = dt_halving(torch, c, x, vel, ps, 0.002, chunk_ps=0.01)
    c.check()
    return {"workload": f"{w.n} atoms, rigid water, a 1.0 nm, h 0.25 nm, FP64; {ps:g} ps NVE after "
                        f"{equilibrate_ps:g} ps rescaled to 300 K", "equilibration_temperature_k":
            [round(t, 1) for t in temps[::10]], **rec}


def bench_mts(torch, msmx, inner_steps=100, dt_inner=0.002, equilibrate_ps=1.0):
    """Multiple time steps on the 99,999-atom water box (rigid water at 300 K,
    FP32 forces): the grid part every 1 (plain velocity Verlet), 2 and 4
    inner steps of 2 fs; time per inner step and total-energy drift."""
    from workloads import rigid_water_velocities, water_box, water_box_dims, water_model_arrays
    dev = torch.device("cuda", 0)
    n_mol, sites, box = water_box_dims(99999)
    w = water_box(n_mol, sites, box, seed=4, margin=3.0)
    mass, molid, lj, tri = water_model_arrays(w.n)
    v = rigid_water_velocities(w.xyz, 300.0, seed=104)
    c = msmx.MsmContext(1.2, 0.25, w.lo, w.hi, precision="fp32", max_atoms=w.n)
    c.bind_model(w.n, torch.tensor(molid, dtype=torch.int32, device=dev), torch.tensor(lj, device=dev), rigid=True,
                 tri=tri)
    c.set_graphs(True)
    # start every variant from one state equilibrated at 300 K
    x0 = torch.tensor(np.concatenate([w.xyz, w.q[:, None]], 1), device=dev).contiguous()
    v0 = torch.tensor(np.concatenate([v, 1.0 / mass[:, None]], 1), device=dev).contiguous()
    temps = equilibrate(torch, c, x0, v0, equilibrate_ps, dt_inner)
    rec = []
    for ninner in (1, 2, 4):
        x, vv = x0.clone(), v0.clone()
        dt = dt_inner * ninner
        c.vv_mts_run(x.clone(), vv.clone(), 2, ninner, dt, energies=False)   # warm-up, graphs captured
        ep0, ek0 = c.vv_mts_run(x, vv, 0, ninner, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ep1, ek1 = c.vv_mts_run(x, vv, inner_steps // ninner, ninner, dt)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        c.check()
        e0, e1 = ep0.item() + ek0.item(), ep1.item() + ek1.item()
        dof = rigid_dof(w.n)
        ps = inner_steps * dt_inner
        rec.append({"grid_every_inner_steps": ninner, "dt_outer_fs": dt * 1000, "inner_steps": inner_steps,
                    "ms_per_inner_step": secs / inner_steps * 1e3,
                    "drift_kj_mol_per_ps_per_dof": (e1 - e0) / ps / dof,
                    "drift_relative_to_kinetic": (e1 - e0) / ek0.item(),
                    "temperature_start_k": 2 * ek0.item() / (dof * KB),
                    "temperature_end_k": 2 * ek1.item() / (dof * KB)})
    return {"workload": f"{w.n} atoms, rigid water, a 1.2 nm, h 0.25 nm, FP32 forces, inner step "
                        f"{dt_inner * 1000:g} fs; every variant starts from one state after "
                        f"{equilibrate_ps:g} ps of velocity Verlet rescaled to 300 K",
            "equilibration_temperature_k": [round(t, 1) for t in temps[::10]], "variants": rec}


def bench_large(torch, msmx, w64, steps=100, dt=0.002, equilibrate_ps=1.0):
    """Dynamics of the paper's 30 x 65 x 65 nm box (12,675,000 water-like
    atoms, rigid water model, FP32 forces, FP64 state): velocity-Verlet step
    rate, then the energy drift over `steps` steps of dt from a state
    equilibrated at 300 K, and the same stretch at dt/2."""
    from workloads import rigid_water_velocities, water_model_arrays
    dev = torch.device("cuda", 0)
    w = w64.as_dtype(np.float32)
    n = w.n
    mass, molid, lj, tri = water_model_arrays(n)
    v = rigid_water_velocities(w64.xyz, 300.0, seed=105)
    md = msmx.MsmContext(w.a, w.h, w.lo, w.hi, precision="fp32", max_atoms=n)
    md.bind_model(n, torch.tensor(molid, dtype=torch.int32, device=dev), torch.tensor(lj, device=dev), rigid=True,
                  tri=tri)
    md.set_graphs(True)
    x = torch.tensor(np.concatenate([w64.xyz, w64.q[:, None]], 1), device=dev).contiguous()
    vel = torch.tensor(np.concatenate([v, 1.0 / mass[:, None]], 1), device=dev).contiguous()
    del v
    temps = equilibrate(torch, md, x, vel, equilibrate_ps, dt)
    md.check()
    # step rate (graphs captured in the equilibration)
    xs, vs = x.clone(), vel.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    md.vv_run(xs, vs, steps, dt, energies=False)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    md.check()
    del xs, vs
    halving = dt_halving(torch, md, x, vel, steps * dt, dt)
    md.check()
    return {"workload": f"{n} atoms, 30x65x65 nm rigid water, a 1.2 nm, h 0.25 nm, {len(md.grid_shape())} grids, "
                        f"FP32 forces, FP64 state; drift from a state after {equilibrate_ps:g} ps of velocity "
                        f"Verlet rescaled to 300 K",
            "vv_steps": steps, "dt_ps": dt, "vv_seconds": secs, "vv_ms_per_step": secs / steps * 1e3,
            "vv_atom_steps_per_s": n * steps / secs,
            "equilibration_temperature_k": [round(t, 1) for t in temps[::5]],
            "drift": halving["dt"], "drift_dt_half": halving["dt_half"],
            "fluctuation_ratio_dt_vs_half": halving["fluctuation_ratio"],
            "drift_ratio_dt_vs_half": halving["drift_ratio"]}


def log(msg):
    """Progress of the legs on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def big_workload(w):
    return w.n > 2_000_000


def single_fp32(torch, msmx, w32, args, reps):
    """The single-system FP32 path: default launch configuration, then the
    autotuned one eagerly and as a graph replay; stage times in turn."""
    dev = torch.device("cuda", 0)
    n = w32.n
    ctx = msmx.MsmContext(w32.a, w32.h, w32.lo, w32.hi, precision="fp32", max_atoms=n)
    x32 = torch.tensor(w32.xyzq(np.float32), device=dev)
    out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.float32, device=dev))
    eager_default_ms = timed_steps(torch, ctx, x32, out, args.steps, args.warmup)
    if args.tuning and big_workload(w32):
        vals = [int(v) for v in args.tuning.split(",")]
        pw, st, cc = vals[:3]
        ctx.set_tuning(pair_waves=pw, stencil_threads=st, concurrent=cc, pair_cell=vals[3] if len(vals) > 3 else 1)
        tuning = ctx.tuning()
    else:
        tuning = ctx.autotune(x32, reps=reps) if not args.no_autotune else ctx.tuning()
    graph_ms = None
    if not args.no_graphs:
        ctx.set_graphs(True)
        graph_ms = timed_steps(torch, ctx, x32, out, args.steps, args.warmup)
        ctx.check()
        ctx.set_graphs(False)
    eager_tuned_ms = timed_steps(torch, ctx, x32, out, args.steps, args.warmup)
    stages = stage_profile(torch, ctx, x32, out, max(args.steps // 2, 3))
    ctx.check()
    # the headline uses the faster of the two launch modes; both are reported
    mode = "graph" if graph_ms is not None and graph_ms < eager_tuned_ms else "eager"
    ms = graph_ms if mode == "graph" else eager_tuned_ms
    launch = {"mode": mode, "tuning": tuning, "graph_ms_per_step": graph_ms,
              "eager_default_ms_per_step": eager_default_ms, "eager_tuned_ms_per_step": eager_tuned_ms}
    return ms, stages, launch, ctx, x32, out


def single_fp64(torch, msmx, w32, args, reps):
    dev = torch.device("cuda", 0)
    n = w32.n
    ctx64 = msmx.MsmContext(w32.a, w32.h, w32.lo, w32.hi, precision="fp64", max_atoms=n)
    x64 = torch.tensor(w32.xyzq(np.float64), device=dev)
    out64 = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
             torch.empty(n, dtype=torch.float64, device=dev))
    tuning64 = ctx64.autotune(x64, reps=reps) if not args.no_autotune else ctx64.tuning()
    k = max(args.steps // 4, 3)
    ms64 = timed_steps(torch, ctx64, x64, out64, k, max(args.warmup // 2, 1))
    if not args.no_graphs:
        ctx64.set_graphs(True)
        ms64 = min(ms64, timed_steps(torch, ctx64, x64, out64, k, max(args.warmup // 2, 1)))
        ctx64.check()
        ctx64.set_graphs(False)
    stages64 = stage_profile(torch, ctx64, x64, out64, k)
    ctx64.check()
    rec = {"value": n / (ms64 * 1e-3), "ms_per_step": ms64, "tuning": tuning64,
           "stage_ms": {k_: round(v, 5) for k_, v in stages64.items()}}
    del ctx64, x64
    return rec, out64


def composite_roofline(n, pairs, shapes, taps, ms_eval, elem=4):
    """The whole evaluation against its roofline: t_roof = sum over the stages
    of max(algorithmic flops / FP32 VALU peak, algorithmic bytes / HBM peak),
    over the measured evaluation time. Flops: 38 per unique pair; 2 per
    stencil tap and node plus the top level's all pairs; anterpolation 2 per
    node-atom pair plus 12 evaluations of the cubic basis (7 flops each) per
    atom; interpolation 8 per node-atom pair (value and gradient) plus 24 basis
    and derivative evaluations. Bytes: atoms in and out of each stage, every
    grid node read and written once per transfer."""
    m = [d[0] * d[1] * d[2] for _, d in shapes]
    m0, mk = m[0], sum(m[1:])
    peak_f, peak_b = PEAK_FP32_VALU * 1e12, PEAK_HBM * 1e9
    terms = {
        "bin": (0.0, n * (16 + 16 + 12) + 8.0 * m0),
        "short": (FLOPS_PER_PAIR * pairs, n * 32.0),
        "anterp": (n * (2 * 64 + 12 * 7.0), n * 16.0 + m0 * elem),
        "restrict": (0.0, 2.0 * mk * elem + m0 * elem),
        "cutoff": (stencil_flops(shapes, taps), 2.0 * sum(m) * elem),
        "prolong": (0.0, 2.0 * mk * elem + m0 * elem),
        "interp": (n * (8 * 64 + 24 * 7.0), n * 16.0 + m0 * elem + n * 16.0),
    }
    t = {k: max(f / peak_f, b / peak_b) * 1e3 for k, (f, b) in terms.items()}
    t_roof = sum(t.values())
    return {"t_roof_ms": round(t_roof, 5), "t_measured_ms": round(ms_eval, 5), "frac": round(t_roof / ms_eval, 4),
            "peaks": {"fp32_valu_tflops": PEAK_FP32_VALU, "hbm_gbs": PEAK_HBM},
            "terms_ms": {k: round(v, 5) for k, v in t.items()}}


def roofline_of(stages, pairs, shapes, taps, form, workload):
    """Per-stage records and the roofline of the dominant kernel (algorithmic
    flops over the stage's HIP-event time)."""
    work = {"short": FLOPS_PER_PAIR * pairs, "cutoff": stencil_flops(shapes, taps)}
    dominant = max(stages, key=stages.get)
    kernels = {}
    for st, ms in stages.items():
        rec = {"ms": round(ms, 5)}
        if st in work:
            rec["tflops"] = round(work[st] / (ms * 1e-3) / 1e12, 3)
            rec["frac_fp32_valu"] = round(work[st] / (ms * 1e-3) / 1e12 / PEAK_FP32_VALU, 4)
        kernels[st] = rec
    if dominant in work:
        achieved = work[dominant] / (stages[dominant] * 1e-3) / 1e12
        kname = {"short": "pair_short", "cutoff": "stencil"}[dominant]
        roofline = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU, 4),
                    # the published peak counts packed FP32; this code is built without it
                    "peak_unpacked_fp32": PEAK_FP32_UNPACKED,
                    "frac_of_unpacked": round(achieved / PEAK_FP32_UNPACKED, 4),
                    "traffic": traffic_record("pair.hip", kname, workload, form) if dominant == "short" else None,
                    "algorithmic_flops_per_launch": float(work[dominant]), "kernel_ms": round(stages[dominant], 5),
                    "unique_pairs": int(pairs), "flops_per_pair": FLOPS_PER_PAIR, "stencil_taps": taps}
    else:
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": None, "peak": PEAK_HBM, "unit": "GB/s",
                    "frac": None, "traffic": None}
    return roofline, kernels


def rel_rms(x, ref):
    return float(np.sqrt(((x - ref) ** 2).sum() / (ref ** 2).sum()))


def small_box_record(torch, msmx, args):
    """The 99,999-atom water box (10 nm cube, 5 grids): FP32 and FP64 single
    evaluations, the pair kernel's roofline there, and the accuracy against
    the oracle."""
    from workloads import named
    w32 = named("water_99999").as_dtype(np.float32)
    ms32, stages32, launch, ctx, x32, out32 = single_fp32(torch, msmx, w32, args, 5)
    pairs = unique_pairs(w32.xyz, w32.a)
    roofline, kernels = roofline_of(stages32, pairs, ctx.grid_shape(), sphere_taps(w32.a, w32.h),
                                    ctx.tuning()["pair_waves"], "water_99999")
    rec = {"workload": f"water_99999: {w32.n} atoms, 10 nm cube, a 1.2 nm, h 0.25 nm, 5 grids",
           "fp32_ms_per_step": ms32, "fp32_value": w32.n / (ms32 * 1e-3), "launch": launch,
           "roofline": roofline, "stage_ms": kernels,
           "composite_roofline": composite_roofline(w32.n, pairs, ctx.grid_shape(), sphere_taps(w32.a, w32.h), ms32)}
    fp64, out64 = (None, None) if args.no_fp64 else single_fp64(torch, msmx, w32, args, 5)
    rec["fp64_plain"] = fp64
    if fp64:
        rec["speedup_fp32_vs_fp64_plain"] = rec["fp32_value"] / fp64["value"]
    if not args.no_accuracy:
        import oracle
        eo, fo, po = oracle.msm(oracle.OracleParams.of(w32), w32.xyz, w32.q)
        rec["accuracy"] = {"fp32_force_rel_rms": rel_rms(out32[1].double().cpu().numpy(), fo),
                           "fp32_energy_rel": abs(out32[0].item() - eo) / abs(eo)}
        if out64 is not None:
            rec["accuracy"]["fp64_force_rel_rms"] = rel_rms(out64[1].cpu().numpy(), fo)
            rec["accuracy"]["fp64_energy_rel"] = abs(out64[0].item() - eo) / abs(eo)
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1 (the multi-GPU "
                                   "sharding is a design in the documentation, not code)"}))
        sys.exit(2)

    import torch
    import paper_1309_1889_amd as msmx
    from workloads import named

    w64 = named(args.workload)
    w32 = w64.as_dtype(np.float32)
    n = w32.n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    big = big_workload(w32)
    log(f"{args.workload}: {n} atoms")

    result = {"metric": METRIC}
    # ---- single-precision path (the headline) ----
    ms32, stages32, launch, ctx, x32, out32 = single_fp32(torch, msmx, w32, args, 2 if big else 5)
    value = n / (ms32 * 1e-3)
    shapes = ctx.grid_shape()
    form = ctx.tuning()["pair_waves"]
    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    del ctx, x32
    log(f"fp32 {ms32:.4f} ms per evaluation")

    # ---- double-precision plain path on the same box ----
    fp64, out64 = (None, None) if args.no_fp64 else single_fp64(torch, msmx, w32, args, 2 if big else 5)
    if fp64:
        log(f"fp64 {fp64['ms_per_step']:.4f} ms per evaluation")

    # ---- roofline of the dominant kernel (timed live, HIP events on the context stream) ----
    pairs = unique_pairs(w32.xyz, w32.a)
    roofline, kernels = roofline_of(stages32, pairs, shapes, sphere_taps(w32.a, w32.h), form, args.workload)
    log(f"{pairs} unique pairs inside the cutoff")

    # ---- accuracy against the FP64 oracle; the oracle as the CPU baseline ----
    accuracy = None
    cpu = None
    if not (args.no_accuracy and args.no_cpu_baseline):
        import oracle
        threads = oracle.threads()
        t0 = time.perf_counter()
        eo, fo, po = oracle.msm(oracle.OracleParams.of(w32), w32.xyz, w32.q)
        t_all = time.perf_counter() - t0
        log(f"oracle on {threads} threads: {t_all:.1f} s")
        if not args.no_accuracy:
            accuracy = {"fp32_force_rel_rms": rel_rms(out32[1].double().cpu().numpy(), fo),
                        "fp32_potential_rel_rms": rel_rms(out32[2].double().cpu().numpy(), po),
                        "fp32_energy_rel": abs(out32[0].item() - eo) / abs(eo), "oracle_energy": eo}
            if out64 is not None:
                accuracy["fp64_force_rel_rms"] = rel_rms(out64[1].cpu().numpy(), fo)
                accuracy["fp64_potential_rel_rms"] = rel_rms(out64[2].cpu().numpy(), po)
                accuracy["fp64_energy_rel"] = abs(out64[0].item() - eo) / abs(eo)
        del fo, po
        if not args.no_cpu_baseline:
            # one thread on a 10 nm cube cut from the same box (about as many
            # atoms as the 99,999-atom workload), repeated up to the bound
            sel = np.all((w32.xyz >= 0.0) & (w32.xyz < 10.0), axis=1)
            sub = w32.xyz[sel]
            p1 = oracle.OracleParams(w32.a, w32.h, (0.0, 0.0, 0.0), (10.0, 10.0, 10.0), 0, 138.935458)
            oracle.set_threads(1)
            t1 = time.perf_counter()
            ev = 0
            while ev == 0 or time.perf_counter() - t1 < args.cpu_seconds:
                oracle.msm(p1, sub, w32.q[sel])
                ev += 1
            t_one = time.perf_counter() - t1
            oracle.set_threads(threads)
            cpu = {"value": n / t_all, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
                   "sample": f"one full FP64 oracle evaluation of the same {n}-atom box on {threads} threads "
                             f"({t_all:.1f} s; it is also the accuracy reference)",
                   "single_thread": {"value": int(sel.sum()) * ev / t_one, "unit": "atom-steps/s", "cores": 1,
                                     "sample": f"{ev} oracle evaluation(s) of the {int(sel.sum())} atoms of a "
                                               f"10 nm cube cut from the same box, {t_one:.1f} s"},
                   "cpu_model": cpu_model()}
    del out32, out64

    small = batched = uneven = par = large = orders = mts = window = None
    if not args.no_small:
        small = small_box_record(torch, msmx, args)
        log("99,999-atom record done")
    states = None
    if not args.no_parareal:
        par, states = bench_parareal(torch, msmx, args.slices)
        log("parareal done")
    if not args.no_batched and states is not None:
        batched, uneven = bench_batched(torch, msmx, *states, args.steps, args.warmup, autotune=not args.no_autotune)
        log("batched done")
    del states
    if not args.no_large:
        large = bench_large(torch, msmx, named("water_12675000", margin=1.0), equilibrate_ps=args.equilibrate_ps)
        log("large box dynamics done")
    if not args.no_orders:
        orders = bench_orders(torch, msmx, named("water_99999").as_dtype(np.float32))
        log("orders done")
    dt_half = None
    if not args.no_mts:
        mts = bench_mts(torch, msmx, equilibrate_ps=args.equilibrate_ps)
        log("multiple time steps done")
        dt_half = bench_dt_halving(torch, msmx, equilibrate_ps=args.equilibrate_ps)
        log("dt halving done")
    if not args.no_window:
        window = bench_window(torch, msmx)
        log("window done")

    dims = "x".join(f"{d:g}" for d in np.round(w32.hi - w32.lo, 2))
    result.update({
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {n} atoms, rigid 3-site water, {dims} nm domain, a={w32.a} nm, "
                               f"h={w32.h} nm, {len(shapes)} grids, one energy+force+potential evaluation, "
                               f"FP32 bulk + FP64 energy reduction",
                   "atoms": n, "levels": len(shapes), "a_nm": w32.a, "h_nm": w32.h},
        "roofline": roofline,
        "composite_roofline": composite_roofline(n, pairs, shapes, sphere_taps(w32.a, w32.h), ms32),
        "cpu_baseline": cpu,
        "fp64_plain": fp64,
        "speedup_fp32_vs_fp64_plain": (value / fp64["value"]) if fp64 else None,
        "fp32_batched": batched,
        "speedup_fp32_batched_vs_fp64_plain": (batched["value"] / fp64["value"]) if (batched and fp64) else None,
        "uneven_batch": uneven,
        "parareal": par,
        "large_box": large,
        "box_99999": small,
        "orders": orders,
        "mts": mts,
        "dt_halving_fp64": dt_half,
        "window": window,
        "launch": launch,
        "accuracy": accuracy,
        "stage_ms": kernels,
    })
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
