"""Benchmark: D3Q19 FP32 fused stream-collide-force update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload channel|ogrid|batch|moving|...]
                    [--precision fp32|fp32c|fp64|fp16s|bf16s] [--no-cpu]

Prints ONE JSON line: MLUPS of the whole job (inputs resident in HBM), the
roofline of the fused step kernel (algorithmic bytes per launch / average
launch duration from HIP events on the stream the kernel runs on), and the FP64
CPU oracle timed on a bounded sample of the same workload.

--workload moving times a deforming D3Q19 periodic box of the same size in
FP64: every step computes the geometry of the next node positions and then
runs the fused step of a moving mesh.

--workload batch times the 256-mesh uneven D2Q9 batch instead: one persistent
launch per step replayed from captured graphs, with the launch shape chosen by
the library's autotuner, beside the same batch stepped by one launch per mesh
(plain and graph-captured).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp32c": 4, "fp16s": 2, "bf16s": 2}
# modes that store deviations from a 16-bit per-slot reference
SHIFTED = ("fp32", "fp16s", "bf16s")
REBASE_EVERY = 10


def algorithmic_bytes_per_cell(Q, d, precision, has_force, has_farfield=False):
    """Bytes one fused step launch must move per cell: the Q populations read
    once and written once, the packed per-cell geometry words (J, g^{ij} upper,
    A^i_a for a >= 1, a_ext when a body force acts, U_inf when there is a far
    field; FP64 words for FP64 storage, FP32 otherwise, with a second FP32
    word per g^{ij} for FP32 storage, whose arithmetic is FP64, and a_ext
    always there: it also cancels the FP32 rounding of A), and for the deviation
    storage modes the Q 16-bit references of the slots (each read by its
    writer and, at the offset of the population, by its reader: one array)."""
    sb = STORAGE_BYTES[precision]
    gb = 8 if precision == "fp64" else 4
    aext = has_force or precision == "fp32"
    words = 1 + d * (d + 1) // 2 + (Q - 1) * d + (d if aext else 0) + (d if has_farfield else 0)
    if precision == "fp32":   # FP64 arithmetic on FP32 words: g^{ij} as a hi + lo pair
        words += d * (d + 1) // 2
    refs = Q * 2 if precision in SHIFTED else 0
    return 2 * Q * sb + words * gb + refs


def rebase_bytes_per_cell(Q, precision):
    """Bytes one re-basing launch moves per cell: populations and references
    read and written once (deviation storage only)."""
    return 2 * Q * (STORAGE_BYTES[precision] + 2) if precision in SHIFTED else 0


def host_cpu():
    """Host cores and CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cores": os.cpu_count(), "cpu_model": model}


def copy_ceiling(vlbm):
    """STREAM-style rates of the device (library kernels, 2 GiB buffers):
    the best of regular and non-temporal accesses for copy, read and write."""
    out = {}
    for kind in ("copy", "read", "write"):
        best = 0.0
        for nt in (False, True):
            g, _ = vlbm.membench(kind, nontemporal=nt, bytes_=2 << 30, reps=8)
            best = max(best, g)
        out[kind] = round(best, 1)
    return out


def make_workload(name):
    from paper_2401_17183_amd import workloads as W
    if name == "channel":
        return W.tanh_channel_3d(256, 128, 128)
    if name == "ogrid":
        return W.ogrid_3d()
    if name == "d3q39":
        # sixth-order isotropic lattice: periodic wavy box, 128^3 cells
        return W.wavy_periodic("D3Q39", (128, 128, 128), 2.0)
    if name == "d2q21":
        return W.wavy_periodic("D2Q21", (2048, 1024), 8.0)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(workload="channel", seconds_target=12.0, tau_g=None, tau=None):
    """The FP64 NumPy oracle, one BLAS thread, on a bounded replica of the
    workload (same lattice, stretching, tau and boundaries, fewer cells), stepped
    until ~seconds_target; MLUPS = cell updates / wall time."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import geometry, lattice, sim
    from paper_2401_17183_amd import workloads as W

    if workload == "batch":
        ws = W.batch_meshes(256)[:4]
        label = "first 4 meshes of the 256-mesh D2Q9 bump batch"
    elif workload == "ogrid":
        ws = [W.ogrid_3d(32, 64, 8)]
        label = "D3Q19 O-grid 32x64x8"
    elif workload == "d3q39":
        ws = [W.wavy_periodic("D3Q39", (16, 16, 16), 0.25)]
        label = "D3Q39 wavy periodic 16^3"
    elif workload == "d2q21":
        ws = [W.wavy_periodic("D2Q21", (64, 64), 0.25)]
        label = "D2Q21 wavy periodic 64^2"
    else:
        ws = [W.tanh_channel_3d(32, 32, 16)]
        label = "D3Q19 tanh(2.5) channel 32x32x16"
    with threadpool_limits(limits=1):
        sims = []
        for w in ws:
            lat = lattice.by_name(w["lattice"])
            m = geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])
            s = sim.Sim(m, sim.Params(w["tau"] if tau is None or workload == "batch" else tau, body_force=w.get("body_force", (0, 0, 0)),
                                      rho_inf=w.get("rho_inf", 1.0), u_inf=w.get("u_inf", (0, 0, 0)),
                                      tau_g=tau_g))
            s.init(w.get("rho"), w.get("u"))
            s.step(1)
            sims.append(s)
        cells = sum(int(np.prod(w["n"])) for w in ws)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            for s in sims:
                s.step(1)
            steps += 1
        dt = time.perf_counter() - t0
    out = {"value": round(cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "sample": f"{label}, FP64, {steps} steps, {dt:.1f} s, 1 thread"}
    out.update(host_cpu())
    if workload == "batch":
        # the whole host: one oracle process per mesh of a sample, all cores at once
        one = {k: out[k] for k in ("value", "cores", "sample")}
        out.update(oracle_batch_pool())
        out["one_core"] = one
    return out


def cpu_baseline_moving(seconds_target=12.0, tau=None):
    """The FP64 moving-mesh oracle, one BLAS thread, on a 16x16x8 replica of the
    deforming box (same motion, waviness scaled with the size); the node
    positions of one period are made before timing, the geometry of each new
    position is computed inside the timed steps, as on the device."""
    from threadpoolctl import threadpool_limits

    from oracle import lattice, moving
    from paper_2401_17183_amd import workloads as W

    w = W.wavy_periodic("D3Q19", (16, 16, 8), 0.25)
    if tau is not None:
        w["tau"] = tau
    period = MOVING_MOTION["period"]
    pos = [W.moving_coords(w, t, **MOVING_MOTION) for t in range(period)]
    rng = np.random.default_rng(MOVING_SEED)
    shape = tuple(reversed(w["n"]))
    with threadpool_limits(limits=1):
        o = moving.MovingSim(lattice.by_name("D3Q19"), w["n"], pos[0][0], pos[0][1], w["dx"], w["tau"])
        o.init(1.0 + 0.01 * rng.standard_normal(shape), 0.01 * rng.standard_normal((3,) + shape))
        o.step(*pos[1])
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            o.step(*pos[(steps + 2) % period])
            steps += 1
        dt = time.perf_counter() - t0
    cells = int(np.prod(w["n"]))
    out = {"value": round(cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
           "sample": f"D3Q19 deforming wavy periodic 16x16x8, FP64 moving-mesh oracle, {steps} steps, "
                     f"{dt:.1f} s, 1 thread"}
    out.update(host_cpu())
    return out


def _oracle_mesh_worker(task):
    """Pool task: the oracle on batch mesh k, stepped for about `seconds`; returns
    (cell updates, seconds)."""
    k, seconds = task
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import geometry, lattice, sim
    from paper_2401_17183_amd import workloads as W
    w = W.batch_meshes(256)[k]
    with threadpool_limits(limits=1):
        lat = lattice.by_name(w["lattice"])
        m = geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])
        s = sim.Sim(m, sim.Params(w["tau"], body_force=w.get("body_force", (0, 0, 0))))
        s.init()
        s.step(1)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds:
            s.step(1)
            steps += 1
        dt = time.perf_counter() - t0
    return int(np.prod(w["n"])) * steps, dt


def oracle_batch_pool(seconds=10.0):
    """The FP64 oracle on every host core (at most 16, the share of one GPU's
    host): one process per mesh of the first `cores` meshes of the batch, each
    stepped for ~seconds; MLUPS = all cell updates / wall time of the pool."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")   # fresh interpreters: nothing of this process's GPU state
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_mesh_worker, [(k, seconds) for k in range(cores)])
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": round(upd / busy / 1e6, 4), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"first {cores} meshes of the 256-mesh D2Q9 bump batch, FP64, one process per mesh "
                      f"and core, {busy:.1f} s of stepping each ({wall:.1f} s with start-up)"}


# committed counter summaries per single-mesh workload: <stem>_<precision>[_tau..][_taug..].md
PROFILE_STEM = {"channel": "k_step_d3q19_channel_256x128x128", "d3q39": "k_step_d3q39_wavy_128x128x128"}

STEP_SOURCES = ["paper_2401_17183_amd/csrc/common.hpp", "paper_2401_17183_amd/csrc/dynamics.hpp",
                "paper_2401_17183_amd/csrc/stepcore.hpp", "paper_2401_17183_amd/csrc/step.hip"]
BATCH_SOURCES = STEP_SOURCES[:3] + ["paper_2401_17183_amd/csrc/batch.hip"]
MOVING_SOURCES = STEP_SOURCES[:3] + ["paper_2401_17183_amd/csrc/moving.hip"]
MOVING_PROFILE = "k_step_moving_d3q19_wavy_256x128x128_fp64.md"


def profile_values(profile, sources, require=None):
    """The `key = value` lines of a committed rocprofv3 summary, or None when
    there is no summary, the kernel sources changed since it was taken, or one
    of the `require` entries (e.g. the launch shape) differs from the summary's."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(path) as fh:
        for line in fh:
            if " = " in line:
                k, v = line.split(" = ", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != h.hexdigest()[:16]:
        return None
    if any(vals.get(k) != str(v) for k, v in (require or {}).items()):
        return None
    return vals


def profiled_traffic(profile, sources, require=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by a plain copy's reading), or None
    (see profile_values)."""
    vals = profile_values(profile, sources, require)
    if vals is None or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def profiled_valu(profile, sources):
    """The VALU evidence of a committed summary (SQ counters of the same
    kernel): instructions per wavefront, the SIMD's VALU busy fraction while
    its wavefronts are resident, and the graphics clock under the load."""
    vals = profile_values(profile, sources)
    keys = ("valu_insts_per_wave", "valu_busy_while_resident", "graphics_clock_GHz")
    if vals is None or any(k not in vals for k in keys):
        return None
    return {"kind": "valu", "valu_insts_per_wave": float(vals[keys[0]]),
            "valu_busy_while_resident": float(vals[keys[1]]), "graphics_clock_GHz": float(vals[keys[2]]),
            "source": f"profiles/{profile}"}


def _event_pair(torch, stream):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    return e0, e1


def _timed(torch, stream, fn, steps):
    """Milliseconds of `fn(steps)` between HIP events recorded on `stream`."""
    e0, e1 = _event_pair(torch, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    fn(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _copy_ref(torch, out, vlbm):
    """One plain 1 GiB device copy with the library's STREAM copy kernel
    (k_copy; the reference the HBM counters are scaled by), its best rate
    beside it."""
    g, grid = vlbm.membench("copy", nontemporal=False, bytes_=1 << 30, reps=1)
    out["config"]["copy_ref_bytes"] = 2 << 30
    out["config"]["copy_ref_GBps"] = round(g, 1)
    out["config"]["copy_ref_grid"] = grid


# Seconds of load before each measured run of steps: the GPU lowers its clocks
# within about 10 ms of idling (the host-side state copies of this script idle
# it for much longer) and needs some 40 ms of sustained load to raise them
# again; a 20-step window of the channel started from idle ran at 0.59 ms per
# step against 0.48 ms right after other work.
DEVICE_WARMUP_S = 0.3


def _device_warmup(torch, sim, seconds=DEVICE_WARMUP_S):
    """Keep the device busy for about `seconds` with `sim`, a separate copy of
    the workload (its state is never measured), and return the steps it ran."""
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        sim.step(20)
        torch.cuda.synchronize()
        n += 20
    return n


def collision_name(tau_g):
    if tau_g is None:
        return "BGK"
    return "regularised (tau_g = 1)" if tau_g == 1.0 else f"general (tau_g = {tau_g})"


def run_single(args, torch, vlbm):
    w = make_workload(args.workload)
    if args.tau is not None:
        w["tau"] = args.tau
    print(f"[bench] building {w['name']}", file=sys.stderr, flush=True)
    mesh = vlbm.Mesh.from_workload(w)
    p = vlbm.make_params(w["tau"], body_force=w.get("body_force", (0, 0, 0)), rho_inf=w.get("rho_inf", 1.0),
                         u_inf=w.get("u_inf", (0, 0, 0)), precision=args.precision, tau_g=args.tau_g,
                         fp_tol=args.fp_tol)
    rho = w.get("rho")
    u = w.get("u")
    sim = vlbm.Sim(mesh, p, rho=None if rho is None else rho.ravel(),
                   u=None if u is None else u.reshape(mesh.d, -1))
    # a second copy of the workload, stepped only to load the device before
    # each measured run (see DEVICE_WARMUP_S)
    heat = vlbm.Sim(mesh, p, rho=None if rho is None else rho.ravel(),
                    u=None if u is None else u.reshape(mesh.d, -1))
    cells = mesh.ncells
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()   # the Sim launches on torch's current stream
    blob = sim.save()                      # the state the timed steps start from
    heat_steps = _device_warmup(torch, heat)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ms = _timed(torch, stream, sim.step, args.steps)
    wall = time.perf_counter() - t0
    ms_per_step = ms / args.steps
    mlups = cells * args.steps / (ms / 1e3) / 1e6
    state = "ok"
    try:
        mo = sim.moments()
        finite = bool(torch.isfinite(mo["u"]).all().item())
    except vlbm.VlbmError as e:   # the timed steps ran; the state they reached is reported
        finite = False
        state = str(e)
    # the same steps again from the same state: durations of each kernel from
    # HIP events around its launches, then the fixed point's iteration counts
    print("[bench] kernel durations and fixed-point statistics of the same steps", file=sys.stderr, flush=True)
    sim.restore(blob)
    _device_warmup(torch, heat)
    sim.kernel_timing(True)
    sim.step(args.steps)
    kt = sim.kernel_timing(False)
    sim.restore(blob)
    sim.step_stats(True)
    sim.step(args.steps)
    st = sim.step_stats(False)
    del blob
    heat.close()
    k_ms = kt["step_ms"] / max(kt["step_launches"], 1)
    rb_ms = kt["rebase_ms"] / kt["rebase_launches"] if kt["rebase_launches"] else None
    has_force = any(v != 0 for v in w.get("body_force", (0, 0, 0)))
    has_ff = any(f == vlbm.FARFIELD for face in w["faces"] for f in face)
    bpc = algorithmic_bytes_per_cell(mesh.Q, mesh.d, args.precision, has_force, has_ff)
    achieved = bpc * cells / (k_ms / 1e3) / 1e9
    traffic = None
    binding = None
    if args.workload in PROFILE_STEM:
        tag = ("" if args.tau is None else f"_tau{args.tau:g}") + ("" if args.tau_g is None else f"_taug{args.tau_g:g}")
        traffic = profiled_traffic(f"{PROFILE_STEM[args.workload]}_{args.precision}{tag}.md", STEP_SOURCES)
        binding = profiled_valu(f"{PROFILE_STEM[args.workload]}_{args.precision}{tag}.md", STEP_SOURCES)
    print("[bench] STREAM-style ceiling", file=sys.stderr, flush=True)
    ceil = copy_ceiling(vlbm)
    return {
        "metric": METRIC,
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ARITH[args.precision],
        "data": "synthetic",
        "config": {"workload": w["name"] + f" {args.precision.upper()}", "cells": cells, "lattice": w["lattice"],
                   "tau": w["tau"], "collision": collision_name(args.tau_g), "storage": STORAGE[args.precision],
                   "wall_s": round(wall, 3), "finite": finite, "state": state,
                   "fp_iters_per_cell_step": round(st["iters_per_cell"], 3),
                   "fp_wave_max_iters_per_step": round(st["wave_max_iters"], 3),
                   "k_step_ms": round(k_ms, 5), "k_rebase_ms": None if rb_ms is None else round(rb_ms, 5),
                   "rebase_every": REBASE_EVERY if args.precision in SHIFTED else None,
                   "device_warmup": f"{DEVICE_WARMUP_S:g} s ({heat_steps} steps) of a separate copy of the "
                                    "workload between the warm-up and the timed steps"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": bpc * cells,
                     "bytes_per_cell": bpc, "kernel": "k_step",
                     "kernel_ms": round(k_ms, 5),
                     "copy_ceiling_GBps": ceil["copy"], "read_ceiling_GBps": ceil["read"],
                     "write_ceiling_GBps": ceil["write"],
                     "frac_of_copy_ceiling": round(achieved / ceil["copy"], 4) if ceil["copy"] else None,
                     # what limits the kernel short of the HBM roofline (SQ counters of the same
                     # sources), or None where no counter summary covers it
                     "binding_limit": binding},
    }


# The deforming-mesh workload: a periodic wavy D3Q19 box of the benchmarked
# channel's size whose node displacements from the uniform lattice breathe by
# 30 % with a period of 40 steps (the node positions of one period are made
# before timing and cycled).
MOVING_MOTION = dict(breathe=0.3, period=40)
MOVING_SEED = 7


def moving_bytes_per_cell(Q, d):
    """Bytes the fused step of a moving mesh moves per cell (FP64 only): the Q
    populations read and written once; J, g^{ij} upper and g^i of the cell;
    and g_i on the geometry boxes of three times (each box word once), from
    which the step computes its outgoing and incoming link coefficients."""
    nup = d * (d + 1) // 2
    return 2 * Q * 8 + (1 + nup + d * d + 3 * d * d) * 8


def moving_basis_bytes(d, ncells, nbox):
    """Bytes of k_basis per launch of a moving step: the d coordinates of each
    geometry-box node read, g_i written on the box (d*d words) and J, g^i and
    g^{ij} (full d x d) on the real cells (the real-cell g_i are made on
    demand from the box)."""
    return 8 * (nbox * (d + d * d) + ncells * (1 + 2 * d * d))


def run_moving(args, torch, vlbm):
    from paper_2401_17183_amd import workloads as W
    if args.precision != "fp64":
        raise SystemExit("--workload moving runs in FP64 (moving meshes are built for FP64 storage)")
    w = W.wavy_periodic("D3Q19", (256, 128, 128), 2.0)
    if args.tau is not None:
        w["tau"] = args.tau
    period = MOVING_MOTION["period"]
    print(f"[bench] building {w['name']} and the node positions of one period ({period} steps)",
          file=sys.stderr, flush=True)
    coords, wraps = [], []
    for t in range(period):
        X, wr = W.moving_coords(w, t, **MOVING_MOTION)
        if t == 0:
            mesh = vlbm.Mesh(w["lattice"], w["n"], X, w["faces"], wr, w["dx"])
        coords.append(torch.from_numpy(X.ravel()).to("cuda"))
        wraps.append(wr)
    del X
    rng = np.random.default_rng(MOVING_SEED)
    cells, d = mesh.ncells, mesh.d
    rho = 1.0 + 0.01 * rng.standard_normal(cells)
    u = 0.01 * rng.standard_normal((d, cells))
    sim = vlbm.Sim(mesh, vlbm.make_params(w["tau"], precision="fp64", fp_tol=args.fp_tol), rho=rho, u=u)
    del rho, u
    t = [0]

    def steps(n):
        for _ in range(n):
            t[0] += 1
            k = t[0] % period
            sim.step_moving(coords[k], wraps[k])

    stream = torch.cuda.current_stream()   # the Sim launches on torch's current stream
    print(f"[bench] warmup {args.warmup} + device warm-up", file=sys.stderr, flush=True)
    steps(args.warmup)
    torch.cuda.synchronize()
    # the mesh state cannot be restored once it moved: the device is loaded by
    # more untimed steps of the same run instead of a separate copy
    t0 = time.perf_counter()
    heat_steps = 0
    while time.perf_counter() - t0 < DEVICE_WARMUP_S:
        steps(10)
        torch.cuda.synchronize()
        heat_steps += 10
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ms = _timed(torch, stream, steps, args.steps)
    wall = time.perf_counter() - t0
    # the next steps of the same run, with HIP events around each kernel, then
    # as many with the fixed point's iteration counts
    sim.kernel_timing(True)
    steps(args.steps)
    kt = sim.kernel_timing(False)
    sim.step_stats(True)
    steps(args.steps)
    st = sim.step_stats(False)
    sim.sync()
    mo = sim.moments()
    finite = bool(torch.isfinite(mo["u"]).all().item())
    u_max = float(mo["u"].abs().max().item())
    ms_per_step = ms / args.steps
    nbox = int(np.prod([n + 2 for n in w["n"]]))   # one layer around the real cells (one-cell links)
    kernels = {}
    for key, name, nbytes in (("step", "k_step_moving", moving_bytes_per_cell(mesh.Q, d) * cells),
                              ("basis", "k_basis", moving_basis_bytes(d, cells, nbox))):
        if kt[f"{key}_launches"] == 0:
            continue
        kms = kt[f"{key}_ms"] / kt[f"{key}_launches"]
        kernels[name] = {"ms": round(kms, 5), "algorithmic_bytes_per_launch": nbytes,
                         "GBps": round(nbytes / (kms / 1e3) / 1e9, 1)}
    dominant = max(kernels, key=lambda k: kernels[k]["ms"])
    dk = kernels[dominant]
    traffic = binding = None
    if dominant == "k_step_moving" and args.tau is None:
        traffic = profiled_traffic(MOVING_PROFILE, MOVING_SOURCES)
        binding = profiled_valu(MOVING_PROFILE, MOVING_SOURCES)
    sim.close()
    mesh.close()
    return {
        "metric": METRIC,
        "value": round(cells * args.steps / (ms / 1e3) / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w['name']} deforming (displacements breathe by 30 %, period {period} steps), "
                               "FP64; per step the geometry of the next node positions and the fused step",
                   "cells": cells, "lattice": w["lattice"], "tau": w["tau"], "storage": "f64",
                   "wall_s": round(wall, 3), "finite": finite, "u_max": u_max,
                   "kernels": kernels,
                   "fp_iters_per_cell_step": round(st["iters_per_cell"], 3),
                   "fp_wave_max_iters_per_step": round(st["wave_max_iters"], 3),
                   "device_warmup": f"{heat_steps} more untimed steps of the same run (>= {DEVICE_WARMUP_S:g} s)"},
        # the kernel of the step with the longest average duration
        "roofline": {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": dk["algorithmic_bytes_per_launch"],
                     "kernel": dominant, "kernel_ms": dk["ms"],
                     # what limits the kernel short of the HBM roofline (SQ counters of the same
                     # sources), or None where no counter summary covers it
                     "binding_limit": binding},
    }


def run_batch(args, torch, vlbm):
    from paper_2401_17183_amd import workloads as W
    ws = W.batch_meshes(256)
    print("[bench] building 256 bump-channel meshes", file=sys.stderr, flush=True)
    meshes = [vlbm.Mesh.from_workload(w) for w in ws]
    params = [vlbm.make_params(w["tau"], body_force=w["body_force"], precision=args.precision, tau_g=args.tau_g)
              for w in ws]
    b = vlbm.Batch(meshes, params)   # every member starts at rest
    cells = b.info()["cells"]
    stream = torch.cuda.ExternalStream(b.info()["stream"])
    print("[bench] autotune", file=sys.stderr, flush=True)
    block, gpc = b.autotune(trial_steps=10, cache_path=args.tune_cache)
    modes = {}
    plan = [("persistent_graph", vlbm.BATCH_PERSISTENT_GRAPH, args.steps),
            ("persistent", vlbm.BATCH_PERSISTENT, max(32, args.steps // 4)),
            ("eager_per_mesh", vlbm.BATCH_EAGER, max(32, args.steps // 10)),
            ("graph_per_mesh", vlbm.BATCH_EAGER_GRAPH, max(32, args.steps // 10))]
    for name, mode, steps in plan[:1] if args.persistent_only else plan:
        b.set_mode(mode)
        print(f"[bench] {name}: warmup {args.warmup + 32}, timing {steps} steps", file=sys.stderr, flush=True)
        b.step(args.warmup + 32)   # includes the graph capture
        b.sync()
        ms = _timed(torch, stream, b.step, steps)
        b.sync()
        modes[name] = {"steps": steps, "ms_per_step": round(ms / steps, 5),
                       "MLUPS": round(cells * steps / (ms / 1e3) / 1e6, 1)}
    b.set_mode(vlbm.BATCH_PERSISTENT_GRAPH)
    main = modes["persistent_graph"]
    bpc = algorithmic_bytes_per_cell(9, 2, args.precision, True)
    achieved = bpc * cells / (main["ms_per_step"] / 1e3) / 1e9
    finite = all(bool(torch.isfinite(m.moments()["u"]).all().item()) for m in b.members[:8])
    traffic = None
    if args.precision == "fp32":
        traffic = profiled_traffic("k_batch_d2q9_bump256_fp32.md", BATCH_SOURCES,
                                   {"launch_block": block, "launch_grid_per_cu": gpc})
    out = {
        "metric": METRIC,
        "value": main["MLUPS"], "unit": "MLUPS", "n_gpus": 1, "steps": main["steps"], "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": ARITH[args.precision], "data": "synthetic",
        "config": {"workload": f"256 uneven D2Q9 bump channels {args.precision.upper()}, one persistent launch "
                               "per step, graph-replayed", "cells": cells, "meshes": 256,
                   "storage": STORAGE[args.precision], "block": block, "grid_per_cu": gpc, "modes": modes,
                   "finite": finite},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": bpc * cells,
                     "bytes_per_cell": bpc, "kernel": "k_batch"},
    }
    b.close()
    return out


def surrogate_flops_per_sample(H, W):
    """Multiply-adds x 2 of the conv layers of one forward pass (the network
    of paper_2401_17183_amd.surrogate), from the layer shapes."""
    from paper_2401_17183_amd import surrogate as S
    C = S.LEVEL_CHANNELS
    total = 0
    res = [(H >> l) * (W >> l) for l in range(5)]
    shapes = S.layer_shapes()
    out_res = [res[0], res[0], res[1], res[1], res[2], res[2], res[3], res[3], res[4], res[4],
               res[3], res[3], res[2], res[2], res[1], res[1], res[0], res[0], res[0]]
    for (co, ci), px in zip(shapes, out_res):
        total += 2 * px * co * 9 * ci
    return total


def run_train(args, torch, vlbm):
    """Throughput of the surrogate's training step alone (forward, MSE,
    backward, Adam; BF16 MFMA) on one minibatch of bump-channel inputs with
    seeded targets, 128 x 64 cells."""
    from paper_2401_17183_amd import surrogate as S
    from paper_2401_17183_amd import workloads as W
    ws = W.surrogate_meshes(args.batch)
    H, Wd = ws[0]["n"][1], ws[0]["n"][0]
    x = torch.tensor(np.stack([S.features(w) for w in ws])).cuda()
    rng = np.random.default_rng(2401)
    t = torch.tensor(rng.standard_normal((args.batch, H, Wd, 3)).astype(np.float32)).cuda()
    net = vlbm.Surrogate(H, Wd, args.batch, S.he_init(2401))
    for _ in range(args.warmup):
        net.train_step(x, t, 1e-4, want_loss=False)
    stream = torch.cuda.current_stream()
    ms = _timed(torch, stream, lambda n: [net.train_step(x, t, 1e-4, want_loss=False) for _ in range(n)],
                args.steps)
    ms_step = ms / args.steps
    flops = 3 * surrogate_flops_per_sample(H, Wd) * args.batch
    tf = flops / (ms_step / 1e3) / 1e12
    net.close()
    return {
        "metric": METRIC, "value": round(args.batch / (ms_step / 1e3), 1), "unit": "samples/s (training)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"surrogate training step, minibatch {args.batch}, {Wd}x{H} bump channels",
                   "flop_per_step": flops},
        "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tf / 2500.0, 5), "traffic": None,
                     "kernel": "k_conv_tile / k_wgrad_tile (forward, input and weight gradients)"},
    }


def run_surrogate(args, torch, vlbm):
    """Steady states of bump channels from the batched solver, training of the
    BF16-MFMA surrogate, then the test meshes solved to r <= 1e-6 from rest
    (cold) and from the surrogate's prediction (warm, inference included)."""
    from paper_2401_17183_amd import surrogate as S
    from paper_2401_17183_amd import workloads as W
    log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)
    ntr, nva, nte = args.train, args.val, args.test
    ws = W.surrogate_meshes(ntr + nva + nte)
    wtr, wva, wte = ws[:ntr], ws[ntr:ntr + nva], ws[ntr + nva:]
    H, Wd = ws[0]["n"][1], ws[0]["n"][0]
    log(f"steady states of {ntr + nva} training/validation meshes")
    b, _ = S.make_batch(wtr + wva)
    gen_steps, gen_total, gen_wall = S.solve_steady(b, tol=args.tol, log=log)
    F = S.fields(b, wtr + wva)
    b.close()
    del b
    log(f"generated in {gen_wall:.1f} s, {gen_total} steps; unconverged {(gen_steps < 0).sum()}")
    norm = S.Normaliser.fit(F[:ntr], ws[0]["u_bulk"])
    Xall = np.stack([S.features(w) for w in wtr + wva])
    X = torch.tensor(Xall[:ntr]).cuda()
    T = torch.tensor(norm.encode(F[:ntr])).cuda()
    Xv = torch.tensor(Xall[ntr:]).cuda()
    Tv = torch.tensor(norm.encode(F[ntr:])).cuda()
    net = vlbm.Surrogate(H, Wd, args.batch, S.he_init(2401))
    log(f"training {args.epochs} epochs")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = S.train(net, X, T, Xv, Tv, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    torch.cuda.synchronize()
    train_wall = time.perf_counter() - t0
    train_steps = args.epochs * max(1, ntr // args.batch)
    flops = 3 * surrogate_flops_per_sample(H, Wd) * args.batch * train_steps
    # cold
    log(f"cold solves of {nte} test meshes")
    bc, _ = S.make_batch(wte)
    cold_steps, cold_total, cold_wall = S.solve_steady(bc, tol=args.tol, log=log)
    Fte = S.fields(bc, wte)
    bc.close()
    del bc
    # warm (inference timed with the solve)
    log(f"warm solves of {nte} test meshes")
    bw, mw = S.make_batch(wte)
    Xte = torch.tensor(np.stack([S.features(w) for w in wte])).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = S.predict(net, norm, Xte, args.batch)
    S.warm_start(bw, P, mw)
    torch.cuda.synchronize()
    infer_wall = time.perf_counter() - t0
    warm_steps, warm_total, warm_solve = S.solve_steady(bw, tol=args.tol, log=log)
    Fw = S.fields(bw, wte)
    bw.close()
    warm_wall = infer_wall + warm_solve
    uerr = [float(np.linalg.norm(P[k, ..., :2] - Fte[k, ..., :2]) / np.linalg.norm(Fte[k, ..., :2]))
            for k in range(nte)]
    agree = [float(np.linalg.norm(Fw[k, ..., :2] - Fte[k, ..., :2]) / np.linalg.norm(Fte[k, ..., :2]))
             for k in range(nte)]
    ok = (cold_steps > 0) & (warm_steps > 0)
    ratio = cold_steps[ok] / warm_steps[ok]
    out = {
        "metric": METRIC, "value": round(cold_wall / warm_wall, 3),
        "unit": "x (cold / warm wall time to r <= 1e-6, inference included)",
        "n_gpus": 1, "steps": int(warm_total), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"surrogate warm start, {nte} test bump channels {Wd}x{H} (D2Q9 FP32 storage)",
                   "train": ntr, "val": nva, "test": nte, "epochs": args.epochs, "batch": args.batch,
                   "tol": args.tol, "generation_wall_s": round(gen_wall, 2), "generation_steps": int(gen_total),
                   "train_wall_s": round(train_wall, 2), "final_train_loss": hist[-1][0],
                   "final_val_loss": hist[-1][1],
                   "cold_wall_s": round(cold_wall, 3), "warm_wall_s": round(warm_wall, 3),
                   "inference_wall_s": round(infer_wall, 4),
                   "cold_steps_median": float(np.median(cold_steps[cold_steps > 0])) if (cold_steps > 0).any() else None,
                   "warm_steps_median": float(np.median(warm_steps[warm_steps > 0])) if (warm_steps > 0).any() else None,
                   "steps_ratio_median": float(np.median(ratio)) if ratio.size else None,
                   "steps_ratio_min": float(np.min(ratio)) if ratio.size else None,
                   "steps_ratio_max": float(np.max(ratio)) if ratio.size else None,
                   "unconverged": {"cold": int((cold_steps < 0).sum()), "warm": int((warm_steps < 0).sum())},
                   "surrogate_u_rel_l2_median": float(np.median(uerr)), "surrogate_u_rel_l2_max": float(np.max(uerr)),
                   "warm_vs_cold_final_u_rel_l2_max": float(np.max(agree))},
        "roofline": {"bound": "mfma", "achieved": round(flops / train_wall / 1e12, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(flops / train_wall / 1e12 / 2500.0, 5), "traffic": None,
                     "kernel": "k_conv_tile / k_wgrad_tile (whole training loop, BF16 MFMA)"},
    }
    net.close()
    return out


METRIC = "MLUPS + % HBM roofline (D3Q19 FP32); warm vs cold time-to-1e-6 residual"
# the arithmetic type of each storage mode: fp32 storage computes in FP64 registers
ARITH = {"fp32": "f64", "fp32c": "f32", "fp64": "f64", "fp16s": "f32", "bf16s": "f32"}
STORAGE = {"fp32": "f32", "fp32c": "f32", "fp64": "f64", "fp16s": "f16", "bf16s": "bf16"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="channel",
                    choices=["channel", "ogrid", "d3q39", "d2q21", "batch", "surrogate", "train", "moving"])
    ap.add_argument("--precision", default=None, choices=sorted(STORAGE_BYTES),
                    help="storage precision (default: fp32; fp64 for --workload moving)")
    ap.add_argument("--tune-cache", default=None, help="autotune cache file for --workload batch")
    ap.add_argument("--persistent-only", action="store_true",
                    help="--workload batch: time only the persistent graph-replayed mode (for counter runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tau", type=float, default=None,
                    help="channel / O-grid: override the workload's relaxation time")
    ap.add_argument("--fp-tol", type=float, default=-1.0,
                    help="stopping tolerance of the per-cell fixed point (default: the library's for the precision)")
    ap.add_argument("--tau-g", type=float, default=None,
                    help="general collision matrix: relaxation time of the non-hydrodynamic part "
                         "(default: BGK; 1 = regularised)")
    ap.add_argument("--train", type=int, default=4096, help="surrogate: training meshes")
    ap.add_argument("--val", type=int, default=128, help="surrogate: validation meshes")
    ap.add_argument("--test", type=int, default=64, help="surrogate: test meshes")
    ap.add_argument("--epochs", type=int, default=200, help="surrogate: training epochs")
    ap.add_argument("--batch", type=int, default=32, help="surrogate: minibatch")
    ap.add_argument("--lr", type=float, default=1e-3, help="surrogate: peak learning rate")
    ap.add_argument("--tol", type=float, default=1e-6, help="surrogate: steady residual target")
    ap.add_argument("--copy-ref", action="store_true",
                    help="after timing, run one plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "fp64" if args.workload == "moving" else "fp32"
    if args.gpus != 1:
        print("this build runs on one GPU only: --gpus must be 1 (the multi-GPU slab "
              "decomposition is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2401_17183_amd import vlbm

    torch.cuda.set_device(0)
    if args.workload == "batch":
        out = run_batch(args, torch, vlbm)
    elif args.workload == "surrogate":
        out = run_surrogate(args, torch, vlbm)
    elif args.workload == "train":
        out = run_train(args, torch, vlbm)
    elif args.workload == "moving":
        out = run_moving(args, torch, vlbm)
    else:
        out = run_single(args, torch, vlbm)
    if args.copy_ref:
        _copy_ref(torch, out, vlbm)
    if not args.no_cpu and args.workload not in ("surrogate", "train"):
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = (cpu_baseline_moving(tau=args.tau) if args.workload == "moving" else
                               cpu_baseline(args.workload, tau_g=args.tau_g, tau=args.tau))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
