"""Benchmark: D3Q19 FP32 fused stream-collide-force update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload channel|ogrid] [--no-cpu]

Prints ONE JSON line: MLUPS of the whole job (inputs resident in HBM), the
roofline of the fused step kernel (algorithmic bytes per launch / average
launch duration from HIP events on the stream the kernel runs on), and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_cell(Q, d, storage_bytes, has_force):
    """Populations read + written once (2 Q s) plus the packed per-cell geometry
    the kernel must read: J, g^{ij} (upper), A^i_a (a >= 1), a_ext."""
    words = 1 + d * (d + 1) // 2 + (Q - 1) * d + (d if has_force else 0)
    return 2 * Q * storage_bytes + words * storage_bytes


def make_workload(name):
    from paper_2401_17183_amd import workloads as W
    if name == "channel":
        return W.tanh_channel_3d(256, 128, 128)
    if name == "ogrid":
        return W.ogrid_3d()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(seconds_target=12.0):
    """The FP64 NumPy oracle, single BLAS thread, on a 32x32x16 replica of the
    stretched channel (same strength and tau); steps until ~seconds_target."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import geometry, lattice, sim
    from paper_2401_17183_amd import workloads as W

    w = W.tanh_channel_3d(32, 32, 16)
    lat = lattice.by_name(w["lattice"])
    with threadpool_limits(limits=1):
        m = geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])
        s = sim.Sim(m, sim.Params(w["tau"], body_force=w["body_force"]))
        s.init(w["rho"], w["u"])
        s.step(1)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            s.step(1)
            steps += 1
        dt = time.perf_counter() - t0
    cells = int(np.prod(w["n"]))
    return {"value": cells * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"D3Q19 tanh(2.5) channel 32x32x16 FP64, {steps} steps, {dt:.1f} s, 1 thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="after timing, run one plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this build runs on one GPU only: --gpus must be 1 (the multi-GPU slab "
              "decomposition is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2401_17183_amd import vlbm

    torch.cuda.set_device(0)
    w = make_workload(args.workload)
    print(f"[bench] building {w['name']}", file=sys.stderr, flush=True)
    mesh = vlbm.Mesh.from_workload(w)
    p = vlbm.make_params(w["tau"], body_force=w.get("body_force", (0, 0, 0)), rho_inf=w.get("rho_inf", 1.0),
                         u_inf=w.get("u_inf", (0, 0, 0)), precision=args.precision)
    rho = w.get("rho")
    u = w.get("u")
    sim = vlbm.Sim(mesh, p, rho=None if rho is None else rho.ravel(),
                   u=None if u is None else u.reshape(mesh.d, -1))
    cells = mesh.ncells
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    mlups = cells * args.steps / (ms / 1e3) / 1e6
    sb = {"fp64": 8, "fp32": 4, "fp32c": 4, "fp16s": 2, "bf16s": 2}[args.precision]
    has_force = any(v != 0 for v in w.get("body_force", (0, 0, 0)))
    bpc = algorithmic_bytes_per_cell(mesh.Q, mesh.d, sb, has_force)
    achieved = bpc * cells / (ms_per_step / 1e3) / 1e9
    mo = sim.moments()
    finite = bool(torch.isfinite(mo["u"]).all().item())
    out = {
        "metric": "MLUPS + % HBM roofline (D3Q19 FP32); warm vs cold time-to-1e-6 residual",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        # the arithmetic type: the fp32 storage mode computes in FP64 registers
        "vs_baseline": None, "dtype": {"fp32": "f64", "fp32c": "f32", "fp64": "f64", "fp16s": "f32",
                                       "bf16s": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w["name"] + f" {args.precision.upper()}", "cells": cells, "lattice": w["lattice"],
                   "tau": w["tau"], "storage": {"fp32": "f32", "fp32c": "f32", "fp64": "f64", "fp16s": "f16",
                                                "bf16s": "bf16"}[args.precision],
                   "wall_s": round(wall, 3), "finite": finite},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_cell": bpc, "kernel": "k_step"},
    }
    if args.copy_ref:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["config"]["copy_ref_bytes"] = 2 * src.numel() * 4
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
