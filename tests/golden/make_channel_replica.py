"""Writes channel_replica_64x32x32.npz: the FP64 oracle's velocity on a
64x32x32 replica of the 256x128x128 D3Q19 channel workload (x, z periodic,
walls at y = +-1 with y = tanh(2.5 eta)/tanh(2.5), dx = sqrt(3) times the
smallest central wall-normal spacing, tau = 0.52, G = (1e-6, 0, 0), rho = 1,
u ~ U(-1e-3, 1e-3) per component from numpy.random.default_rng(2401)), run
from the initial state of the initial-state reading for 1000 steps.

Stored: the Euclidean velocity u = Ut^i g_i (the output mapping of the
oracle) after 200 and 1000 steps on every cell of the columns x = 0, 4, ...,
60 (all y and z), as float32: the velocity's relative L2 error bar of the GPU
comparison is 1e-5, far above float32's rounding.  Only oracle/ computes; the
seeded inputs come from the workload generator.

    python tests/golden/make_channel_replica.py      # about 30 minutes, one core
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import geometry, lattice, sim  # noqa: E402
from paper_2401_17183_amd import workloads as W  # noqa: E402

N = (64, 32, 32)
STEPS = (200, 1000)
XCOLS = np.arange(0, N[0], 4)


def main():
    from threadpoolctl import threadpool_limits
    w = W.tanh_channel_3d(*N)
    lat = lattice.by_name(w["lattice"])
    m = geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])
    s = sim.Sim(m, sim.Params(w["tau"], body_force=w["body_force"]))
    out = {"xcols": XCOLS, "steps": np.array(STEPS)}
    t0 = time.time()
    with threadpool_limits(limits=1):
        s.init(w["rho"], w["u"])
        done = 0
        for k in STEPS:
            s.step(k - done)
            done = k
            u = s.moments()["u"]            # (3, n3, n2, n1)
            out[f"u_{k}"] = u[..., XCOLS].astype(np.float32)
            print(f"step {k}: {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "channel_replica_64x32x32.npz"), **out)


if __name__ == "__main__":
    main()
