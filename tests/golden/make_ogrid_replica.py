"""Writes ogrid_replica_256x128x2.npz: the FP64 oracle's velocity on a
radially faithful replica of the 256x512x64 D3Q19 O-grid workload: the same
256 log-spaced radii r = 20^(k/255) between the cylinder wall (r = 1,
bounce-back) and the far field (r = 20, imposed equilibrium), the same
dx = radial spacing at r = 1, u_inf = 0.05 along x and Re = 100
(tau = 0.754), with 128 instead of 512 cells around (theta periodic) and 2
instead of 64 along the periodic z axis (the flow is planar).  Started from
the far-field flow (rho = 1, u = u_inf everywhere) and run for 200 steps.

Stored: the Euclidean velocity u = Ut^i g_i after 50, 100 and 200 steps on
every cell of the theta rows 0, 4, ..., 124 (all radii and both z), as
float32 (far below the 1e-5 relative error bar of the comparison).  Only
oracle/ computes; the mesh comes from the workload generator.

    python tests/golden/make_ogrid_replica.py      # about 6 minutes, one core
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

N = (256, 128, 2)
STEPS = (50, 100, 200)
ROWS = np.arange(0, N[1], 4)


def main():
    from threadpoolctl import threadpool_limits
    w = W.ogrid_3d(*N)
    lat = lattice.by_name(w["lattice"])
    m = geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])
    s = sim.Sim(m, sim.Params(w["tau"], rho_inf=w["rho_inf"], u_inf=w["u_inf"]))
    nc = int(np.prod(N))
    u0 = np.zeros((3,) + m.shape)
    u0[0] = w["u_inf"][0]
    out = {"rows": ROWS, "steps": np.array(STEPS)}
    t0 = time.time()
    with threadpool_limits(limits=1):
        s.init(np.ones(m.shape), u0)
        done = 0
        for k in STEPS:
            s.step(k - done)
            done = k
            u = s.moments()["u"]            # (3, n3, n2, n1)
            out[f"u_{k}"] = u[:, :, ROWS, :].astype(np.float32)
            print(f"step {k}: {time.time() - t0:.0f} s", flush=True)
    assert nc == m.ncells
    np.savez_compressed(os.path.join(HERE, "ogrid_replica_256x128x2.npz"), **out)


if __name__ == "__main__":
    main()
