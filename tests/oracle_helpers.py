"""Glue between the seeded workloads and the oracle (tests only)."""
import numpy as np

from oracle import geometry, lattice, sim


def mesh_of(w):
    lat = lattice.by_name(w["lattice"])
    return geometry.Mesh(lat, w["n"], w["coords"], w["faces"], w["wrap"], w["dx"])


def sim_of(w, tau=None, **kw):
    m = mesh_of(w)
    p = sim.Params(w["tau"] if tau is None else tau, body_force=w.get("body_force"),
                   rho_inf=w.get("rho_inf", 1.0), u_inf=w.get("u_inf"), **kw)
    return sim.Sim(m, p)


def near_equilibrium_state(s, amp=1e-2, seed=7):
    """A random non-equilibrium state: the consistent equilibrium of random
    rho, u, plus a random perturbation of relative size amp."""
    rng = np.random.default_rng(seed)
    m = s.mesh
    rho = 1.0 + 0.05 * rng.standard_normal(m.shape)
    u = 0.02 * rng.standard_normal((m.d,) + m.shape)
    N = s.init(rho, u)
    N = N * (1.0 + amp * rng.standard_normal(N.shape))
    s.set_state(N)
    return N
