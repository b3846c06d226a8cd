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


class SampleGeometry:
    """Oracle geometry of selected cells of a large mesh, each computed on its
    own 5x5(x5) coordinate patch (the cell plus two node layers, periodic
    wraps applied): the quantities are local, so they equal the full-mesh
    ones.  Arrays carry the sample as their last axis."""

    def __init__(self, w, cells, body_force=None):
        from oracle import geometry, lattice
        lat = lattice.by_name(w["lattice"])
        d = lat.d
        n = w["n"]
        X = w["coords"]
        faces = w["faces"]
        wrap = np.array([np.asarray(v, dtype=np.float64)[:d] for v in w["wrap"]])
        parts = {"J": [], "gup": [], "A": [], "g": [], "gco": []}
        for cell in cells:
            q = []
            r = int(cell)
            for i in range(d):
                q.append(r % n[i])
                r //= n[i]
            idx = []
            shift = []
            for i in range(d):
                k = np.arange(q[i] - 2, q[i] + 3)
                if faces[i][0] == geometry.PERIODIC:
                    idx.append(np.mod(k, n[i]))
                    shift.append(np.floor_divide(k, n[i]).astype(np.float64))
                else:
                    idx.append(k + 2)
                    shift.append(np.zeros(5))
            P = X[np.ix_(*reversed(idx))].copy()
            for i in range(d):
                shp = [1] * d
                shp[d - 1 - i] = -1
                P += shift[i].reshape(shp)[..., None] * wrap[i]
            m = geometry.Mesh(lat, (1,) * d, P, [(geometry.WALL, geometry.WALL)] * d, [(0,) * d] * d, w["dx"])
            gg = geometry.Geometry(m, body_force)
            for k in parts:
                parts[k].append(getattr(gg, k).reshape(getattr(gg, k).shape[: -d]))
        self.lat = lat
        self.J = np.array(parts["J"]).reshape(-1)
        for k in ("gup", "A", "g", "gco"):
            setattr(self, k, np.moveaxis(np.array(parts[k]), 0, -1))
        G = np.zeros(d) if body_force is None else np.asarray(body_force, dtype=np.float64)[:d]
        self.G = G
        self.aext = np.einsum("k,ik...->i...", G, self.gco)
