"""Time-varying coordinates: a mesh whose node positions move in time.

Test infrastructure (the FP64 oracle), as the rest of this package.

The paper's closing discussion (Sec. 4) names a coordinate system that varies
in time -- flows around a dynamically deforming body -- as a next step and
gives no equations for it.  This module is the library's reading, obtained
from the static construction of Sec. 2.2 by following every particle along
its hop in space and in time:

* the mesh is given at every integer time t by its node positions x(q, t);
  the geometry of Sec. 2.1 at time t (g_i, J, g^i, g^{ij}, a_ext) is that of
  x(q, t);
* a population that leaves cell q at time t along c_a leaves with the lattice
  velocity e_a(q, t) = c_a^j g_j(q, t) (eq. (lattice)) and arrives at q + c_a at
  time t + 1 with e_a(q + c_a, t + 1).  The momentum it gains on the way is
  split, as in eqs. (forceI) and (forceO), half to the cell it leaves and half
  to the cell it reaches:
      J chi^o(q, t) = - sum_a [e_a(q + c_a, t + 1) - e_a(q, t)] N'_a(q, t)
      J chi^I(q, t) = - sum_a [e_a(q, t) - e_a(q - c_a, t - 1)] N_a(q, t)
  With the outgoing and incoming link coefficients
      A+^i_a(q, t) = [e_a(q + c_a, t + 1) - e_a(q, t)] . g^i(q, t)
      A-^i_a(q, t) = [e_a(q, t) - e_a(q - c_a, t - 1)] . g^i(q, t)
  eq. (compo-constr) reads J F^i = -1/2 sum_a [A+^i_a N'_a + A-^i_a N_a].  On a
  static mesh A+_a = A_a and A-_a = A_opp(a), the static coefficients;
* the momentum-flux correction of eq. (delta-flux) takes A+_a + A-_a where
  the static form has A_a + A_opp(a);
* before the first step the mesh is at rest (x(q, -1) = x(q, 0)), and the
  initial state is the static one on x(q, 0);
* the output mapping at time t treats the mesh as momentarily at rest
  (x(q, t + 1) = x(q, t)): it is the static one on x(q, t).
Periodic meshes only (walls and far fields of a moving body are left out);
a periodic axis may change its translation vector in time.

Conserved exactly (to roundoff), on any deforming periodic mesh: the mass,
and the mid-link Euclidean momentum with each e_a taken at the time the
particle has it,
    I(t) = 1/2 sum_q sum_a [e_a(q, t) + e_a(q - c_a, t - 1)] N_a(q, t)
         = sum_q g_i(q, t) sum_a (c_a^i - A-^i_a(q, t) / 2) N_a(q, t),
which grows by G times the mass per step under a body force G: the cell
balance of the static case, sum_a (e_a + e_a') N' = sum_a (e_a + e_a'') N,
with e_a' = e_a(q + c_a, t + 1) and e_a'' = e_a(q - c_a, t - 1), summed over the
cells and carried by the advection (eq. (adv)).

Pinned by (tests/test_oracle_moving.py): equality with the static method on a
mesh that does not move and on a mesh in rigid translation (its tangent
vectors do not change), the two conservation laws on deforming and rotating
meshes, a fluid at rest staying at rest on a rigidly rotating uniform mesh,
and planted mistakes (the time levels of the coefficients swapped) breaking
the momentum balance.
"""
import numpy as np

from . import collide as _c
from .geometry import Mesh, PERIODIC, _view, basis, box_layers, real
from .stream import sources, stream


def _e(lat, g_box, a, offset, L):
    """e_a = c_a^j g_j on the real cells shifted by `offset`, from g on the box."""
    d = len(offset)
    gs = _view(g_box, 2, list(offset), L, 0)
    return np.einsum("j,jk...->k...", lat.cf[a], gs)


def link_coefficients(lat, box_prev, box_cur, box_next, gco_cur, d):
    """A+ and A- (Q, d, *n) of the step at time t from g_i on the boxes of the
    times t - 1, t and t + 1 and g^i at time t on the real cells."""
    L = lat.speed
    zero = [0] * d
    Ap = np.zeros((lat.Q, d) + gco_cur.shape[2:])
    Am = np.zeros_like(Ap)
    for a in range(lat.Q):
        c = list(lat.c[a])
        mc = [-v for v in c]
        e_here = _e(lat, box_cur, a, zero, L)
        e_out = _e(lat, box_next, a, c, L) - e_here            # e_a(q + c_a, t + 1) - e_a(q, t)
        e_in = e_here - _e(lat, box_prev, a, mc, L)             # e_a(q, t) - e_a(q - c_a, t - 1)
        Ap[a] = np.einsum("k...,ik...->i...", e_out, gco_cur)
        Am[a] = np.einsum("k...,ik...->i...", e_in, gco_cur)
    return Ap, Am


class _Geo:
    """The per-time quantities collide() needs."""

    def __init__(self, lat, bas, A, G, d):
        self.lat = lat
        self.J = real(bas["J"], 0, d, lat.speed)
        self.gup = real(bas["gup"], 2, d, lat.speed)
        self.gco = real(bas["gco"], 2, d, lat.speed)
        self.g = real(bas["g"], 2, d, lat.speed)
        self.A = A
        self.aext = np.einsum("k,ik...->i...", G, self.gco)


class MovingSim:
    """The method on a periodic mesh whose node positions change every step.

    lat, n, coords0 (x(q, 0), the layout of geometry.Mesh), wrap0, dx, tau,
    body_force (Euclidean acceleration, default 0).  step(coords_next,
    wrap_next) advances from t to t + 1 with the mesh moving to x(q, t + 1).
    """

    def __init__(self, lat, n, coords0, wrap0, dx, tau, body_force=None, tol=1e-14, max_iter=50):
        d = lat.d
        self.lat, self.n, self.d, self.dx = lat, tuple(n), d, float(dx)
        self.faces = [(PERIODIC, PERIODIC)] * d
        self.tau, self.tol, self.max_iter = float(tau), tol, max_iter
        self.G = np.zeros(d) if body_force is None else np.asarray(body_force, dtype=np.float64)[:d]
        self.mesh = Mesh(lat, n, coords0, self.faces, wrap0, dx)
        self.box = basis(self.mesh)
        self.box_prev = self.box                               # at rest before t = 0
        self.src = sources(self.mesh)
        self.N = None
        self.t = 0

    def _static_geo(self):
        """Geometry of x(q, t) as a momentarily resting mesh."""
        from .geometry import Geometry
        return Geometry(self.mesh, self.G)

    def init(self, rho=None, u=None):
        """The static initial state on x(q, 0) (oracle.sim.Sim.init)."""
        m = self.mesh
        rho = np.ones(m.shape) if rho is None else np.asarray(rho, dtype=np.float64)
        u = np.zeros((m.d,) + m.shape) if u is None else np.asarray(u, dtype=np.float64)
        geo = self._static_geo()
        Ut = np.einsum("k...,ik...->i...", u, geo.gco)
        self.N = _c.consistent_equilibrium(geo, self.tau, rho, Ut)
        self.t = 0
        return self.N

    def step(self, coords_next, wrap_next=None):
        """N(t) -> N(t + 1) with the mesh moving from x(q, t) to x(q, t + 1)."""
        lat, d = self.lat, self.d
        mesh_next = Mesh(lat, self.n, coords_next, self.faces,
                         self.mesh.wrap if wrap_next is None else wrap_next, self.dx)
        box_next = basis(mesh_next)
        gco = real(self.box["gco"], 2, d, lat.speed)
        Ap, Am = link_coefficients(lat, self.box_prev["g"], self.box["g"], box_next["g"], gco, d)
        geo = _Geo(lat, self.box, Ap, self.G, d)
        Np, info = _c.collide(geo, self.tau, self.N, self.tol, self.max_iter, A_in=Am)
        if not info["converged"]:
            raise RuntimeError("collision fixed point did not converge")
        self.N = stream(self.mesh, Np, None, self.src)
        self.box_prev, self.box, self.mesh = self.box, box_next, mesh_next
        self.t += 1
        return info

    def incoming(self):
        """A- of the current state (the arrivals of the last step)."""
        lat, d = self.lat, self.d
        gco = real(self.box["gco"], 2, d, lat.speed)
        _, Am = link_coefficients(lat, self.box_prev["g"], self.box["g"], self.box["g"], gco, d)
        return Am

    def momentum_I(self):
        """I(t) = sum_q g_i(q, t) sum_a (c_a^i - A-^i_a / 2) N_a(q, t)."""
        lat, d = self.lat, self.d
        g = real(self.box["g"], 2, d, lat.speed)
        inner = np.einsum("ai,a...->i...", lat.cf, self.N) - 0.5 * np.einsum("ai...,a...->i...",
                                                                            self.incoming(), self.N)
        return np.einsum("i...,ik...->k...", inner, g).reshape(d, -1).sum(axis=1)

    def mass(self):
        return float(self.N.sum())

    def moments(self):
        """rho and Euclidean u = Ut^i g_i at time t, the mesh taken as
        momentarily at rest."""
        geo = self._static_geo()
        _, info = _c.collide(geo, self.tau, self.N, self.tol, self.max_iter)
        u = np.einsum("i...,ik...->k...", info["Ut"], geo.g)
        return {"rho": info["rho"], "u": u, "U": info["U"], "Ut": info["Ut"]}
