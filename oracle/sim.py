"""Time stepping, initial state, output mapping and audits (Sec. 2.2).

State: the arrived populations N(t) (after advection, before collision).
One step: N'(t) = collide(N(t)); N(t + 1) = stream(N'(t)).

Readings (the paper specifies none of these):
* initial state: N(0) = J f^eq(rho, U, Ut) with Ut^i = u . g^i the prescribed
  Euclidean velocity and U chosen so that the collision fixed point of N(0)
  reproduces that Ut (collide.consistent_equilibrium);
* far-field populations: N_inf_a(q) = J f^eq_a(rho_inf, U_inf, U_inf) with
  U_inf^i = u_inf . g^i(q);
* output mapping: eq. (result) maps rho and U^i g_i; the velocity that obeys the
  continuity and Navier-Stokes equations of Sec. 3 is the shifted one, so the
  reported velocity is u = Ut^i g_i, with U returned beside it;
* audits: total mass sum N; the mid-link Euclidean momentum
      I(t) = sum_q g_i(q) sum_a (c^i_a - A^i_opp(a)(q) / 2) N_a(q, t)
           = 1/2 sum_q sum_a [e_a(q) + e_a(q - c_a)] N_a(q, t),
  which the method conserves up to the body-force impulse G * mass and the
  impulse W taken by bounced links,
      W(t - 1) = sum_{bounced (q, a)} g_i(q) (2 c^i_a - A^i_opp(a)(q)) N_a(q, t)
  (derived from eq. (constraints) and eq. (adv)).
"""
import numpy as np

from . import collide as _c
from .equilibrium import feq
from .geometry import Geometry
from .stream import FARFIELD, WALL, sources, stream


class Params:
    def __init__(self, tau, body_force=None, rho_inf=1.0, u_inf=None, tol=1e-14,
                 max_iter=50, stream_only=False, tau_g=None):
        self.tau = float(tau)
        self.tau_g = None if tau_g is None else float(tau_g)   # None: BGK
        self.body_force = body_force
        self.rho_inf = float(rho_inf)
        self.u_inf = u_inf
        self.tol = float(tol)
        self.max_iter = int(max_iter)
        self.stream_only = bool(stream_only)


class Sim:
    def __init__(self, mesh, params, geom=None):
        self.mesh = mesh
        self.lat = mesh.lat
        self.p = params
        self.geom = geom if geom is not None else Geometry(mesh, params.body_force)
        self.src = sources(mesh)
        self.t = 0
        self.N = None
        self.u_prev = None
        self.N_inf = None
        if any(FARFIELD in f for f in mesh.faces):
            d = mesh.d
            uinf = np.zeros(d) if params.u_inf is None else np.asarray(params.u_inf, dtype=np.float64)[:d]
            Uinf = np.einsum("k,ik...->i...", uinf, self.geom.gco)
            rinf = np.full(mesh.shape, params.rho_inf)
            self.N_inf = self.geom.J[None] * feq(self.lat, rinf, Uinf, Uinf, self.geom.gup)

    def _impose_farfield(self, N):
        if self.N_inf is None:
            return N
        for a in range(self.lat.Q):
            _, kind = self.src[a]
            N[a] = np.where(kind == FARFIELD, self.N_inf[a], N[a])
        return N

    def init(self, rho=None, u=None):
        """rho (*n) and Euclidean u (d, *n); defaults rho = 1, u = 0."""
        m = self.mesh
        rho = np.ones(m.shape) if rho is None else np.asarray(rho, dtype=np.float64)
        u = np.zeros((m.d,) + m.shape) if u is None else np.asarray(u, dtype=np.float64)
        Ut = np.einsum("k...,ik...->i...", u, self.geom.gco)
        N = _c.consistent_equilibrium(self.geom, self.p.tau, rho, Ut)
        self.N = self._impose_farfield(N)
        self.t = 0
        self.u_prev = None
        return self.N

    def set_state(self, N):
        """Replace the arrived populations; far-field links keep their imposed
        value (they carry no information from inside the mesh)."""
        self.N = self._impose_farfield(np.array(N, dtype=np.float64, copy=True))

    def step(self, n=1):
        info = None
        for _ in range(n):
            if self.p.stream_only:
                Np = self.N
            else:
                Np, info = _c.collide(self.geom, self.p.tau, self.N, self.p.tol, self.p.max_iter, self.p.tau_g)
                if not info["converged"]:
                    raise RuntimeError("collision fixed point did not converge")
            self.N = stream(self.mesh, Np, self.N_inf, self.src)
            self.t += 1
        return info

    def moments(self):
        """rho, Euclidean u = Ut^i g_i, contravariant U and Ut, fixed-point iters."""
        _, info = _c.collide(self.geom, self.p.tau, self.N, self.p.tol, self.p.max_iter, self.p.tau_g)
        u = np.einsum("i...,ik...->k...", info["Ut"], self.geom.g)
        return {"rho": info["rho"], "u": u, "U": info["U"], "Ut": info["Ut"],
                "F": info["F"], "iters": info["iters"]}

    def momentum_I(self):
        g, A, c, opp = self.geom.g, self.geom.A, self.lat.cf, self.lat.opp
        inner = np.einsum("ai,a...->i...", c, self.N) - 0.5 * np.einsum("ai...,a...->i...", A[opp], self.N)
        d = self.mesh.d
        return np.einsum("i...,ik...->k...", inner, g).reshape(d, -1).sum(axis=1)

    def wall_impulse(self):
        """W of the step that produced the current state: per bounced link
        (q, a) with source cell q_s, the arriving mid-link momentum minus the
        departing one, g_i(q) (c^i_a - A^i_opp(a)(q)/2) N_a(q) + g_i(q_s)
        (c^i_a - A^i_opp(a)(q_s)/2) N_a(q); for one-cell links q_s = q and
        this is g_i(q) (2 c^i_a - A^i_opp(a)(q)) N_a(q)."""
        g, A, c, opp = self.geom.g, self.geom.A, self.lat.cf, self.lat.opp
        d = self.mesh.d
        gf = g.reshape(d, d, -1)
        Af = A.reshape(A.shape[0], d, -1)
        tot = np.zeros(d)
        for a in range(self.lat.Q):
            src, kind = self.src[a]
            m = (kind == WALL).ravel()
            if not np.any(m):
                continue
            qs = src.ravel()[m]
            qq = np.arange(self.mesh.ncells)[m]
            n = self.N[a].ravel()[m]
            here = c[a][:, None] - 0.5 * Af[opp[a]][:, qq]      # (i, links)
            there = c[a][:, None] - 0.5 * Af[opp[a]][:, qs]
            vec = np.einsum("il,ikl->kl", here, gf[:, :, qq]) + np.einsum("il,ikl->kl", there, gf[:, :, qs])
            tot += np.sum(vec * n[None], axis=1)
        return tot

    def audit(self):
        mom = self.moments()
        u = mom["u"]
        if self.u_prev is None:
            resid = float("nan")
        else:
            resid = float(np.linalg.norm(u - self.u_prev) / np.linalg.norm(u))
        self.u_prev = u.copy()
        mass = float(self.N.sum())
        return {
            "step": self.t, "mass": mass, "mom_I": self.momentum_I(),
            "wall_impulse": self.wall_impulse(),
            "force_impulse": self.geom.G * mass,
            "residual": resid, "max_fp_iters": int(mom["iters"].max()),
            "nonfinite": int(np.sum(~np.isfinite(self.N))),
            "negative": int(np.sum(self.N < 0)),
        }
