"""Pins for oracle.collide (Sec. 2.2): conservation, the moment constraints on
dN, the mid-link momentum identity and the continuum limit of dPi."""
import numpy as np
import pytest

from oracle import collide as C
from oracle import geometry, lattice
from oracle.equilibrium import feq
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import near_equilibrium_state, sim_of
from tests.test_oracle_geometry import central_gamma, refine_wavy

CASES = [W.wavy_channel_3d(8, 8, 6), W.tanh_channel_2d(12, 16), W.wavy_periodic("D2Q9", (10, 12), 0.2)]


def converged_pieces(s, N):
    Np, info = C.collide(s.geom, s.p.tau, N)
    assert info["converged"]
    g = s.geom
    lat = s.lat
    rho, U, Ut, F = info["rho"], info["U"], info["Ut"], info["F"]
    fe = feq(lat, rho, U, Ut, g.gup)
    Om = -(N - g.J[None] * fe) / s.p.tau
    dN = Np - N - Om
    Ft = F + rho[None] * g.aext
    dPi = C.delta_pi(lat, s.p.tau, g.A, fe, Ut, rho, g.aext)
    return Np, info, Om, dN, Ft, dPi


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w["name"])
def test_collision_conserves_mass_and_momentum(wl):
    """sum Omega = 0 and sum c Omega = 0 (eqs. (conserv), (omcons))."""
    s = sim_of(wl)
    N = near_equilibrium_state(s)
    _, _, Om, _, _, _ = converged_pieces(s, N)
    scale = np.abs(N).max()
    assert np.max(np.abs(Om.sum(0))) < 1e-14 * scale * s.lat.Q
    assert np.max(np.abs(np.einsum("ai,a...->i...", s.lat.cf, Om))) < 1e-14 * scale * s.lat.Q


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w["name"])
def test_delta_n_moment_constraints(wl):
    """sum dN = 0, sum c dN = J F, sum c c dN = J (dPi + dPi^T) (eqs. (constraints),
    (constraint2), (constraint3))."""
    s = sim_of(wl)
    N = near_equilibrium_state(s)
    _, _, _, dN, Ft, dPi = converged_pieces(s, N)
    c = s.lat.cf
    J = s.geom.J
    scale = np.abs(dN).max() + 1e-300
    assert np.max(np.abs(dN.sum(0))) < 1e-13 * max(scale, 1e-3)
    assert np.allclose(np.einsum("ai,a...->i...", c, dN), J[None] * Ft, rtol=0, atol=1e-14 * J.max())
    second = np.einsum("ai,aj,a...->ij...", c, c, dN)
    assert np.allclose(second, J[None, None] * (dPi + np.swapaxes(dPi, 0, 1)), rtol=0, atol=1e-14 * J.max())


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w["name"])
def test_mid_link_momentum_identity(wl):
    """sum (c + A/2) N' = sum (c - A_opp/2) N + J rho a_ext at the converged fixed
    point; derived from eq. (constraint2) and eq. (compo-constr) (the discrete
    Euclidean momentum conservation the inertial force is built for)."""
    s = sim_of(wl)
    N = near_equilibrium_state(s)
    Np, info, _, _, _, _ = converged_pieces(s, N)
    g = s.geom
    c = s.lat.cf
    lhs = np.einsum("ai,a...->i...", c, Np) + 0.5 * np.einsum("ai...,a...->i...", g.A, Np)
    rhs = (np.einsum("ai,a...->i...", c, N) - 0.5 * np.einsum("ai...,a...->i...", g.A[s.lat.opp], N)
           + g.J[None] * info["rho"][None] * g.aext)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * g.J.max()
    assert np.max(np.abs(info["F"])) > 1e-4  # the mesh is curvilinear: the force is not trivially zero


def test_force_vanishes_on_uniform_lattice():
    """F = 0 on a uniform Cartesian lattice (after eq. (compo-constr))."""
    wl = W.affine_mesh("D3Q19", (5, 4, 6), np.eye(3))
    s = sim_of(wl)
    N = near_equilibrium_state(s)
    _, info = C.collide(s.geom, s.p.tau, N)
    assert np.all(info["F"] == 0)


def test_fixed_point_converges_fast():
    """The map contracts: FP64 convergence within a few tens of iterations on the
    stretched channel (the implicit relation remark after eq. (deltaN))."""
    s = sim_of(W.tanh_channel_2d(16, 32))
    N = near_equilibrium_state(s, amp=1e-3)
    _, info = C.collide(s.geom, s.p.tau, N)
    assert info["converged"] and info["iters"].max() <= 20


def test_delta_pi_continuum_limit():
    """dPi^{ij} -> -(1 - 1/2tau) Gamma^i_kl Q^{jkl,eq} (eq. (delta-fluxb)); the
    symmetrised discrete tensor converges at second order to the symmetrised
    continuum one, with Gamma the centred discrete Christoffel symbol and Q the
    lattice third moment of f^eq."""
    errs = []
    tau = 0.8
    for level in (1, 2):
        m, h = refine_wavy(8, level)
        g = geometry.Geometry(m)
        lat = lattice.D3Q19
        rng = np.random.default_rng(5)
        rho = np.ones(m.shape)
        U = np.zeros((3,) + m.shape) + np.array([0.05, -0.03, 0.02]).reshape(3, 1, 1, 1)
        Ut = U + 0.01
        fe = feq(lat, rho, U, Ut, g.gup)
        dPi = C.delta_pi(lat, tau, g.A, fe, Ut, rho, 0 * g.aext)
        G = central_gamma(m, g.box)
        Q = np.einsum("aj,ak,al,a...->jkl...", lat.cf, lat.cf, lat.cf, fe)
        cont = -(1 - 0.5 / tau) * np.einsum("ikl...,jkl...->ij...", G, Q)
        cont = 0.5 * (cont + np.swapaxes(cont, 0, 1))
        errs.append(np.max(np.abs(dPi - cont)) / np.max(np.abs(cont)))
    assert errs[1] < errs[0] / 3.0, errs
    assert errs[1] < 0.05, errs
