"""System pins for the oracle: exact conservation, the Cartesian reduction,
and hydrodynamics (Poiseuille on a stretched mesh, shear-wave viscosity)."""
import numpy as np
import pytest

from oracle import collide as C
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import near_equilibrium_state, sim_of


@pytest.mark.parametrize("tau_g", [None, 1.0], ids=["bgk", "regularised"])
@pytest.mark.parametrize("wl", [W.tanh_channel_2d(8, 16), W.wavy_channel_3d(8, 8, 6),
                                W.tanh_channel_2d(6, 12, strength=0.3, lattice="D2Q21", dx_ratio=1.0),
                                W.tanh_channel_3d(5, 8, 4, strength=0.3, tau=0.8, lattice="D3Q39", dx_ratio=1.0)],
                         ids=lambda w: w["name"])
def test_mass_and_mid_link_momentum_balance(wl, tau_g):
    """Mass is exact; I(t+1) = I(t) + G * mass + W(t) (derived from
    eq. (constraints) and eq. (adv)), to roundoff, every step; with BGK and with
    the general collision matrix."""
    s = sim_of(wl, tau_g=tau_g)
    near_equilibrium_state(s, amp=1e-3)
    M0 = s.N.sum()
    I0 = s.momentum_I()
    for _ in range(5):
        s.step()
        I1 = s.momentum_I()
        bal = I1 - I0 - s.geom.G * M0 - s.wall_impulse()
        assert np.max(np.abs(bal)) < 1e-13 * s.N.sum()
        assert abs(s.N.sum() / M0 - 1) < 1e-14
        I0 = I1


def test_naive_momentum_is_not_the_conserved_one():
    """P = sum e_a N_a is not conserved on a curvilinear mesh (eq. (momentum));
    the mid-link I is."""
    s = sim_of(W.wavy_periodic("D2Q9", (10, 12), 0.25))
    near_equilibrium_state(s, amp=1e-2)
    def P():
        e = np.einsum("ai,ik...->ak...", s.lat.cf, s.geom.g)
        return np.einsum("ak...,a...->k...", e, s.N).reshape(2, -1).sum(1)
    P0, I0 = P(), s.momentum_I()
    s.step(3)
    assert np.max(np.abs(s.momentum_I() - I0)) < 1e-12
    assert np.max(np.abs(P() - P0)) > 1e-6


def textbook_bgk(N, c, w, tau, steps, t0=1.0 / 3.0):
    """An independent plain BGK with the third-order Hermite equilibrium on a
    uniform periodic lattice (unit spacing), lattice temperature t0."""
    d = c.shape[1]
    for _ in range(steps):
        rho = N.sum(0)
        u = np.einsum("ai,a...->i...", c, N) / rho
        cu = np.einsum("ai,i...->a...", c, u)
        u2 = np.sum(u * u, axis=0)[None]
        fe = w.reshape((-1,) + (1,) * d) * rho[None] * (1 + cu / t0 + cu ** 2 / (2 * t0 ** 2) - u2 / (2 * t0)
                                                        + cu ** 3 / (6 * t0 ** 3) - cu * u2 / (2 * t0 ** 2))
        Np = N - (N - fe) / tau
        N = np.stack([np.roll(Np[a], shift=tuple(int(v) for v in c[a][::-1]), axis=tuple(range(d)))
                      for a in range(len(w))])
    return N


@pytest.mark.parametrize("lat,n", [("D2Q9", (9, 7)), ("D3Q19", (6, 5, 4)), ("D2Q21", (9, 7)), ("D3Q39", (6, 5, 4))])
def test_cartesian_reduction_to_textbook_bgk(lat, n):
    """On a uniform Cartesian lattice (g^{ij} = delta, Theta = 0) the scheme is the
    standard LBM (remark after eq. (equilibrium)), with the lattice's T0."""
    wl = W.affine_mesh(lat, n, np.eye(len(n)))
    s = sim_of(wl, tau=0.7)
    N0 = near_equilibrium_state(s, amp=1e-2)
    ref = textbook_bgk(N0.copy(), s.lat.cf, s.lat.w, 0.7, 10, s.lat.T0)
    s.step(10)
    assert np.max(np.abs(s.N - ref)) < 1e-15


def poiseuille_hold_error(n2, steps=2000):
    wl = W.tanh_channel_2d(4, n2)
    s = sim_of(wl)
    rho, u = W.poiseuille_fields(wl)
    s.init(rho, u)
    s.step(steps)
    m = s.moments()
    return np.linalg.norm(m["u"][0] - u[0]) / np.linalg.norm(u[0])


def test_poiseuille_holds_on_stretched_mesh_and_converges():
    """Plane Poiseuille u = G (H^2 - y^2) / (2 nu) with nu = (tau - 1/2) T0 (Sec. 3,
    eq. (NS)): started at the analytic profile on the tanh-stretched mesh, the
    profile holds; the departure after 2000 steps falls at least at second
    order under refinement of the wall-normal axis."""
    e = [poiseuille_hold_error(n2) for n2 in (16, 32, 64)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
    assert e[1] < 3e-3, e


def test_poiseuille_with_multi_cell_walls_converges():
    """D2Q21 (links up to three cells, multi-cell halfway bounce-back) holds the
    analytic Poiseuille profile, nu = (tau - 1/2) 2/3, on a mildly stretched
    channel, with second-order convergence under wall-normal refinement."""
    e = []
    for n2 in (16, 32, 64):
        wl = W.tanh_channel_2d(4, n2, strength=0.3, lattice="D2Q21", dx_ratio=1.0)
        s = sim_of(wl)
        rho, u = W.poiseuille_fields(wl)
        s.init(rho, u)
        s.step(2000)
        e.append(np.linalg.norm(s.moments()["u"][0] - u[0]) / np.linalg.norm(u[0]))
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
    assert e[2] < 1e-3, e


def test_poiseuille_needs_the_inertial_force(monkeypatch):
    """Planted mistake: without the inertial force the same run leaves the
    analytic profile by orders of magnitude more."""
    good = poiseuille_hold_error(32, steps=300)
    zero = lambda lat, J, A, N, Np, A_in=None: np.zeros((lat.d,) + J.shape)
    monkeypatch.setattr(C, "inertial_force", zero)
    bad = poiseuille_hold_error(32, steps=300)
    assert bad > 30 * good, (good, bad)


def shear_wave_rate(wl, steps=200, u0=1e-3, tau_g=None):
    """Decay rate of a shear wave u_x = u0 sin(k y), measured on the difference
    from a run started at rest on the same mesh (which removes the small
    stationary truncation-error currents of a curvilinear mesh)."""
    runs = []
    for amp in (u0, 0.0):
        s = sim_of(wl, tau_g=tau_g)
        m = s.mesh
        L = m.n[1] * m.dx
        y = m.coords[..., 1]
        k = 2 * np.pi / L
        u = np.zeros((2,) + m.shape)
        u[0] = amp * np.sin(k * y)
        s.init(None, u)
        s.step(50)   # skip the initial layer of an equilibrium start
        us = [s.moments()["u"][0]]
        s.step(steps)
        us.append(s.moments()["u"][0])
        runs.append(us)
    J = s.geom.J
    amps = [np.sum(J * (runs[0][t] - runs[1][t]) * np.sin(k * y)) / np.sum(J * np.sin(k * y) ** 2)
            for t in (0, 1)]
    return -np.log(amps[1] / amps[0]) / steps / (k / m.dx) ** 2


@pytest.mark.parametrize("lat,n,amp,tol,tau_g", [("D2Q9", 48, 0.0, 3e-3, None), ("D2Q9", 32, 0.2, 2e-2, None),
                                                  ("D2Q9", 48, 0.0, 3e-3, 1.0), ("D2Q9", 32, 0.2, 2e-2, 1.0),
                                                  ("D2Q21", 48, 0.0, 3e-3, None), ("D2Q21", 32, 0.2, 2e-2, None)])
def test_shear_wave_viscosity(lat, n, amp, tol, tau_g):
    """A decaying shear wave has nu = (tau - 1/2) T0 (Sec. 3, mu = (tau - 1/2) rho T0),
    on a Cartesian and on a wavy curvilinear periodic mesh; with the general
    collision matrix too, whose stress relaxes at 1/tau by eq. (matrix); and on
    the sixth-order lattice, whose T0 is 2/3."""
    from oracle import lattice
    wl = W.wavy_periodic(lat, (n, n), amp)
    nu_meas = shear_wave_rate(wl, tau_g=tau_g)
    nu = (wl["tau"] - 0.5) * lattice.by_name(lat).T0
    assert abs(nu_meas / nu - 1) < tol, nu_meas / nu
