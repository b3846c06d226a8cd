"""Pins for the initial-state reading (oracle.collide.consistent_equilibrium).

The paper gives no initial state.  The reading: N(0) = J f^eq(rho, U, Ut) with
the prescribed Euclidean velocity u entering as the shifted velocity
Ut^i = u . g^i (the velocity of the continuity and Navier-Stokes equations of
Sec. 3), and U = Ut - F_tot / (2 rho) chosen so that the collision fixed point
of N(0) (eq. (compo-constr) with the shift Ut = U + a/2 stated after
eq. (equilmoments)) returns that same Ut.

Its defining property is checked here against the collision itself: on
curvilinear meshes where the inertial force is far from zero, colliding N(0)
returns the prescribed rho and Ut, and the output mapping (eq. (result) with
the shifted velocity) returns the prescribed Euclidean u.  Planted mistakes
(the sign of the F / (2 rho) shift flipped, the body force left out of F_tot,
the shift dropped altogether) must each break that property.
"""
import numpy as np
import pytest

from oracle import collide as OC
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import sim_of

CASES = [W.wavy_channel_3d(8, 8, 6, G=1e-3), W.tanh_channel_3d(10, 16, 6, G=1e-3),
         W.tanh_channel_2d(12, 16, G=1e-3), W.wavy_periodic("D2Q9", (10, 12), 0.2),
         W.wavy_periodic("D3Q39", (6, 5, 7), 0.08)]


def prescribed(s, seed=5):
    rng = np.random.default_rng(seed)
    m = s.mesh
    rho = 1.0 + 0.03 * rng.standard_normal(m.shape)
    u = 0.02 * rng.standard_normal((m.d,) + m.shape)
    return rho, u


def init_error(s, rho, u):
    """Largest deviation of what the collision of N(0) returns from what was
    prescribed: (rho error, Ut error, Euclidean u error, max |F|)."""
    s.init(rho, u)
    Ut = np.einsum("k...,ik...->i...", u, s.geom.gco)
    _, info = OC.collide(s.geom, s.p.tau, s.N)
    assert info["converged"]
    mo = s.moments()
    return (float(np.max(np.abs(info["rho"] - rho))), float(np.max(np.abs(info["Ut"] - Ut))),
            float(np.max(np.abs(mo["u"] - u))), float(np.max(np.abs(info["F"]))))


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w["name"])
def test_initial_state_reproduces_prescribed_fields(wl):
    s = sim_of(wl)
    rho, u = prescribed(s)
    e_rho, e_ut, e_u, fmax = init_error(s, rho, u)
    print(wl["name"], "rho", e_rho, "Ut", e_ut, "u", e_u, "max|F|", fmax)
    # the reading only means something where the inertial force is not small
    assert fmax > 1e-3, fmax
    assert e_rho <= 1e-13
    assert e_ut <= 1e-13
    assert e_u <= 1e-13


def _planted(monkeypatch, kind):
    """Plant one mistake in the oracle's initial state (the collision used to
    check it stays correct)."""
    real = OC.consistent_equilibrium
    real_feq = OC.feq

    def flipped(geom, tau, rho, Ut, tol=1e-14, max_iter=50):
        # U = Ut + F_tot / (2 rho) instead of Ut - F_tot / (2 rho)
        def feq_flip(lat, rho_, U, Ut_, gup):
            return real_feq(lat, rho_, 2.0 * Ut_ - U, Ut_, gup)
        monkeypatch.setattr(OC, "feq", feq_flip)
        try:
            return real(geom, tau, rho, Ut, tol, max_iter)
        finally:
            monkeypatch.setattr(OC, "feq", real_feq)

    def no_body_force(geom, tau, rho, Ut, tol=1e-14, max_iter=50):
        aext = geom.aext
        geom.aext = np.zeros_like(aext)
        try:
            return real(geom, tau, rho, Ut, tol, max_iter)
        finally:
            geom.aext = aext

    def no_shift(geom, tau, rho, Ut, tol=1e-14, max_iter=50):
        return geom.J[None] * real_feq(geom.lat, rho, Ut, Ut, geom.gup)

    monkeypatch.setattr(OC, "consistent_equilibrium", {"flipped": flipped, "no_body_force": no_body_force,
                                                       "no_shift": no_shift}[kind])


@pytest.mark.parametrize("kind", ["flipped", "no_body_force", "no_shift"])
def test_planted_initial_state_mistakes_are_caught(monkeypatch, kind):
    wl = W.wavy_channel_3d(8, 8, 6, G=1e-3)
    s = sim_of(wl)
    rho, u = prescribed(s)
    _planted(monkeypatch, kind)
    e_rho, e_ut, e_u, fmax = init_error(s, rho, u)
    print(kind, "rho", e_rho, "Ut", e_ut, "u", e_u)
    assert max(e_ut, e_u) > 1e-8, (kind, e_ut, e_u)
