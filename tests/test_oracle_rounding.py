"""The rest-state compensation of rounded link coefficients (the library's
precision reading for FP32 coefficient words, eq. (compo-constr)), checked
with the oracle on the CPU: rounding A to FP32 alone pushes a fluid at rest,
and storing a_ext - kappa with
    kappa^i = -1/2 sum_a (dA^i_a + dA^i_opp(a)) f^eq_a(rho = 1, U = Ut = 0)
takes that push away up to terms of second order in the velocity."""
import numpy as np

from oracle import collide as OC
from oracle import stream as OS
from oracle.equilibrium import feq
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import sim_of


def _f32(x):
    return x.astype(np.float32).astype(np.float64)


def _velocity_after(w, steps, mode):
    """Euclidean velocity after `steps` steps from rest with the exact
    coefficients ("exact"), FP32-rounded ones ("rounded") or rounded ones with
    the compensated a_ext ("compensated")."""
    s = sim_of(w)
    shape = s.mesh.shape
    s.init(np.ones(shape), np.zeros((s.mesh.d,) + shape))
    g = s.geom
    if mode != "exact":
        A = g.A.copy()
        g.A = _f32(A)
        if mode == "compensated":
            zero = np.zeros((s.mesh.d,) + shape)
            f = feq(g.lat, np.ones(shape), zero, zero, g.gup)
            dA = g.A - A
            kappa = -0.5 * np.einsum("ai...,a...->i...", dA + dA[g.lat.opp], f)
            g.aext = g.aext - kappa
    for _ in range(steps):
        Np, _ = OC.collide(g, s.p.tau, s.N)
        s.N = OS.stream(s.mesh, Np, s.N_inf, s.src)
    out = sim_of(w)
    out.N = s.N
    return out.moments()["u"]


import pytest


@pytest.mark.parametrize("w", [W.tanh_channel_3d(8, 32, 4, strength=1.0, tau=0.6, G=0.0),
                               W.wavy_periodic("D2Q9", (16, 16), 0.1)], ids=["tanh(1) channel", "wavy D2Q9"])
def test_compensation_removes_the_rest_state_push_of_rounded_coefficients(w):
    """Ten steps from the consistent equilibrium at rest on stretched meshes
    that the exact method keeps near rest (its mesh-truncation currents stay
    below 5e-3; measured 5.9e-5 and 1.7e-3): FP32 coefficients push the
    velocity away from the exact run,
    and the compensated a_ext takes at least 90 % of that push away (measured:
    65x and 125x smaller).  What is left comes from the non-equilibrium part
    of the truncation currents, which the rest-state derivation leaves out."""
    steps = 10
    u_exact = _velocity_after(w, steps, "exact")
    u_rounded = _velocity_after(w, steps, "rounded")
    u_comp = _velocity_after(w, steps, "compensated")
    push = np.abs(u_rounded - u_exact).max()
    left = np.abs(u_comp - u_exact).max()
    print(w["name"], "|u| exact", np.abs(u_exact).max(), "push of rounded A", push, "compensated", left)
    assert np.abs(u_exact).max() < 5e-3
    assert push > 1e-11                      # FP32 coefficients do push the fluid
    assert left < 0.1 * push                 # the compensation takes the push away
