"""Pins for the moving-mesh reading (oracle.moving): reductions to the static
method, the two conservation laws on deforming and rotating meshes, the
behaviour of resting and uniform flows on a rigidly rotating uniform mesh,
and planted mistakes that must break the momentum balance."""
import numpy as np
import pytest

from oracle import lattice, moving
from oracle import geometry as OG
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import sim_of

CASES = [("D2Q9", (10, 12), 0.2), ("D3Q19", (6, 5, 7), 0.1)]


def _wavy(name, n, amp):
    w = W.wavy_periodic(name, n, amp)
    w["tau"] = 0.7
    return w


def _moving(w, **motion):
    lat = lattice.by_name(w["lattice"])
    X0, wr0 = W.moving_coords(w, 0, **motion)
    ms = moving.MovingSim(lat, w["n"], X0, wr0, w["dx"], w["tau"], body_force=w.get("body_force"))
    return ms


def _state(ms, seed=3):
    rng = np.random.default_rng(seed)
    m = ms.mesh
    rho = 1.0 + 0.02 * rng.standard_normal(m.shape)
    u = 0.02 * rng.standard_normal((m.d,) + m.shape)
    return rho, u


def _run(w, steps, **motion):
    ms = _moving(w, **motion)
    ms.init(*_state(ms))
    for t in range(steps):
        ms.step(*W.moving_coords(w, t + 1, **motion))
    return ms


@pytest.mark.parametrize("name,n,amp", CASES)
def test_static_mesh_is_the_static_method(name, n, amp):
    """x(q, t) = x(q, 0): A+ = A and A- = A_opp, so the step is the static one."""
    w = _wavy(name, n, amp)
    ms = _run(w, 6)
    s = sim_of(w)
    s.init(*_state(ms))
    s.step(6)
    J = s.geom.J
    assert np.max(np.abs(ms.N - s.N) / J) <= 1e-15


@pytest.mark.parametrize("name,n,amp", CASES)
def test_rigid_translation_is_the_static_method(name, n, amp):
    """A mesh shifted by V t keeps its tangent vectors: the same result as the
    static mesh, up to the rounding of the shifted node positions."""
    w = _wavy(name, n, amp)
    ms = _run(w, 6, velocity=[0.3, -0.2, 0.1])
    s = sim_of(w)
    s.init(*_state(ms))
    s.step(6)
    assert np.max(np.abs(ms.N - s.N) / s.geom.J) <= 1e-12


@pytest.mark.parametrize("name,n,amp", CASES)
@pytest.mark.parametrize("G", [None, (2e-4, -1e-4, 5e-5)])
def test_mass_and_mid_link_momentum_on_a_deforming_mesh(name, n, amp, G):
    """Mass is conserved and I(t + 1) = I(t) + G mass, to roundoff, while the
    mesh deforms (its waviness breathes by 30 %) and turns."""
    w = _wavy(name, n, amp)
    if G is not None:
        w["body_force"] = G[: len(n)]
    motion = dict(breathe=0.3, omega=0.01, period=12.0)
    ms = _moving(w, **motion)
    ms.init(*_state(ms))
    Gv = np.zeros(len(n)) if G is None else np.asarray(G[: len(n)])
    m0 = ms.mass()
    I_prev = ms.momentum_I()
    for t in range(12):
        mass = ms.mass()
        ms.step(*W.moving_coords(w, t + 1, **motion))
        I = ms.momentum_I()
        assert abs(ms.mass() / m0 - 1) <= 1e-14
        bal = I - I_prev - Gv * mass
        assert np.max(np.abs(bal)) <= 1e-13 * mass, (t, bal)
        I_prev = I


@pytest.mark.parametrize("mistake", ["static", "outgoing_from_now", "incoming_from_now", "swapped_times"])
def test_planted_time_level_mistakes_break_the_balance(monkeypatch, mistake):
    """The coefficients must take e_a at the time the particle has it: the
    static coefficients of the time t mesh (the motion ignored), the time t
    mesh for the neighbour's t + 1 or t - 1 position, or the two swapped, each
    break the mid-link momentum balance on a deforming mesh."""
    real = moving.link_coefficients

    def planted(lat, box_prev, box_cur, box_next, gco_cur, d):
        if mistake == "static":
            return real(lat, box_cur, box_cur, box_cur, gco_cur, d)
        if mistake == "outgoing_from_now":
            return real(lat, box_prev, box_cur, box_cur, gco_cur, d)
        if mistake == "incoming_from_now":
            return real(lat, box_cur, box_cur, box_next, gco_cur, d)
        return real(lat, box_next, box_cur, box_prev, gco_cur, d)

    w = _wavy("D2Q9", (10, 12), 0.2)
    motion = dict(breathe=0.3, omega=0.01, period=12.0)
    ms = _moving(w, **motion)
    ms.init(*_state(ms))
    monkeypatch.setattr(moving, "link_coefficients", planted)
    worst = 0.0
    I_prev = real_I(ms, real)
    for t in range(6):
        ms.step(*W.moving_coords(w, t + 1, **motion))
        I = real_I(ms, real)
        worst = max(worst, float(np.max(np.abs(I - I_prev))) / ms.mass())
        I_prev = I
    assert worst > 1e-8, worst


def real_I(ms, real):
    """I(t) with the correct incoming coefficients (whatever the step used)."""
    lat, d = ms.lat, ms.d
    gco = OG.real(ms.box["gco"], 2, d, lat.speed)
    g = OG.real(ms.box["g"], 2, d, lat.speed)
    _, Am = real(lat, ms.box_prev["g"], ms.box["g"], ms.box["g"], gco, d)
    inner = np.einsum("ai,a...->i...", lat.cf, ms.N) - 0.5 * np.einsum("ai...,a...->i...", Am, ms.N)
    return np.einsum("i...,ik...->k...", inner, g).reshape(d, -1).sum(axis=1)


@pytest.mark.parametrize("name,n", [("D2Q9", (10, 12)), ("D3Q19", (6, 5, 7))])
def test_rotating_uniform_mesh_rest_and_uniform_flow(name, n):
    """A uniform mesh in rigid rotation: a fluid at rest stays at rest, and a
    uniform Euclidean flow stays uniform and steady in the Euclidean frame
    (its reported velocity does not change in time) while the mesh turns by
    0.02 per step."""
    d = len(n)
    w = W.affine_mesh(name, n, np.eye(d) + 0.1 * np.eye(d)[::-1])
    w["tau"] = 0.8
    motion = dict(omega=0.02)
    rest = _moving(w, **motion)
    rest.init()
    flow = _moving(w, **motion)
    V = np.array([0.03, -0.02, 0.01][:d])
    flow.init(None, np.zeros((d,) + flow.mesh.shape) + V.reshape((d,) + (1,) * d))
    u_prev = None
    for t in range(30):
        X, wr = W.moving_coords(w, t + 1, **motion)
        rest.step(X, wr)
        flow.step(X, wr)
        if t % 10 == 9:
            assert np.max(np.abs(rest.moments()["u"])) <= 1e-14
            u = flow.moments()["u"].reshape(d, -1)
            assert np.max(np.abs(u - u.mean(axis=1, keepdims=True))) <= 1e-14
            if u_prev is not None:
                assert np.max(np.abs(u - u_prev)) <= 1e-12
            u_prev = u
