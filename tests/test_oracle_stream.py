"""Pins for oracle.stream (eq. (adv)): a permutation, identity after a period."""
import numpy as np
import pytest

from oracle import stream as S
from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import mesh_of, sim_of


@pytest.mark.parametrize("wl", [W.tanh_channel_2d(6, 5), W.wavy_channel_3d(5, 4, 3),
                                W.wavy_periodic("D3Q19", (4, 5, 3), 0.1), W.wavy_periodic("D2Q21", (5, 4), 0.1),
                                W.wavy_periodic("D3Q39", (4, 5, 3), 0.1),
                                W.tanh_channel_2d(6, 7, strength=0.3, lattice="D2Q21", dx_ratio=1.0),
                                W.tanh_channel_3d(5, 7, 4, strength=0.3, lattice="D3Q39", dx_ratio=1.0)],
                         ids=lambda w: w["name"])
def test_stream_is_a_permutation(wl):
    """Every post-collision population lands in exactly one slot, also with the
    multi-cell bounce-back of the long-link lattices (a wrong mirror source
    would send two links to one slot)."""
    m = mesh_of(wl)
    ids = np.arange(m.lat.Q * m.ncells, dtype=np.float64).reshape((m.lat.Q,) + m.shape)
    out = S.stream(m, ids)
    assert np.array_equal(np.sort(out.ravel()), ids.ravel())


@pytest.mark.parametrize("lat,n", [("D2Q9", (7, 7)), ("D3Q19", (5, 5, 5)), ("D2Q21", (7, 7)), ("D3Q39", (5, 5, 5))])
def test_period_of_pure_streaming_is_identity(lat, n):
    wl = W.wavy_periodic(lat, n, 0.1)
    s = sim_of(wl, stream_only=True)
    rng = np.random.default_rng(0)
    N0 = rng.random((s.lat.Q,) + s.mesh.shape)
    s.set_state(N0)
    s.step(n[0])
    assert np.array_equal(s.N, N0)
    s.step(1)
    assert not np.array_equal(s.N, N0)


def test_bounce_back_period_in_a_channel():
    """Periodic x (8 cells), walls on y (4 cells): every population returns to its
    slot after lcm(8, 2*4) = 8 pure-streaming steps, bit for bit."""
    wl = W.tanh_channel_2d(8, 4)
    s = sim_of(wl, stream_only=True)
    rng = np.random.default_rng(1)
    N0 = rng.random((9,) + s.mesh.shape)
    s.set_state(N0)
    s.step(8)
    assert np.array_equal(s.N, N0)


@pytest.mark.parametrize("lat_name,n", [("D2Q9", (6, 5)), ("D3Q19", (4, 5, 3))])
def test_uniform_far_field_state_is_steady(lat_name, n):
    """Far-field reading pinned by an invariant: on a uniform (sheared) lattice
    Theta = 0, so a uniform state rho_inf, u_inf is a fixed point of the interior
    update, and the populations imposed on far-field links must be exactly the
    ones that state streams in; twenty steps leave it unchanged."""
    from paper_2401_17183_amd import workloads as W
    from tests.oracle_helpers import sim_of
    d = len(n)
    A = np.eye(d) + 0.15 * np.roll(np.eye(d), 1, axis=1)
    w = W.affine_mesh(lat_name, n, A, periodic=False)
    w["faces"] = [f if i != 1 else (W.FARFIELD, W.FARFIELD) for i, f in enumerate(w["faces"])]
    w["rho_inf"] = 1.02
    w["u_inf"] = tuple([0.03, -0.02, 0.01][:d])
    s = sim_of(w)
    rho = np.full(s.mesh.shape, 1.02)
    u = np.broadcast_to(np.array(w["u_inf"]).reshape((d,) + (1,) * d), (d,) + s.mesh.shape).copy()
    s.init(rho, u)
    N0 = s.N.copy()
    s.step(20)
    assert np.max(np.abs(s.N - N0)) <= 1e-14 * np.max(np.abs(N0))
    m = s.moments()
    assert np.allclose(m["u"], u, rtol=0, atol=1e-14)
