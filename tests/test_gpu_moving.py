"""Steps on a moving mesh (vlbm_step_moving) against the moving-mesh oracle:
FP64 populations within 1e-12 on deforming and rotating periodic meshes, the
audits' mass and mid-link momentum against the oracle's and their balance,
the state's coefficients made when first read, the reduction to the static
step, the calls it rejects, and the benchmarked configuration at full size
(balances every step, reduction to the static step)."""
import numpy as np
import pytest

from oracle import lattice, moving
from paper_2401_17183_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vlbm():
    from paper_2401_17183_amd import vlbm
    return vlbm


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


MOTION = dict(breathe=0.3, omega=0.01, period=12.0)
CASES = [("D2Q9", (12, 10), 0.2, None), ("D2Q9", (12, 10), 0.2, (2e-4, -1e-4)),
         ("D3Q19", (7, 6, 5), 0.1, None), ("D3Q19", (7, 6, 5), 0.1, (2e-4, -1e-4, 5e-5)),
         # rows longer than a block (two x-chunks) and a ragged last y-band of the
         # moving step's block order (bands of 16 rows: 16 + 4)
         ("D3Q19", (70, 20, 6), 0.1, None), ("D2Q9", (300, 20), 0.2, None)]


def _setup(name, n, amp, G, motion, seed=3, audit_every=1):
    v = _vlbm()
    w = W.wavy_periodic(name, n, amp)
    w["tau"] = 0.7
    d = len(n)
    G = (0.0,) * d if G is None else G
    X0, wr0 = W.moving_coords(w, 0, **motion)
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    rho = 1.0 + 0.02 * rng.standard_normal(shape)
    u = 0.02 * rng.standard_normal((d,) + shape)
    lat = lattice.by_name(name)
    o = moving.MovingSim(lat, n, X0, wr0, w["dx"], w["tau"], body_force=G)
    o.init(rho, u)
    m = v.Mesh(name, n, X0, w["faces"], wr0, w["dx"])
    s = v.Sim(m, v.make_params(w["tau"], body_force=G, precision="fp64", audit_every=audit_every),
              rho=rho.ravel(), u=u.reshape(d, -1))
    return w, o, s, m


@pytest.mark.parametrize("name,n,amp,G", CASES, ids=lambda x: str(x))
def test_moving_mesh_fp64_parity_and_balance(name, n, amp, G):
    announce(f"moving mesh {name} {n} G={G}")
    w, o, s, m = _setup(name, n, amp, G, MOTION)
    Q = lattice.by_name(name).Q
    s.audit_now()
    mass0 = o.mass()
    I_o = [o.momentum_I()]
    for t in range(12):
        X, wr = W.moving_coords(w, t + 1, **MOTION)
        s.step_moving(X, wr)
        o.step(X, wr)
        I_o.append(o.momentum_I())
    s.sync()
    J = moving.real(o.box["J"], 0, len(n), 1).ravel()
    err = np.max(np.abs(s.populations().cpu().numpy() - o.N.reshape(Q, -1)) / J)
    print("moving mesh max |f_gpu - f_oracle|", err)
    assert err <= 1e-12
    aud = s.audits()
    assert len(aud) == 13
    for k, a in enumerate(aud):
        assert abs(a["mass"] / mass0 - 1) <= 1e-13
        assert np.allclose(a["mom_I"][: len(n)], I_o[k], rtol=0, atol=1e-12 * mass0), (k, a["mom_I"], I_o[k])
        if k:
            bal = a["mom_I"] - aud[k - 1]["mom_I"] - aud[k - 1]["force_impulse"]
            assert np.max(np.abs(bal)) <= 1e-12 * mass0, (k, bal)
    s.close()
    m.close()


@pytest.mark.parametrize("name,n,amp", [("D2Q9", (12, 10), 0.2), ("D3Q19", (7, 6, 5), 0.1)], ids=str)
def test_state_coefficients_made_when_read(name, n, amp):
    """Moving steps without audits leave the coefficients of the state the
    mesh moved into (its incoming ones, and the mesh's outgoing ones of the
    new positions) to be made when first read: after 6 steps the mid-link
    momentum of an audit matches the oracle's, the moments match the oracle's
    output mapping (the mesh momentarily at rest), and the mesh's A, g_i and J
    match the static geometry of the final positions; static steps then
    continue on the re-packed mesh, conserving mass."""
    announce(f"moving mesh {name} {n}: state coefficients made when read")
    w, o, s, m = _setup(name, n, amp, None, MOTION, audit_every=0)
    Q, d = lattice.by_name(name).Q, len(n)
    for t in range(6):
        X, wr = W.moving_coords(w, t + 1, **MOTION)
        s.step_moving(X, wr)
        o.step(X, wr)
    s.sync()
    mass0 = o.mass()
    s.audit_now()
    a = s.audits()[-1]
    assert np.allclose(a["mom_I"][:d], o.momentum_I(), rtol=0, atol=1e-12 * mass0), (a["mom_I"], o.momentum_I())
    mg, mo = s.moments(), o.moments()
    assert float(np.max(np.abs(mg["rho"].cpu().numpy() - mo["rho"].ravel()))) <= 1e-12
    assert float(np.max(np.abs(mg["u"].cpu().numpy() - mo["u"].reshape(d, -1)))) <= 1e-12
    f, geo = m.fields(), o._static_geo()
    A_o = geo.A.reshape(Q, d, -1)
    assert float(np.max(np.abs(f["A"].cpu().numpy() - A_o))) <= 1e-12
    assert float(np.max(np.abs(f["g"].cpu().numpy() - geo.g.reshape(d, d, -1)))) <= 1e-12
    assert float(np.max(np.abs(f["J"].cpu().numpy() - geo.J.ravel()))) <= 1e-12
    s.step(3)
    s.audit_now()
    s.sync()
    assert abs(s.audits()[-1]["mass"] / mass0 - 1) <= 1e-13
    s.close()
    m.close()
    # a mesh outliving the simulation that moved it keeps the coefficients of
    # its final positions
    w, o, s, m = _setup(name, n, amp, None, MOTION, audit_every=0)
    for t in range(3):
        X, wr = W.moving_coords(w, t + 1, **MOTION)
        s.step_moving(X, wr)
        o.step(X, wr)
    s.close()
    A = m.fields()["A"].cpu().numpy()
    assert float(np.max(np.abs(A - o._static_geo().A.reshape(Q, d, -1)))) <= 1e-12
    m.close()


def test_kernel_timing_of_moving_steps():
    """vlbm_kernel_timing records one fused step and one geometry launch per
    moving step, with positive durations, and nothing once it is off."""
    v = _vlbm()
    announce("moving mesh kernel timing")
    w = W.wavy_periodic("D3Q19", (7, 6, 5), 0.1)
    w["tau"] = 0.7
    m = v.Mesh.from_workload(w)
    s = v.Sim(m, v.make_params(0.7, precision="fp64"))
    s.kernel_timing(True)
    for t in range(5):
        s.step_moving(*W.moving_coords(w, t + 1, **MOTION))
    kt = s.kernel_timing(False)
    assert kt["step_launches"] == 5 and kt["basis_launches"] == 5 and kt["rebase_launches"] == 0
    assert kt["step_ms"] > 0 and kt["basis_ms"] > 0
    s.step_moving(*W.moving_coords(w, 6, **MOTION))
    kt = s.kernel_timing(False)
    assert kt["step_launches"] == 0 and kt["basis_launches"] == 0
    s.close()
    m.close()


def test_mesh_at_rest_equals_the_static_step():
    """Moving steps to unchanged positions are the static step (the incoming
    coefficients are computed from the two time levels instead of taken from
    the opposite direction: equal up to rounding)."""
    v = _vlbm()
    announce("moving steps on a mesh at rest vs static steps")
    w = W.wavy_periodic("D3Q19", (7, 6, 5), 0.1)
    w["tau"] = 0.7
    rng = np.random.default_rng(5)
    u = 0.02 * rng.standard_normal((3, 5 * 6 * 7))
    m1 = v.Mesh.from_workload(w)
    m2 = v.Mesh.from_workload(w)
    p = v.make_params(w["tau"], precision="fp64")
    s1 = v.Sim(m1, p, u=u)
    s2 = v.Sim(m2, p, u=u)
    for _ in range(8):
        s1.step_moving(w["coords"], w["wrap"])
    s2.step(8)
    a, b = s1.populations(), s2.populations()
    assert float((a - b).abs().max()) <= 1e-13


def test_moving_step_rejections_and_static_continuation():
    v = _vlbm()
    announce("moving-mesh rejections")
    w = W.wavy_periodic("D2Q9", (12, 10), 0.2)
    w["tau"] = 0.7
    X1, wr1 = W.moving_coords(w, 1, **MOTION)
    m = v.Mesh.from_workload(w)
    s32 = v.Sim(m, v.make_params(0.7, precision="fp32"))
    with pytest.raises(v.VlbmError) as e:
        s32.step_moving(X1, wr1)
    assert e.value.code == v.ERR_UNSUPPORTED
    s64 = v.Sim(m, v.make_params(0.7, precision="fp64"))
    with pytest.raises(v.VlbmError) as e:   # two simulations share the mesh
        s64.step_moving(X1, wr1)
    assert e.value.code == v.ERR_STATE
    s32.close()
    wc = W.tanh_channel_2d(12, 10)
    mc = v.Mesh.from_workload(wc)
    sc = v.Sim(mc, v.make_params(0.8, precision="fp64"))
    with pytest.raises(v.VlbmError) as e:   # walls
        sc.step_moving(wc["coords"], None)
    assert e.value.code == v.ERR_UNSUPPORTED
    # a mesh folded onto itself is reported at the next sync
    folded = np.array(w["coords"])
    folded[..., 0] *= -1.0
    s64.step_moving(folded, None)
    with pytest.raises(v.VlbmError) as e:
        s64.sync()
    assert e.value.code == v.ERR_MESH
    # static steps continue on a moved mesh (re-packed geometry), conserving mass
    m2 = v.Mesh.from_workload(w)
    s = v.Sim(m2, v.make_params(0.7, precision="fp64", audit_every=1))
    for t in range(4):
        s.step_moving(*W.moving_coords(w, t + 1, **MOTION))
    s.step(4)
    s.sync()
    aud = s.audits()
    assert abs(aud[-1]["mass"] / aud[0]["mass"] - 1) <= 1e-13
    assert aud[-1]["nonfinite"] == 0


def test_benchmarked_moving_configuration_properties():
    """The benchmarked moving configuration at its full size (D3Q19 256x128x128,
    waviness 2 cells, displacements breathing by 30 % over 40 steps), where
    the oracle is too slow to run: three moving steps conserve the mass to
    1e-13 and balance the mid-link momentum to 1e-12 of the mass every step;
    and on the same mesh held at rest, moving steps (coefficients computed in
    the step, banded block order) equal static steps (packed coefficients)
    within 1e-13 in every cell."""
    v = _vlbm()
    announce("moving mesh D3Q19 256x128x128: balances and rest")
    w = W.wavy_periodic("D3Q19", (256, 128, 128), 2.0)
    motion = dict(breathe=0.3, period=40)
    rng = np.random.default_rng(7)
    nc = 256 * 128 * 128
    rho = 1.0 + 0.01 * rng.standard_normal(nc)
    u = 0.01 * rng.standard_normal((3, nc))
    X0, wr0 = W.moving_coords(w, 0, **motion)
    m = v.Mesh("D3Q19", w["n"], X0, w["faces"], wr0, w["dx"])
    s = v.Sim(m, v.make_params(w["tau"], precision="fp64", audit_every=1), rho=rho, u=u)
    s.audit_now()
    for t in range(3):
        s.step_moving(*W.moving_coords(w, t + 1, **motion))
    s.sync()
    aud = s.audits()
    mass0 = aud[0]["mass"]
    for k in range(1, len(aud)):
        assert abs(aud[k]["mass"] / mass0 - 1) <= 1e-13, (k, aud[k]["mass"], mass0)
        bal = aud[k]["mom_I"] - aud[k - 1]["mom_I"] - aud[k - 1]["force_impulse"]
        assert np.max(np.abs(bal)) <= 1e-12 * mass0, (k, bal)
        assert aud[k]["nonfinite"] == 0
    s.close()
    m.close()
    m1 = v.Mesh("D3Q19", w["n"], X0, w["faces"], wr0, w["dx"])
    m2 = v.Mesh("D3Q19", w["n"], X0, w["faces"], wr0, w["dx"])
    p = v.make_params(w["tau"], precision="fp64")
    s1 = v.Sim(m1, p, rho=rho, u=u)
    s2 = v.Sim(m2, p, rho=rho, u=u)
    for _ in range(3):
        s1.step_moving(X0, wr0)
    s2.step(3)
    err = float((s1.populations() - s2.populations()).abs().max())
    print("moving at rest vs static, 256x128x128:", err)
    assert err <= 1e-13
    for o in (s1, s2, m1, m2):
        o.close()
