"""Sixth-order isotropic lattices (D2Q21, D3Q39: eq. (iso) in full, T0 = 2/3,
links up to three cells long, on periodic boxes and on channels whose walls
reflect the long links) on the GPU versus the FP64 oracle: geometry,
streaming, initial state, steps, audits."""
import numpy as np
import pytest

from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import mesh_of, sim_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vlbm():
    from paper_2401_17183_amd import vlbm
    return vlbm


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


def cpu(t):
    return t.detach().cpu().numpy()


def gpu_sim(w, precision="fp64", rho=None, u=None, mesh=None, **kw):
    v = _vlbm()
    mesh = mesh or v.Mesh.from_workload(w)
    p = v.make_params(w["tau"], body_force=w.get("body_force", (0, 0, 0)), precision=precision, **kw)
    return v.Sim(mesh, p, rho=rho, u=u), mesh


# ragged sizes, several periods of the longest link on every axis; the
# channels have walls (multi-cell bounce-back) on their second axis
MESHES = [W.wavy_periodic("D2Q21", (22, 17), 0.12), W.wavy_periodic("D3Q39", (9, 7, 6), 0.08),
          W.tanh_channel_2d(12, 14, strength=0.3, lattice="D2Q21", dx_ratio=1.0),
          W.tanh_channel_3d(7, 9, 5, strength=0.3, tau=0.8, lattice="D3Q39", dx_ratio=1.0)]
IDS = [w["lattice"] + (" channel" if "channel" in w["name"] else " wavy") for w in MESHES]


def seeded_flow(o, seed=11, amp=0.02):
    rng = np.random.default_rng(seed)
    shape = o.mesh.shape
    d = o.mesh.d
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = amp * rng.standard_normal((d,) + shape)
    return rho, u


@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_geometry_parity(w):
    """J, g^{ij} and A (up to three-cell links, periodic wrap) equal the oracle's."""
    announce(f"geometry {w['name']}")
    from oracle import geometry
    m = _vlbm().Mesh.from_workload(w)
    f = m.fields()
    og = geometry.Geometry(mesh_of(w))
    flat = lambda a: a.reshape(a.shape[:2] + (-1,))
    assert np.allclose(cpu(f["J"]), og.J.ravel(), rtol=1e-14, atol=0)
    assert np.allclose(cpu(f["gup"]), flat(og.gup), rtol=1e-13, atol=1e-14)
    assert np.max(np.abs(cpu(f["A"]) - flat(og.A))) <= 1e-13 * max(np.abs(og.A).max(), 1.0)
    rep = og.report()
    assert abs(m.report["min_rest_feq_over_w"] - rep["min_rest_feq_over_w"]) <= 1e-12 * max(1, abs(rep["min_rest_feq_over_w"]))


@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_stream_only_is_bit_exact(w):
    """Advection alone is the oracle's permutation bit for bit; after n_1 steps
    along a periodic box the state returns only for the axis-aligned links, so
    several steps exercise every wrap."""
    announce(f"stream-only {w['name']}")
    o = sim_of(w, stream_only=True)
    rng = np.random.default_rng(3)
    N0 = rng.random((o.lat.Q,) + o.mesh.shape)
    o.set_state(N0)
    s, _ = gpu_sim(w, stream_only=True)
    s.set_populations(N0.reshape(o.lat.Q, -1))
    assert np.array_equal(cpu(s.populations()), o.N.reshape(o.lat.Q, -1))
    s.step(7)
    o.step(7)
    assert np.array_equal(cpu(s.populations()), o.N.reshape(o.lat.Q, -1))


@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_initial_state_parity(w):
    announce(f"init {w['name']}")
    o = sim_of(w)
    rho, u = seeded_flow(o)
    o.init(rho, u)
    d = o.mesh.d
    s, _ = gpu_sim(w, rho=rho.ravel(), u=u.reshape(d, -1))
    J = o.geom.J.ravel()
    err = np.max(np.abs(cpu(s.populations()) / J - o.N.reshape(o.lat.Q, -1) / J))
    assert err < 1e-13, err


@pytest.mark.parametrize("tau_g", [None, 1.0])
@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_fp64_step_parity(w, tau_g):
    """FP64: max |f_gpu - f_oracle| <= 1e-12 after 100 steps (BGK and the general
    collision matrix)."""
    announce(f"fp64 step {w['name']} tau_g={tau_g} x100")
    o = sim_of(w, tau_g=tau_g)
    rho, u = seeded_flow(o)
    o.init(rho, u)
    d = o.mesh.d
    s, _ = gpu_sim(w, rho=rho.ravel(), u=u.reshape(d, -1), tau_g=tau_g)
    s.step(100)
    o.step(100)
    J = o.geom.J.ravel()
    err = np.max(np.abs(cpu(s.populations()) / J - o.N.reshape(o.lat.Q, -1) / J))
    print("fp64 max |f_gpu - f_oracle|", err)
    assert err <= 1e-12, err
    assert np.allclose(cpu(s.moments()["u"]), o.moments()["u"].reshape(d, -1), rtol=0, atol=1e-11)


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-5), ("fp32c", 1e-3)])
@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_reduced_precision_velocity(w, precision, bound):
    """FP32 storage: velocity relative L2 error after 100 steps within the
    bars of the D3Q19 path (FP64 arithmetic 1e-5; FP32 arithmetic takes the
    1e-3 bar of the modes computed in FP32)."""
    announce(f"{precision} {w['name']} x100")
    o = sim_of(w)
    rho, u = seeded_flow(o)
    o.init(rho, u)
    d = o.mesh.d
    s, _ = gpu_sim(w, precision=precision, rho=rho.ravel(), u=u.reshape(d, -1))
    s.step(100)
    o.step(100)
    ug = cpu(s.moments()["u"])
    uo = o.moments()["u"].reshape(d, -1)
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    print(precision, "velocity rel L2", rel)
    assert rel <= bound, rel


@pytest.mark.parametrize("w", MESHES, ids=IDS)
def test_audits_balance(w):
    """Mass is conserved to roundoff and the mid-link momentum obeys
    I(t+1) = I(t) + G * mass + W(t) every step, W the wall impulse of the
    bounced links (multi-cell bounce-back included); the audits equal the
    oracle's."""
    announce(f"audits {w['name']}")
    o = sim_of(w)
    rho, u = seeded_flow(o)
    o.init(rho, u)
    d = o.mesh.d
    s, _ = gpu_sim(w, rho=rho.ravel(), u=u.reshape(d, -1), audit_every=1)
    s.audit_now()
    s.step(4)
    aud = s.audits()
    assert len(aud) == 5
    prev = None
    for k, a in enumerate(aud):
        if k > 0:
            o.step()
        oa = o.audit()
        scale = oa["mass"]
        assert abs(a["mass"] - oa["mass"]) <= 1e-13 * scale
        assert np.allclose(a["mom_I"][:d], oa["mom_I"], rtol=0, atol=1e-12 * scale)
        assert np.allclose(a["wall_impulse"][:d], oa["wall_impulse"], rtol=0, atol=1e-12 * scale)
        if prev is not None:
            bal = a["mom_I"] - prev["mom_I"] - prev["force_impulse"] - a["wall_impulse"]
            assert np.max(np.abs(bal)) <= 1e-12 * scale, bal
        assert a["nonfinite"] == 0 and a["unconverged"] == 0
        prev = a


def test_sixteen_bit_storage_and_batches_are_rejected():
    v = _vlbm()
    w = MESHES[1]
    m = v.Mesh.from_workload(w)
    announce("D3Q39 rejections")
    with pytest.raises(v.VlbmError) as e:
        v.Sim(m, v.make_params(0.8, precision="fp16s"))
    assert e.value.code == v.ERR_UNSUPPORTED
    with pytest.raises(v.VlbmError) as e:
        v.Batch([m], [v.make_params(0.8, precision="fp32")])
    assert e.value.code == v.ERR_UNSUPPORTED
