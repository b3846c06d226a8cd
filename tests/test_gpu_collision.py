"""General collision matrix (eq. (collide) with eq. (matrix)) on the GPU versus
the FP64 oracle: M = -I/tau_g + (1/tau_g - 1/tau) H, tau_g = 1 the regularised
collision.  Same bars as the BGK path."""
import numpy as np
import pytest

from paper_2401_17183_amd import workloads as W
from tests.oracle_helpers import sim_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vlbm():
    from paper_2401_17183_amd import vlbm
    return vlbm


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


def cpu(t):
    return t.detach().cpu().numpy()


def gpu_sim(w, tau_g, mesh=None, precision="fp64", rho=None, u=None, **kw):
    v = _vlbm()
    mesh = mesh or v.Mesh.from_workload(w)
    p = v.make_params(w["tau"], body_force=w.get("body_force", (0, 0, 0)), rho_inf=w.get("rho_inf", 1.0),
                      u_inf=w.get("u_inf", (0, 0, 0)), precision=precision, tau_g=tau_g, **kw)
    return v.Sim(mesh, p, rho=rho, u=u), mesh


def start_fields(w):
    rho, u = w.get("rho"), w.get("u")
    if w["lattice"] == "D2Q9" and "half_height" in w:
        rho, u = W.poiseuille_fields(w)
    return rho, u


@pytest.mark.parametrize("tau_g", [1.0, 1.4])
@pytest.mark.parametrize("w,steps", [(W.tanh_channel_2d(64, 32), 100), (W.wavy_channel_3d(16, 12, 8), 100),
                                     (W.ogrid_3d(8, 96, 4, rmax=1.5, dx_factor=1.3), 50)],
                         ids=lambda x: str(x) if isinstance(x, int) else x["name"])
def test_general_collision_fp64_parity(w, steps, tau_g):
    """FP64: max |f_gpu - f_oracle| <= 1e-12 after `steps` steps (f = N/J)."""
    announce(f"general collision fp64 {w['name']} tau_g={tau_g} x{steps}")
    o = sim_of(w, tau_g=tau_g)
    rho, u = start_fields(w)
    o.init(rho, u)
    d = o.mesh.d
    s, _ = gpu_sim(w, tau_g, rho=None if rho is None else rho.ravel(), u=None if u is None else u.reshape(d, -1))
    s.step(steps)
    o.step(steps)
    J = o.geom.J.ravel()
    err = np.max(np.abs(cpu(s.populations()) / J - o.N.reshape(o.lat.Q, -1) / J))
    print("fp64 general max |f_gpu - f_oracle|", err)
    assert err <= 1e-12, err
    mo, om = s.moments(), o.moments()
    assert np.allclose(cpu(mo["u"]), om["u"].reshape(d, -1), rtol=0, atol=1e-11)
    # the general matrix changes the result: not the BGK run
    b = sim_of(w)
    b.init(rho, u)
    b.step(steps)
    assert np.max(np.abs(b.N - o.N)) > 1e-9


@pytest.mark.parametrize("precision,bound", [("fp32", 1e-5), ("fp32c", 1e-3), ("fp16s", 1e-3)])
def test_general_collision_reduced_precision(precision, bound):
    """Velocity relative L2 vs the FP64 oracle after 200 steps on the stretched
    channel, tau_g = 1: the bars of the BGK path (FP32 storage with FP64
    arithmetic 1e-5; the modes computed in FP32, FP32C and FP16S, take the
    1e-3 bar of FP32 arithmetic)."""
    w = W.tanh_channel_3d(32, 24, 16, strength=1.5, tau=0.6, G=1e-5)
    announce(f"general collision {precision} tanh(1.5) channel 32x24x16 x200")
    o = sim_of(w, tau_g=1.0)
    o.init(w["rho"], w["u"])
    s, _ = gpu_sim(w, 1.0, precision=precision, rho=w["rho"].ravel(), u=w["u"].reshape(3, -1))
    s.step(200)
    o.step(200)
    u_g = cpu(s.moments()["u"])
    u_o = o.moments()["u"].reshape(3, -1)
    rel = np.linalg.norm(u_g - u_o) / np.linalg.norm(u_o)
    print(precision, "general collision velocity rel L2", rel)
    assert rel <= bound, rel


def test_general_collision_audits_balance():
    """Mass is exact and I(t+1) = I(t) + G*mass + W(t) with the general matrix
    (it conserves mass and momentum, eqs. (conserv), (omcons)); the audits
    equal the oracle's."""
    w = W.wavy_channel_3d(10, 8, 6)
    announce("general collision audits wavy channel")
    o = sim_of(w, tau_g=1.0)
    o.init(w["rho"], w["u"])
    s, _ = gpu_sim(w, 1.0, rho=w["rho"].ravel(), u=w["u"].reshape(3, -1), audit_every=1)
    s.audit_now()
    s.step(4)
    aud = s.audits()
    prev = None
    for k, a in enumerate(aud):
        if k > 0:
            o.step()
        oa = o.audit()
        assert abs(a["mass"] - oa["mass"]) <= 1e-13 * oa["mass"]
        assert np.allclose(a["mom_I"][:3], oa["mom_I"], rtol=0, atol=1e-12 * oa["mass"])
        if prev is not None:
            bal = a["mom_I"] - prev["mom_I"] - prev["force_impulse"] - a["wall_impulse"]
            assert np.max(np.abs(bal)) <= 1e-12 * a["mass"], bal
            assert abs(a["mass"] / prev["mass"] - 1) <= 1e-14
        assert a["nonfinite"] == 0 and a["unconverged"] == 0
        prev = a


def test_batch_with_mixed_collisions():
    """A batch whose members mix BGK and general matrices: general members equal
    their solo runs bit for bit, BGK members (stepped by the general kernel with
    tau_g = tau) equal theirs to FP64 roundoff, and all match the oracle."""
    v = _vlbm()
    ws = [W.bump_channel_2d(37, 13, 0.2, 2.0, 0.7), W.bump_channel_2d(20, 9, 0.0, 1.0, 0.95),
          W.bump_channel_2d(45, 30, 0.1, 1.5, 0.8)]
    tgs = [1.0, None, 0.6]
    announce("batch mixed collisions fp64 x60")
    meshes = [v.Mesh.from_workload(w) for w in ws]
    ps = [v.make_params(w["tau"], body_force=w["body_force"], precision="fp64", tau_g=t) for w, t in zip(ws, tgs)]
    b = v.Batch(meshes, ps)
    solo = [v.Sim(m, p) for m, p in zip(meshes, ps)]
    b.step(60)
    for s in solo:
        s.step(60)
    b.sync()
    for k, (m, s, w, t) in enumerate(zip(b.members, solo, ws, tgs)):
        x, y = m.populations().cpu(), s.populations().cpu()
        if t is not None:
            assert torch.equal(x, y), (k, float((x - y).abs().max()))
        else:
            assert float((x - y).abs().max()) <= 1e-13, k
        o = sim_of(w, tau_g=t)
        o.init(None, None)
        o.step(60)
        err = np.max(np.abs(x.numpy() - o.N.reshape(o.N.shape[0], -1)))
        assert err <= 1e-12, (k, err)
    b.close()


def test_tau_g_is_validated():
    v = _vlbm()
    w = W.wavy_periodic("D2Q9", (12, 10), 0.1)
    m = v.Mesh.from_workload(w)
    announce("tau_g validation")
    for bad in (0.5, 0.3, -1.0, float("nan"), float("inf")):
        with pytest.raises(v.VlbmError) as e:
            v.Sim(m, v.make_params(0.8, tau_g=bad))
        assert e.value.code == v.ERR_ARG
    # tau_g = tau is BGK exactly (the BGK kernel runs)
    a = v.Sim(m, v.make_params(0.8))
    c = v.Sim(m, v.make_params(0.8, tau_g=0.8))
    a.step(20)
    c.step(20)
    assert torch.equal(a.populations(), c.populations())
