"""Batched stepping of many uneven meshes (one persistent launch per step).

A batch member must evolve exactly as the same mesh stepped on its own: the
batch kernel runs the same per-cell update, so populations agree bit for bit
in every launch mode (persistent + graph, persistent, eager, eager + graph)
and launch shape.  Members are also checked against the FP64 oracle."""
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


# ragged sizes (none a multiple of 64), differing tau, bump and stretch
SMALL_BATCH = [W.bump_channel_2d(37, 13, 0.2, 2.0, 0.7), W.bump_channel_2d(20, 9, 0.0, 1.0, 0.95),
               W.bump_channel_2d(64, 16, 0.25, 2.5, 0.6), W.bump_channel_2d(45, 30, 0.1, 1.5, 0.8),
               W.bump_channel_2d(33, 17, 0.3, 3.0, 0.55)]


def _params(v, w, precision):
    return v.make_params(w["tau"], body_force=w["body_force"], precision=precision)


def _batch(ws, precision):
    v = _vlbm()
    meshes = [v.Mesh.from_workload(w) for w in ws]
    return v.Batch(meshes, [_params(v, w, precision) for w in ws]), meshes


def _solo(ws, meshes, precision):
    v = _vlbm()
    return [v.Sim(m, _params(v, w, precision)) for w, m in zip(ws, meshes)]


def _pops(sims):
    return [s.populations().cpu() for s in sims]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32c"])
@pytest.mark.parametrize("mode", ["BATCH_PERSISTENT_GRAPH", "BATCH_PERSISTENT", "BATCH_EAGER", "BATCH_EAGER_GRAPH"])
def test_batch_equals_solo_runs(precision, mode):
    """70 steps = two captured 32-step graphs + an eager remainder; then 3 more
    single steps (odd start parity)."""
    v = _vlbm()
    announce(f"batch vs solo {precision} {mode}")
    b, meshes = _batch(SMALL_BATCH, precision)
    solo = _solo(SMALL_BATCH, meshes, precision)
    b.set_mode(getattr(v, mode))
    b.step(70)
    for s in solo:
        s.step(70)
    b.sync()
    for k, (x, y) in enumerate(zip(_pops(b.members), _pops(solo))):
        assert torch.equal(x, y), (k, float((x - y).abs().max()))
    for _ in range(3):
        b.step(1)
    b.step(33)
    for s in solo:
        s.step(36)
    b.sync()
    for k, (x, y) in enumerate(zip(_pops(b.members), _pops(solo))):
        assert torch.equal(x, y), (k, float((x - y).abs().max()))
    assert all(m.t == 106 for m in b.members)
    b.close()


@pytest.mark.parametrize("block,grid_per_cu", [(64, 1), (128, 8), (256, 0)])
def test_launch_shape_does_not_change_results(block, grid_per_cu):
    v = _vlbm()
    announce(f"batch launch shape block={block} grid_per_cu={grid_per_cu}")
    b, meshes = _batch(SMALL_BATCH, "fp32")
    solo = _solo(SMALL_BATCH, meshes, "fp32")
    b.config(block, grid_per_cu)
    assert b.info()["block"] == block and b.info()["grid_per_cu"] == grid_per_cu
    b.set_mode(v.BATCH_PERSISTENT_GRAPH)
    b.step(40)
    for s in solo:
        s.step(40)
    b.sync()
    for x, y in zip(_pops(b.members), _pops(solo)):
        assert torch.equal(x, y)
    b.close()


def test_autotune_keeps_state_and_caches(tmp_path):
    announce("batch autotune")
    b, meshes = _batch(SMALL_BATCH, "fp32c")
    b.step(5)
    before = _pops(b.members)
    cache = tmp_path / "tune.txt"
    block, gpc = b.autotune(trial_steps=4, cache_path=str(cache))
    assert block in (64, 128, 256) and gpc in (0, 1, 2, 4, 8)
    assert b.info()["block"] == block and b.info()["grid_per_cu"] == gpc
    after = _pops(b.members)
    for x, y in zip(before, after):
        assert torch.equal(x, y)
    assert all(m.t == 5 for m in b.members)
    text = cache.read_text()
    assert f"block={block} grid_per_cu={gpc}" in text
    # a second batch of the same shape takes the cached choice
    b2, _ = _batch(SMALL_BATCH, "fp32c")
    assert b2.autotune(trial_steps=4, cache_path=str(cache)) == (block, gpc)
    assert cache.read_text() == text
    b.close()
    b2.close()


def test_batch_members_match_oracle_fp64():
    announce("batch members vs oracle fp64, 100 steps")
    b, _ = _batch(SMALL_BATCH, "fp64")
    b.step(100)
    b.sync()
    for w, m in zip(SMALL_BATCH, b.members):
        o = sim_of(w)
        o.init(None, None)
        o.step(100)
        got = m.populations().cpu().numpy()
        err = np.max(np.abs(got - o.N.reshape(o.N.shape[0], -1)))
        assert err <= 1e-12, (w["name"], err)
    b.close()


def test_batch_rejects_mixed_or_unsupported():
    v = _vlbm()
    announce("batch argument errors")
    w2 = SMALL_BATCH[0]
    w3 = W.wavy_channel_3d(6, 5, 4)
    m2, m3 = v.Mesh.from_workload(w2), v.Mesh.from_workload(w3)
    with pytest.raises(v.VlbmError) as e:
        v.Batch([m2, m3], [_params(v, w2, "fp32"), _params(v, w3, "fp32")])
    assert e.value.code == v.ERR_ARG
    with pytest.raises(v.VlbmError) as e:
        v.Batch([m2, m2], [_params(v, w2, "fp32"), _params(v, w2, "fp64")])
    assert e.value.code == v.ERR_ARG
    with pytest.raises(v.VlbmError) as e:
        v.Batch([m2], [_params(v, w2, "fp16s")])
    assert e.value.code == v.ERR_UNSUPPORTED
    b, _ = _batch(SMALL_BATCH[:2], "fp32")
    with pytest.raises(v.VlbmError):
        b.set_mode(7)
    with pytest.raises(v.VlbmError):
        b.config(96, 2)
    with pytest.raises(v.VlbmError):
        b.step(-1)
    b.close()


def test_reinit_matches_fresh_init():
    v = _vlbm()
    announce("reinit")
    w = SMALL_BATCH[3]
    m = v.Mesh.from_workload(w)
    s = v.Sim(m, _params(v, w, "fp64"))
    fresh = s.populations().cpu()
    s.step(25)
    s.reinit()
    assert s.t == 0
    assert torch.equal(s.populations().cpu(), fresh)
    rng = np.random.default_rng(7)
    rho = 1.0 + 0.01 * rng.standard_normal(m.ncells)
    u = 0.01 * rng.standard_normal((2, m.ncells))
    s.reinit(rho=rho, u=u)
    s2 = v.Sim(m, _params(v, w, "fp64"), rho=rho, u=u)
    assert torch.equal(s.populations().cpu(), s2.populations().cpu())
    s.close()
    s2.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("start", ["rest", "vortex"])
def test_full_batch_sampled_parity_fp32(start):
    """The 256-mesh uneven batch (2.87 M cells) in FP32 storage, one persistent
    launch per step (graph-replayed, references re-based every 10 steps), 100
    steps from rest (the batch workload's own start) and from a smooth
    0.02-amplitude vortex state; 8 seeded members against the FP64 oracle:
    velocity relative L2 <= 1e-5."""
    v = _vlbm()
    ws = W.batch_meshes(256)
    announce(f"full batch ({start} start): meshes")
    b, _ = _batch(ws, "fp32")
    assert b.info()["count"] == 256
    assert b.info()["cells"] == sum(int(np.prod(w["n"])) for w in ws)
    if start == "vortex":
        announce("full batch: initial fields")
        for w, m in zip(ws, b.members):
            rho, u = W.channel_vortex_fields(w)
            m.reinit(rho=rho.ravel(), u=u.reshape(2, -1))
    announce("full batch: 100 steps")
    b.step(100)
    b.sync()
    rng = np.random.default_rng(2401)
    for k in rng.choice(len(ws), size=8, replace=False):
        w = ws[k]
        announce(f"full batch: oracle member {k} {w['n']}")
        o = sim_of(w)
        if start == "vortex":
            o.init(*W.channel_vortex_fields(w))
        else:
            o.init()
        o.step(100)
        uo = o.moments()["u"].reshape(2, -1)
        ug = b.members[k].moments()["u"].cpu().numpy()
        rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
        print(f"member {k} {w['n']} velocity rel L2 {rel:.3e} (|u| max {np.abs(uo).max():.2e})")
        assert rel <= 1e-5, (k, w["n"], rel)
    b.close()


@pytest.mark.parametrize("mode", ["BATCH_PERSISTENT_GRAPH", "BATCH_EAGER"])
def test_retired_members_keep_their_state(mode):
    """Members retired with set_active keep their state and step count while
    the others advance; every member still equals its solo run bit for bit.
    Members at different step counts cannot be stepped together; the retired
    ones can, once they share a step count; retiring everything makes step a
    no-op."""
    v = _vlbm()
    announce(f"batch retirement {mode}")
    b, meshes = _batch(SMALL_BATCH, "fp32")
    solo = _solo(SMALL_BATCH, meshes, "fp32")
    b.set_mode(getattr(v, mode))
    b.step(40)
    r0 = b.residuals()
    keep = [True, False, True, False, True]
    b.set_active(keep)
    b.step(70)                       # one 40-step graph and an eager remainder
    r1 = b.residuals()
    for k, s in enumerate(solo):
        s.step(110 if keep[k] else 40)
    b.sync()
    for k, (x, y) in enumerate(zip(_pops(b.members), _pops(solo))):
        assert torch.equal(x, y), (k, float((x - y).abs().max()))
        assert b.members[k].t == (110 if keep[k] else 40)
    # retired members report their last residual
    assert np.array_equal(r1[[1, 3]], r0[[1, 3]], equal_nan=True)
    with pytest.raises(v.VlbmError) as e:
        b.set_active(None)
    assert e.value.code == v.ERR_STATE
    b.set_active([not x for x in keep])   # members 1 and 3 share step 40
    b.step(70)
    for k in (1, 3):
        solo[k].step(70)
    b.sync()
    for k, (x, y) in enumerate(zip(_pops(b.members), _pops(solo))):
        assert torch.equal(x, y), (k, float((x - y).abs().max()))
    b.set_active([False] * 5)
    b.step(10)
    b.sync()
    assert all(m.t == 110 for m in b.members)
    b.close()
