"""The geometry precompute that allocates nothing (static device scratch)
against the allocating one, through the C-ABI: the same FP64 geometry bit for
bit and the same report, on two calls in a row (the second on a smaller
mesh), a degenerate mesh in between (its flag must not leak into the next
call), and the size limit."""
import numpy as np
import pytest

from paper_2401_17183_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _vlbm():
    from paper_2401_17183_amd import vlbm
    return vlbm


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


def _pair(w):
    v = _vlbm()
    ref = v.Mesh.from_workload(w)                       # vlbm_geometry_precompute
    got = v.Mesh.from_workload(w, precompute=False)
    got.precompute(noalloc=True)                        # vlbm_geometry_precompute_noalloc
    return ref, got


def _same(ref, got):
    assert ref.report == got.report
    fr, fg = ref.fields(), got.fields()
    for k in ("J", "gup", "A", "g"):
        assert torch.equal(fr[k], fg[k]), k


def test_noalloc_precompute_equals_allocating_one():
    v = _vlbm()
    big = W.wavy_channel_3d(20, 16, 12)
    small = W.tanh_channel_2d(12, 10)
    announce("noalloc geometry: D3Q19 wavy channel 20x16x12")
    ref, got = _pair(big)
    _same(ref, got)
    # the mesh is usable: a simulation on it steps like one on the other
    p = v.make_params(big["tau"], body_force=big["body_force"], precision="fp64")
    s1 = v.Sim(ref, p, rho=big["rho"].ravel(), u=big["u"].reshape(3, -1))
    s2 = v.Sim(got, p, rho=big["rho"].ravel(), u=big["u"].reshape(3, -1))
    s1.step(5)
    s2.step(5)
    assert torch.equal(s1.populations(), s2.populations())
    # a degenerate mesh through the same scratch: rejected, and its flag does
    # not reach the next call
    announce("noalloc geometry: degenerate mesh")
    X = small["coords"].copy()
    X[..., 0] *= -1.0
    bad = v.Mesh(small["lattice"], small["n"], X, small["faces"], small["wrap"], small["dx"], precompute=False)
    with pytest.raises(v.VlbmError) as e:
        bad.precompute(noalloc=True)
    assert e.value.code == v.ERR_MESH
    announce("noalloc geometry: D2Q9 tanh channel 12x10 (second, smaller call)")
    ref2, got2 = _pair(small)
    _same(ref2, got2)
    # and the first mesh again, after the smaller one
    got.precompute(noalloc=True)
    _same(ref, got)


def test_noalloc_precompute_rejects_meshes_beyond_its_scratch():
    v = _vlbm()
    w = W.affine_mesh("D2Q9", (1100, 1000), np.eye(2))
    announce("noalloc geometry: 1100x1000 mesh beyond the scratch")
    m = v.Mesh.from_workload(w, precompute=False)
    with pytest.raises(v.VlbmError) as e:
        m.precompute(noalloc=True)
    assert e.value.code == v.ERR_ARG and "scratch" in str(e.value)
    m.precompute()   # the allocating call takes it
