"""What the learned warm start gains over the method alone (GPU).

Small bump channels (64 x 32): steady states from the batched solver train the
BF16-MFMA surrogate; held-out meshes are then solved to r <= 1e-6 from rest
(cold) and from the surrogate's prediction (warm).  The solver finishes every
solve, so both must reach the same steady state; the warm start must need fewer
steps (median over the held-out meshes)."""
import numpy as np
import pytest

from paper_2401_17183_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.mark.timeout(900)
def test_warm_start_needs_fewer_steps_than_cold_start():
    from paper_2401_17183_amd import surrogate as S
    from paper_2401_17183_amd import vlbm
    ntr, nte = 160, 8
    ws = W.surrogate_meshes(ntr + nte, seed=7, n1=64, n2=32)
    wtr, wte = ws[:ntr], ws[ntr:]
    announce(f"steady states of {ntr} training meshes 64x32")
    b, _ = S.make_batch(wtr)
    steps, total, wall = S.solve_steady(b, tol=1e-6)
    assert (steps > 0).all()
    F = S.fields(b, wtr)
    b.close()
    norm = S.Normaliser.fit(F, ws[0]["u_bulk"])
    X = torch.tensor(np.stack([S.features(w) for w in wtr])).cuda()
    T = torch.tensor(norm.encode(F)).cuda()
    announce("training 250 epochs")
    net = vlbm.Surrogate(32, 64, 16, S.he_init(2401))
    hist = S.train(net, X, T, epochs=250, batch=16, lr=1e-3)
    assert hist[-1][0] < 0.02 * hist[0][0], hist[::25]
    announce(f"cold solves of {nte} held-out meshes")
    bc, _ = S.make_batch(wte)
    cold, _, _ = S.solve_steady(bc, tol=1e-6)
    Fc = S.fields(bc, wte)
    bc.close()
    announce(f"warm solves of {nte} held-out meshes")
    bw, mw = S.make_batch(wte)
    P = S.predict(net, norm, torch.tensor(np.stack([S.features(w) for w in wte])).cuda())
    S.warm_start(bw, P, mw)
    warm, _, _ = S.solve_steady(bw, tol=1e-6)
    Fw = S.fields(bw, wte)
    bw.close()
    net.close()
    err = [np.linalg.norm(P[k, ..., :2] - Fc[k, ..., :2]) / np.linalg.norm(Fc[k, ..., :2]) for k in range(nte)]
    agree = [np.linalg.norm(Fw[k, ..., :2] - Fc[k, ..., :2]) / np.linalg.norm(Fc[k, ..., :2]) for k in range(nte)]
    print("cold steps", cold.tolist(), "warm steps", warm.tolist())
    print("surrogate velocity error", np.round(err, 4).tolist(), "warm vs cold final", np.max(agree))
    assert (cold > 0).all() and (warm > 0).all()
    assert np.median(warm) < np.median(cold)
    assert np.max(agree) <= 1e-2
