"""Learned warm start of steady solves (host orchestration; all arithmetic runs
in the HIP library).

1. Steady states: many bump channels advanced together by the batched
   persistent kernel until each member's residual
   r = ||u_n - u_{n-100}||_2 / ||u_n||_2 (checked every 100 steps) is <= tol.
2. Training: the BF16-MFMA encoder-decoder maps (x / L, y / H, (Re - 55) / 45)
   at every cell to (u_x / U_b, u_y / U_b, (rho - 1) / s_rho).
3. Warm start: the prediction becomes the initial state (consistent
   equilibrium, vlbm_reinit) and the method finishes the solve; the cold start
   is rho = 1, u = 0.

The network never replaces the solver: every reported state is the solver's.
"""
import time

import numpy as np

from . import vlbm

NGHOST = 2
LEVEL_CHANNELS = (32, 64, 128, 256, 256)


def layer_shapes():
    """(c_out, c_in + c_skip) of each conv layer in parameter order (encoder
    levels 0..4, decoder levels 3..0, head) -- the layout of include/vlbm.h."""
    C = LEVEL_CHANNELS
    out = []
    for lvl in range(5):
        out.append((C[lvl], 8 if lvl == 0 else C[lvl - 1]))
        out.append((C[lvl], C[lvl]))
    for lvl in (3, 2, 1, 0):
        out.append((C[lvl], C[lvl + 1] + C[lvl]))
        out.append((C[lvl], C[lvl]))
    out.append((16, C[0]))
    return out


def he_init(seed):
    """He-normal weights (fan-in 9 c_in), zero biases; the head starts 10x smaller."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = layer_shapes()
    for k, (co, ci) in enumerate(shapes):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if k == len(shapes) - 1 else 1.0)
        parts.append(rng.standard_normal(co * 9 * ci).astype(np.float32) * np.float32(std))
        parts.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(parts)


def features(w):
    """[n2][n1][3] inputs of one bump channel: cell position (x / L, y / H) and
    the normalised Reynolds number."""
    n1, n2 = w["n"]
    X = w["coords"][NGHOST:NGHOST + n2]
    f = np.empty((n2, n1, 3), dtype=np.float32)
    f[..., 0] = X[..., 0] / w["wrap"][0][0]
    f[..., 1] = X[..., 1] / w["H"]
    f[..., 2] = (w["Re"] - 55.0) / 45.0
    return f


def make_batch(ws, precision="fp32"):
    meshes = [vlbm.Mesh.from_workload(w) for w in ws]
    params = [vlbm.make_params(w["tau"], body_force=w["body_force"], precision=precision) for w in ws]
    return vlbm.Batch(meshes, params), meshes


def solve_steady(batch, tol=1e-6, check_every=100, max_steps=400000, log=None, retire=True):
    """Step the whole batch until every member's residual is <= tol (or
    max_steps).  With retire, a member stops being stepped once it has
    converged, so the launches cover only the members still running (they are
    left retired: a member is stepped again after vlbm_reinit and set_active).
    The members start at one step count.  Returns per-member steps to
    convergence (-1 if not reached), the total steps taken and the wall time (s)."""
    import torch
    n = len(batch.members)
    steps = np.full(n, -1, dtype=np.int64)
    if retire:
        batch.set_active(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.residuals()              # baseline velocity for the first residual
    t = 0
    while t < max_steps:
        batch.step(check_every)
        t += check_every
        r = batch.residuals()
        newly = (steps < 0) & np.isfinite(r) & (r <= tol)
        steps[newly] = t
        if not np.all(np.isfinite(r)):
            raise RuntimeError(f"non-finite residual in members {np.nonzero(~np.isfinite(r))[0][:8]}")
        if log and t % (100 * check_every) == 0:
            log(f"step {t}: {int((steps >= 0).sum())}/{n} converged, max r {np.max(r):.2e}")
        if np.all(steps >= 0):
            break
        if retire and np.any(newly):
            batch.set_active(steps < 0)
    batch.sync()
    return steps, t, time.perf_counter() - t0


def fields(batch, ws):
    """Steady (rho, u) of every member as a [count][n2][n1][3] float32 array
    (u_x, u_y, rho)."""
    out = []
    for w, m in zip(ws, batch.members):
        n1, n2 = w["n"]
        mo = m.moments()
        f = np.empty((n2, n1, 3), dtype=np.float32)
        u = mo["u"].cpu().numpy()
        f[..., 0] = u[0].reshape(n2, n1)
        f[..., 1] = u[1].reshape(n2, n1)
        f[..., 2] = mo["rho"].cpu().numpy().reshape(n2, n1)
        out.append(f)
    return np.stack(out)


class Normaliser:
    """Targets (u_x / U_b, u_y / U_b, (rho - 1) / s_rho), s_rho from training data."""

    def __init__(self, u_bulk, rho_scale):
        self.u_bulk = float(u_bulk)
        self.rho_scale = float(rho_scale)

    @classmethod
    def fit(cls, F, u_bulk):
        return cls(u_bulk, float(np.std(F[..., 2] - 1.0)) or 1.0)

    def encode(self, F):
        T = np.empty_like(F)
        T[..., 0] = F[..., 0] / self.u_bulk
        T[..., 1] = F[..., 1] / self.u_bulk
        T[..., 2] = (F[..., 2] - 1.0) / self.rho_scale
        return T

    def decode(self, T):
        F = np.empty_like(T)
        F[..., 0] = T[..., 0] * self.u_bulk
        F[..., 1] = T[..., 1] * self.u_bulk
        F[..., 2] = 1.0 + T[..., 2] * self.rho_scale
        return F


def train(net, X, T, Xv=None, Tv=None, epochs=60, batch=32, lr=1e-3, lr_min=1e-5, seed=0, log=None):
    """Adam on minibatches (cosine learning-rate decay); returns the per-epoch
    training and validation losses.  X, T: device float32 [N][H][W][3]."""
    import torch
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=X.device)
        tl = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * k / total))
            last = s == steps_per_epoch - 1
            loss = net.train_step(X.index_select(0, idx), T.index_select(0, idx), cur, want_loss=last)
            k += 1
            if last:
                tl = loss
        vl = validate(net, Xv, Tv, batch) if Xv is not None else float("nan")
        hist.append((tl, vl))
        if log:
            log(f"epoch {ep + 1}/{epochs}: train {tl:.3e} val {vl:.3e}")
    return hist


def validate(net, X, T, batch=32):
    import torch
    se, cnt = 0.0, 0
    for s in range(0, X.shape[0], batch):
        y = net.forward(X[s:s + batch])
        d = (y - T[s:s + batch]).double()
        se += float((d * d).sum())
        cnt += d.numel()
    torch.cuda.synchronize()
    return se / cnt


def predict(net, norm, X, batch=32):
    """Decoded (u_x, u_y, rho) predictions [N][H][W][3] as a numpy array."""
    out = []
    for s in range(0, X.shape[0], batch):
        out.append(net.forward(X[s:s + batch]).cpu().numpy())
    return norm.decode(np.concatenate(out))


def warm_start(batch, F, meshes):
    """Initial state of every member from predicted fields F [count][n2][n1][3].
    The density is shifted so that the total volumetric mass sum_q J rho equals
    that of the rest state (sum_q J): mass is conserved by the method, so the
    steady state a solve reaches depends on it."""
    for k, (m, mesh) in enumerate(zip(batch.members, meshes)):
        f = F[k]
        J = mesh.fields()["J"].cpu().numpy()
        rho = f[..., 2].reshape(-1).astype(np.float64)
        rho = rho + (J.sum() - (J * rho).sum()) / J.sum()
        u = np.stack([f[..., 0].reshape(-1), f[..., 1].reshape(-1)]).astype(np.float64)
        m.reinit(rho=rho, u=u)
