"""FP64 reference layers of the convolutional steady-state surrogate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The learned warm start is not part of the paper: the paper's method is the
solver that produces the surrogate's training targets and finishes every solve.
The network is a small encoder-decoder written out here from the definitions of
its layers, in float64, with no blocking or fusion:

* conv3x3     -- cross-correlation with a 3x3 kernel, zero padding 1, stride
                 1 or 2, bias; NHWC activations, weights [C_out][3][3][C_in]
* conv3x3_backward -- the adjoint of conv3x3 with respect to its input, its
                 weights and its bias (from the definition, by the chain rule)
* upsample2 / its adjoint pool2_sum -- nearest-neighbour 2x upsampling
* relu, mse, adam_step -- rectifier, mean squared error over the first three
                 output channels, and the Adam update (Kingma and Ba 2015)
* Surrogate   -- 5 levels, channels 32, 64, 128, 256, 256; stride-2 3x3 convs
                 down, nearest 2x upsampling up, skip connections by channel
                 concatenation (upsampled tensor first), two 3x3 convs per level
                 with ReLU, a 3x3 head to 16 channels of which the first three
                 are (u_x, u_y, rho - 1) in normalised units; input 8 channels
                 (x, y, Re features and five zero channels).

Pins (tests/test_oracle_nn.py): conv3x3 against scipy.signal.correlate2d
summed over channels; a one-hot kernel reproduces a shifted input; every
backward against central finite differences of its forward; Adam's first step
against its closed form (-lr * sign(g) for |g| >> eps); the whole network's
gradient against finite differences.
"""
import numpy as np

LEVEL_CHANNELS = (32, 64, 128, 256, 256)
IN_CHANNELS = 8
OUT_CHANNELS = 16
TARGET_CHANNELS = 3


def conv3x3(x, w, b, stride=1):
    """y[n,oh,ow,co] = b[co] + sum_{kh,kw,ci} xp[n, s*oh+kh, s*ow+kw, ci] w[co,kh,kw,ci],
    xp = x zero-padded by one pixel on each side; output size ceil(H/s) x ceil(W/s)."""
    N, H, W, C = x.shape
    Co = w.shape[0]
    assert w.shape == (Co, 3, 3, C)
    OH, OW = (H + stride - 1) // stride, (W + stride - 1) // stride
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.broadcast_to(b.astype(np.float64), (N, OH, OW, Co)).copy()
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, kh:kh + stride * (OH - 1) + 1:stride, kw:kw + stride * (OW - 1) + 1:stride, :]
            y += patch @ w[:, kh, kw, :].T
    return y


def conv3x3_backward(x, w, gy, stride=1):
    """Gradients of sum(gy * conv3x3(x, w, b, stride)) with respect to x, w, b."""
    N, H, W, C = x.shape
    Co = w.shape[0]
    OH, OW = gy.shape[1], gy.shape[2]
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w, dtype=np.float64)
    for kh in range(3):
        for kw in range(3):
            sl = (slice(None), slice(kh, kh + stride * (OH - 1) + 1, stride),
                  slice(kw, kw + stride * (OW - 1) + 1, stride), slice(None))
            patch = xp[sl]
            gw[:, kh, kw, :] = np.einsum("nhwo,nhwc->oc", gy, patch)
            gxp[sl] += gy @ w[:, kh, kw, :]
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[:, 1:H + 1, 1:W + 1], gw, gb


def upsample2(x):
    """Nearest-neighbour 2x upsampling of an NHWC tensor."""
    return x.repeat(2, axis=1).repeat(2, axis=2)


def pool2_sum(g):
    """Adjoint of upsample2: sum over each 2x2 block."""
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(z):
    return np.maximum(z, 0.0)


def round_bf16(a):
    """Round to the nearest bfloat16 value (ties to even), returned as float64:
    round to float32 first, then keep the upper 16 bits of the IEEE single after
    adding half an ulp of the kept part (plus one when the kept part is odd).
    NaN and infinity are not expected here."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def mse(y, t):
    """Mean of (y - t)^2 over the first TARGET_CHANNELS channels of y (t holds
    exactly those); returns the loss and its gradient with respect to y."""
    d = y[..., :TARGET_CHANNELS] - t
    n = d.size
    g = np.zeros_like(y)
    g[..., :TARGET_CHANNELS] = 2.0 * d / n
    return float((d * d).sum() / n), g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (bias-corrected moments); returns p, m, v."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def layer_table():
    """The conv layers in execution order: (name, c_in_primary, c_skip,
    upsample, stride, c_out, relu).  The parameter vector stores, layer after
    layer, the weights [c_out][3][3][c_in_primary + c_skip] and the bias [c_out]."""
    C = LEVEL_CHANNELS
    t = []
    for lvl in range(5):
        cin = IN_CHANNELS if lvl == 0 else C[lvl - 1]
        t.append((f"enc{lvl}a", cin, 0, False, 1 if lvl == 0 else 2, C[lvl], True))
        t.append((f"enc{lvl}b", C[lvl], 0, False, 1, C[lvl], True))
    for lvl in (3, 2, 1, 0):
        t.append((f"dec{lvl}a", C[lvl + 1], C[lvl], True, 1, C[lvl], True))
        t.append((f"dec{lvl}b", C[lvl], 0, False, 1, C[lvl], True))
    t.append(("head", C[0], 0, False, 1, OUT_CHANNELS, False))
    return t


def param_count():
    return sum(co * 9 * (ci + cs) + co for _, ci, cs, _, _, co, _ in layer_table())


def unpack(params):
    """Split the flat parameter vector into per-layer (w, b)."""
    out, o = [], 0
    for _, ci, cs, _, _, co, _ in layer_table():
        nw = co * 9 * (ci + cs)
        out.append((params[o:o + nw].reshape(co, 3, 3, ci + cs), params[o + nw:o + nw + co]))
        o += nw + co
    assert o == params.size
    return out


class Surrogate:
    """The encoder-decoder above, FP64 forward and backward."""

    def __init__(self, params):
        self.params = np.asarray(params, dtype=np.float64)
        self.layers = unpack(self.params)
        self.table = layer_table()

    def forward(self, x, q=None):
        """x: (N, H, W, IN_CHANNELS), H and W divisible by 16.  Returns the
        (N, H, W, OUT_CHANNELS) output and keeps what backward needs.

        q (optional) is applied to every stored activation of the hidden layers
        (not the head output) -- with q = round_bf16 this models a network that
        keeps its activations in bfloat16 between layers."""
        self._q = q if q is not None else (lambda a: a)
        qf = self._q
        acts = {}
        inputs = []
        h = x
        enc = []
        k = 0
        for lvl in range(5):
            for _ in range(2):
                name, ci, cs, up, s, co, r = self.table[k]
                w, b = self.layers[k]
                inputs.append(h)
                z = conv3x3(h, w, b, s)
                h = qf(relu(z) if r else z)
                acts[name] = h
                k += 1
            enc.append(h)
        for lvl in (3, 2, 1, 0):
            name, ci, cs, up, s, co, r = self.table[k]
            w, b = self.layers[k]
            xin = np.concatenate([upsample2(h), enc[lvl]], axis=-1)
            inputs.append(xin)
            h = qf(relu(conv3x3(xin, w, b, s)))
            acts[name] = h
            k += 1
            name, ci, cs, up, s, co, r = self.table[k]
            w, b = self.layers[k]
            inputs.append(h)
            h = qf(relu(conv3x3(h, w, b, s)))
            acts[name] = h
            k += 1
        name, ci, cs, up, s, co, r = self.table[k]
        w, b = self.layers[k]
        inputs.append(h)
        y = conv3x3(h, w, b, s)
        self._inputs, self._acts = inputs, acts
        return y

    def backward(self, gy):
        """Gradient of sum(gy * forward(x)) with respect to the flat parameters
        (same order as the parameter vector).  The q given to forward is also
        applied to the gradient entering each layer (after the ReLU mask)."""
        qf = self._q
        grads = [None] * len(self.table)
        g = qf(gy)
        genc = [None] * 5
        k = len(self.table) - 1
        # head
        _, _, _, _, s, _, _ = self.table[k]
        gx, gw, gb = conv3x3_backward(self._inputs[k], self.layers[k][0], g, s)
        grads[k] = (gw, gb)
        g = gx
        k -= 1
        # decoder levels in reverse execution order: dec0 (nearest the head) first
        for lvl in (0, 1, 2, 3):
            name, ci, cs, up, s, co, r = self.table[k]
            assert name == f"dec{lvl}b"
            g = qf(g * (self._acts[name] > 0))
            gx, gw, gb = conv3x3_backward(self._inputs[k], self.layers[k][0], g, s)
            grads[k] = (gw, gb)
            g = gx
            k -= 1
            name, ci, cs, up, s, co, r = self.table[k]
            assert name == f"dec{lvl}a"
            g = qf(g * (self._acts[name] > 0))
            gx, gw, gb = conv3x3_backward(self._inputs[k], self.layers[k][0], g, s)
            grads[k] = (gw, gb)
            genc[lvl] = gx[..., ci:]
            g = pool2_sum(gx[..., :ci])
            k -= 1
        # g is now the gradient of the deepest encoder output (enc4b)
        for lvl in (4, 3, 2, 1, 0):
            if lvl < 4:
                g = g + genc[lvl]
            for part in ("b", "a"):
                name, ci, cs, up, s, co, r = self.table[k]
                assert name == f"enc{lvl}{part}"
                g = qf(g * (self._acts[name] > 0))
                gx, gw, gb = conv3x3_backward(self._inputs[k], self.layers[k][0], g, s)
                grads[k] = (gw, gb)
                g = gx
                k -= 1
        assert k == -1
        return np.concatenate([np.concatenate([gw.ravel(), gb.ravel()]) for gw, gb in grads])
