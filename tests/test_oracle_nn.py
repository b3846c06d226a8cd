"""Pins of the FP64 surrogate layers (oracle/nn.py) against definitions the
oracle does not share: a library correlation, shifted inputs, finite
differences, adjointness and Adam's closed-form steps."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn


def _rand(rng, *shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_library_correlation(stride):
    rng = np.random.default_rng(1)
    x = _rand(rng, 2, 7, 9, 3)
    w = _rand(rng, 4, 3, 3, 3)
    b = _rand(rng, 4)
    y = nn.conv3x3(x, w, b, stride)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(x[n, :, :, ci], w[co, :, :, ci], mode="same", boundary="fill")
                              for ci in range(3))
            assert np.allclose(y[n, :, :, co], ref[::stride, ::stride], rtol=1e-13, atol=1e-13)
    assert y.shape == (2, (7 + stride - 1) // stride, (9 + stride - 1) // stride, 4)


@pytest.mark.parametrize("kh,kw", [(0, 0), (1, 1), (2, 0), (0, 2)])
def test_one_hot_kernel_shifts_input(kh, kw):
    rng = np.random.default_rng(2)
    x = _rand(rng, 1, 6, 5, 2)
    w = np.zeros((2, 3, 3, 2))
    w[0, kh, kw, 1] = 1.0
    y = nn.conv3x3(x, w, np.zeros(2))
    xp = np.zeros((1, 8, 7, 2))
    xp[:, 1:7, 1:6] = x
    assert np.array_equal(y[0, :, :, 0], xp[0, kh:kh + 6, kw:kw + 5, 1])
    assert not y[..., 1].any()


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(3)
    x = _rand(rng, 2, 6, 8, 3)
    w = _rand(rng, 5, 3, 3, 3)
    b = _rand(rng, 5)
    gy = _rand(rng, *nn.conv3x3(x, w, b, stride).shape)
    gx, gw, gb = nn.conv3x3_backward(x, w, gy, stride)
    f = lambda x_, w_, b_: float((gy * nn.conv3x3(x_, w_, b_, stride)).sum())
    h = 1e-6
    for arr, grad, which in ((x, gx, 0), (w, gw, 1), (b, gb, 2)):
        v = _rand(rng, *arr.shape)
        args_p = [x, w, b]
        args_m = [x, w, b]
        args_p[which] = arr + h * v
        args_m[which] = arr - h * v
        fd = (f(*args_p) - f(*args_m)) / (2 * h)
        assert abs(fd - float((grad * v).sum())) <= 1e-7 * max(1.0, abs(fd)), which
    # the objective is linear in each argument, so single entries are exact too
    xe = x.copy()
    xe[1, 5, 7, 2] += 1.0
    assert np.isclose(f(xe, w, b) - f(x, w, b), gx[1, 5, 7, 2], rtol=1e-12, atol=1e-12)


def test_upsample_pool_adjoint():
    rng = np.random.default_rng(4)
    x = _rand(rng, 2, 3, 5, 4)
    g = _rand(rng, 2, 6, 10, 4)
    assert np.isclose((nn.upsample2(x) * g).sum(), (x * nn.pool2_sum(g)).sum(), rtol=1e-13)
    assert np.array_equal(nn.upsample2(x)[:, 1::2, ::2], x)


def test_mse_gradient():
    rng = np.random.default_rng(5)
    y = _rand(rng, 2, 4, 4, nn.OUT_CHANNELS)
    t = _rand(rng, 2, 4, 4, nn.TARGET_CHANNELS)
    L, g = nn.mse(y, t)
    assert np.isclose(L, np.mean((y[..., :3] - t) ** 2))
    v = _rand(rng, *y.shape)
    h = 1e-6
    fd = (nn.mse(y + h * v, t)[0] - nn.mse(y - h * v, t)[0]) / (2 * h)
    assert np.isclose(fd, (g * v).sum(), rtol=1e-7)
    assert not g[..., 3:].any()


def test_adam_constant_gradient_steps_are_lr_sign():
    """With bias correction and a constant gradient, m_hat = g and v_hat = g^2 at
    every step, so each step moves lr * g / (|g| + eps) (Kingma and Ba, Alg. 1)."""
    rng = np.random.default_rng(6)
    p = _rand(rng, 50)
    g = _rand(rng, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    p0 = p.copy()
    for t in range(1, 4):
        p, m, v = nn.adam_step(p, g, m, v, t, lr)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15 * t + 1e-12)


def test_layer_table_and_parameter_count():
    t = nn.layer_table()
    assert len(t) == 19
    assert [x[0] for x in t][:2] == ["enc0a", "enc0b"] and t[-1][0] == "head"
    # skip channels join the upsampled tensor at the same resolution
    C = nn.LEVEL_CHANNELS
    for name, ci, cs, up, s, co, r in t:
        if up:
            lvl = int(name[3])
            assert ci == C[lvl + 1] and cs == C[lvl] and s == 1
    n = nn.param_count()
    p = np.arange(n, dtype=np.float64)
    parts = nn.unpack(p)
    assert parts[0][0].shape == (32, 3, 3, 8) and parts[0][1][0] == 32 * 9 * 8
    assert parts[-1][0].shape == (16, 3, 3, 32)


def _init(rng, scale=1.0):
    parts = []
    for _, ci, cs, _, _, co, _ in nn.layer_table():
        fan = 9 * (ci + cs)
        parts.append(scale * rng.standard_normal(co * fan) * np.sqrt(2.0 / fan))
        parts.append(0.1 * rng.standard_normal(co))
    return np.concatenate(parts)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(7)
    params = _init(rng)
    x = _rand(rng, 1, 16, 16, nn.IN_CHANNELS)
    x[..., 3:] = 0.0
    gy = _rand(rng, 1, 16, 16, nn.OUT_CHANNELS)
    net = nn.Surrogate(params)
    y = net.forward(x)
    assert y.shape == (1, 16, 16, nn.OUT_CHANNELS)
    g = net.backward(gy)
    assert g.shape == params.shape
    f = lambda p: float((gy * nn.Surrogate(p).forward(x)).sum())
    h = 1e-6
    v = rng.standard_normal(params.size)
    fd = (f(params + h * v) - f(params - h * v)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ v)
    # single parameters in the first, a skip-fed, and the last layer
    offs = np.cumsum([0] + [co * 9 * (ci + cs) + co for _, ci, cs, _, _, co, _ in nn.layer_table()])
    for layer, j in ((0, 5), (10, 9 * 256 + 3), (18, 100)):
        e = np.zeros_like(params)
        e[offs[layer] + j] = 1.0
        fd = (f(params + h * e) - f(params - h * e)) / (2 * h)
        assert abs(fd - g[offs[layer] + j]) <= 1e-6 * max(1.0, abs(fd)), (layer, fd, g[offs[layer] + j])


def test_round_bf16_matches_library_conversion():
    import torch
    rng = np.random.default_rng(8)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.0e38, -1e-40]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    got = nn.round_bf16(a)
    assert np.array_equal(got, ref)
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6
    assert got[-4] == 1.0 and got[-3] == 1.0 + 2 ** -6


def test_quantized_network_is_the_plain_one_on_representable_values():
    """With q = round_bf16 the network only differs by the rounding of stored
    activations and gradients: on a tiny input the outputs stay within a few
    bfloat16 ulps relative to the FP64 network."""
    rng = np.random.default_rng(9)
    params = _init(rng)
    x = _rand(rng, 1, 16, 16, nn.IN_CHANNELS)
    x[..., 3:] = 0.0
    y = nn.Surrogate(params).forward(x)
    yq = nn.Surrogate(params).forward(x, q=nn.round_bf16)
    rel = np.linalg.norm(yq - y) / np.linalg.norm(y)
    assert 0 < rel < 5e-2
