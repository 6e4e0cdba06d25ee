"""Pins for the FP64 oracle of the proposal network: scipy's 2-D
correlation, finite differences, closed forms and torch's bfloat16 rounding."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import net as onet


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 2000), rng.uniform(-1e-3, 1e-3, 500),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0]])
    exp = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(onet.bf16(x), exp)
    assert onet.bf16(1.0 + 2 ** -8) == 1.0          # tie to even
    assert onet.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7


def test_conv_is_scipy_correlation_per_channel_pair():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    y = onet.conv3x3(x, w, b)
    for n in range(2):
        for co in range(4):
            exp = b[co] + sum(correlate2d(x[n, :, :, ci], w[:, :, ci, co], mode="same", boundary="fill")
                              for ci in range(3))
            np.testing.assert_allclose(y[n, :, :, co], exp, atol=1e-12)


def test_conv_identity_tap():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 5, 6, 2))
    w = np.zeros((3, 3, 2, 2))
    w[1, 1] = np.eye(2)
    np.testing.assert_allclose(onet.conv3x3(x, w, np.zeros(2)), x, atol=0)
    # a shifted tap moves the image (zero fill at the border)
    w = np.zeros((3, 3, 2, 2))
    w[1, 2] = np.eye(2)  # reads x[:, i, j + 1]
    y = onet.conv3x3(x, w, np.zeros(2))
    np.testing.assert_allclose(y[:, :, :-1], x[:, :, 1:], atol=0)
    assert np.all(y[:, :, -1] == 0)


def _fd(f, a, eps=1e-6, n=12, seed=0):
    rng = np.random.default_rng(seed)
    idx = [tuple(rng.integers(0, s) for s in a.shape) for _ in range(n)]
    out = []
    for i in idx:
        a0 = a[i]
        a[i] = a0 + eps
        fp = f()
        a[i] = a0 - eps
        fm = f()
        a[i] = a0
        out.append((i, (fp - fm) / (2 * eps)))
    return out


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 6, 5, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    gy = rng.normal(size=(2, 6, 5, 4))
    f = lambda: float((onet.conv3x3(x, w, b) * gy).sum())
    gx, gw, gb = onet.conv3x3_backward(x, w, gy)
    for i, v in _fd(f, x):
        assert abs(gx[i] - v) <= 1e-6 * max(1, abs(v))
    for i, v in _fd(f, w):
        assert abs(gw[i] - v) <= 1e-6 * max(1, abs(v))
    for i, v in _fd(f, b, n=4):
        assert abs(gb[i] - v) <= 1e-6 * max(1, abs(v))


def test_net_backward_finite_differences():
    rng = np.random.default_rng(4)
    layers = [(rng.normal(0, 0.3, (3, 3, 4, 6)), rng.normal(0, 0.1, 6)),
              (rng.normal(0, 0.3, (3, 3, 6, 6)), rng.normal(0, 0.1, 6)),
              (rng.normal(0, 0.3, (3, 3, 6, 2)), rng.normal(0, 0.1, 2))]
    net = onet.Net(layers)
    x = rng.normal(size=(2, 5, 7, 4))
    gout = rng.normal(size=(2, 5, 7, 2))
    f = lambda: float((net.forward(x, round_act=False)[0] * gout).sum())
    _, acts = net.forward(x, round_act=False)
    grads = net.backward(acts, gout, round_grad=False)
    for li in range(3):
        w, b = net.layers[li]
        for i, v in _fd(f, w, n=6, seed=li):
            assert abs(grads[li][0][i] - v) <= 1e-5 * max(1, abs(v)), (li, i)
        for i, v in _fd(f, b, n=2, seed=li):
            assert abs(grads[li][1][i] - v) <= 1e-5 * max(1, abs(v)), (li, i)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(5)
    out = rng.normal(0, 2, size=(2, 4, 5, 2))
    tgt = out[..., 0] + rng.choice([-3.0, -0.2, 0.1, 0.3, 2.5], size=(2, 4, 5))
    valid = rng.uniform(size=(2, 4, 5)) < 0.8
    loss, g = onet.loss_and_grad(out, tgt, valid)
    f = lambda: onet.loss_and_grad(out, tgt, valid)[0]
    for i, v in _fd(f, out, eps=1e-7, n=20):
        assert abs(g[i] - v) <= 1e-6 * max(1, abs(v)), i
    # invalid pixels carry no gradient
    assert np.all(g[~valid] == 0)


def test_loss_closed_form():
    out = np.zeros((1, 1, 3, 2))
    out[0, 0, :, 0] = [0.2, 3.0, -1.0]
    out[0, 0, :, 1] = [0.0, 0.0, 2.0]
    tgt = np.zeros((1, 1, 3))
    valid = np.ones((1, 1, 3), bool)
    loss, _ = onet.loss_and_grad(out, tgt, valid, conf_weight=0.0)
    # Huber(0.2) = 0.02; Huber(3) = 2.5; Huber(-1) = 0.5 -> mean 1.0066...
    assert abs(loss - (0.02 + 2.5 + 0.5) / 3) < 1e-12


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = onet.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2 -> w - lr g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-7)


def test_net_input_channels():
    L = np.tile(np.arange(10, dtype=float) * 3 + 100, (4, 1))
    R = L + 6.0
    x = onet.net_input(L, R, ndisp=4)
    assert x.shape == (4, 10, 6)
    np.testing.assert_allclose(x[..., 0], (L - 128) / 64)
    np.testing.assert_allclose(x[..., 1], (R - 128) / 64)
    # R(x - d) = L(x) - 3 d + 6: |L - R(x - d)| = |3 d - 6| away from the left border
    for d in range(4):
        np.testing.assert_allclose(x[:, d:, 2 + d], abs(3 * d - 6) / 64)


def test_oracle_training_resumes_bitwise():
    """The oracle's training step (forward, loss, backward, Adam) run for
    3 + 3 steps with the state written to the checkpoint layout that
    include/bdis.h documents after step 3 and read back from it (FP32, as the
    GPU keeps it) ends where 6 uninterrupted steps end when the run keeps
    FP32 state too: resuming loses nothing."""
    import struct

    rng = np.random.default_rng(9)
    C = 16
    dims = [(16, C), (C, C), (C, C), (C, 2)]
    layers = [(rng.normal(0, np.sqrt(2 / (9 * ci)), (3, 3, ci, co)).astype(np.float32).astype(np.float64),
               np.zeros(co)) for ci, co in dims]
    x = onet.bf16(rng.normal(0, 1, (2, 6, 7, 16)))
    t = rng.uniform(0, 4, (2, 6, 7))
    valid = rng.uniform(size=(2, 6, 7)) > 0.2
    flat = lambda ls: np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ls])

    def unflat(v):
        out, o = [], 0
        for ci, co in dims:
            w = v[o:o + 9 * ci * co].reshape(3, 3, ci, co)
            o += 9 * ci * co
            out.append((w, v[o:o + co]))
            o += co
        return out

    def steps(w, m, v, first, count):
        for s in range(first, first + count):
            ls = [(onet.bf16(a), b) for a, b in unflat(w)]
            out, acts = onet.Net(ls).forward(x)
            _, g = onet.loss_and_grad(out, t, valid)
            grads = onet.Net(ls).backward(acts, g)
            gv = flat(grads)
            w, m, v = onet.adam(w, gv, m, v, s, 1e-3)
            w, m, v = (a.astype(np.float32).astype(np.float64) for a in (w, m, v))
        return w, m, v

    w0 = flat(layers)
    z = np.zeros_like(w0)
    wa, ma, va = steps(w0, z, z, 1, 6)
    wb, mb, vb = steps(w0, z, z, 1, 3)
    n = w0.size
    blob = b"BDISNET\0" + struct.pack("<IiqQ", 1, C, n, 3) + \
        np.concatenate([wb, mb, vb]).astype("<f4").tobytes()
    assert len(blob) == 32 + 12 * n
    ver, ch, nn, step = struct.unpack("<IiqQ", blob[8:32])
    arr = np.frombuffer(blob[32:], "<f4").astype(np.float64)
    assert (ver, ch, nn, step) == (1, C, n, 3)
    wc, mc, vc = steps(arr[:n], arr[n:2 * n], arr[2 * n:], step + 1, 3)
    np.testing.assert_array_equal(wc, wa)
    np.testing.assert_array_equal(mc, ma)
    np.testing.assert_array_equal(vc, va)
