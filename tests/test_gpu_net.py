"""GPU proposal network against its FP64 oracle, on identical bfloat16
operands: forward layer by layer, input and weight gradients, loss and Adam.
Differences come only from FP32 accumulation order and, for values the
kernels store as bfloat16, from a rounding that falls the other way."""
import numpy as np
import pytest

from oracle import net as onet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(torch, C=32, N=2, H=9, W=13, seed=0):
    from paper_2106_07136_amd import net
    rng = np.random.default_rng(seed)
    flat = net.init_params(C, seed)
    # non-trivial biases and a last layer of normal size
    layers = net.unflatten(flat.astype(np.float64), C)
    layers = [(w * (10.0 if i == 3 else 1.0), rng.normal(0, 0.1, b.shape)) for i, (w, b) in enumerate(layers)]
    flat = net.flatten(layers)
    x = onet.bf16(rng.normal(0, 1, (N, H, W, 16)))
    pn = net.ProposalNet(C)
    pn.set_params(flat)
    xt = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
    # the oracle sees what the kernels see: bf16 weights, FP32 biases
    ol = [(onet.bf16(w), np.float32(b).astype(np.float64)) for w, b in net.unflatten(flat.astype(np.float64), C)]
    return pn, xt, x, ol, flat


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("C", [32, 48])
def test_forward_layer_by_layer(torch_cuda, C):
    pn, xt, x, ol, _ = _setup(torch_cuda, C=C)
    out = pn.forward(xt).cpu().numpy().astype(np.float64)
    N, H, W = x.shape[:3]
    acts = [pn.activation(l, (N, H, W)) for l in range(4)]
    np.testing.assert_array_equal(acts[0], x)
    ulp = 2.0 ** -7  # bf16 spacing relative to the value
    for l in range(3):
        w, b = ol[l]
        ref = onet.bf16(onet.relu(onet.conv3x3(acts[l], w, b)))
        got = acts[l + 1]
        diff = np.abs(got - ref)
        assert np.all(diff <= ulp * np.abs(ref) + 1e-30), (l, diff.max())
        assert (diff == 0).mean() >= 0.99, (l, (diff == 0).mean())
    w, b = ol[3]
    ref = onet.conv3x3(acts[3], w, b)
    assert _rel(out, ref) <= 1e-5


def test_backward_matches_oracle(torch_cuda):
    torch = torch_cuda
    C = 32
    pn, xt, x, ol, _ = _setup(torch, C=C, seed=1)
    N, H, W = x.shape[:3]
    pn.forward(xt)
    acts = [pn.activation(l, (N, H, W)) for l in range(4)]
    rng = np.random.default_rng(7)
    gout = rng.normal(0, 1, (N, H, W, 2)).astype(np.float32)
    pn.set_output_grad(torch.from_numpy(gout).cuda())
    pn.backward()
    g = pn.get_grads()
    from paper_2106_07136_amd import net
    gl = net.unflatten(g.astype(np.float64), C)
    ref = onet.Net(ol).backward(acts, gout.astype(np.float64), round_grad=True)
    # last layer: exact operands -> only accumulation order
    assert _rel(gl[3][0], ref[3][0]) <= 1e-5 and _rel(gl[3][1], ref[3][1]) <= 1e-5
    # earlier layers: the propagated gradient is stored in bfloat16 by both
    for l in range(3):
        assert _rel(gl[l][0], ref[l][0]) <= 2e-3, l
        assert _rel(gl[l][1], ref[l][1]) <= 2e-3, l
    # deterministic
    pn.backward()
    np.testing.assert_array_equal(pn.get_grads(), g)


def test_loss_and_adam_match_oracle(torch_cuda):
    torch = torch_cuda
    C = 32
    pn, xt, x, ol, flat = _setup(torch, C=C, seed=2)
    N, H, W = x.shape[:3]
    out = pn.forward(xt).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(3)
    tgt = (out[..., 0] + rng.choice([-2.0, -0.3, 0.1, 0.4, 1.7], size=(N, H, W))).astype(np.float32)
    valid = (rng.uniform(size=(N, H, W)) < 0.8)
    loss = pn.loss(torch.from_numpy(tgt).cuda(), torch.from_numpy(valid.astype(np.uint8)).cuda()).item()
    rl, rg = onet.loss_and_grad(out, tgt.astype(np.float64), valid)
    assert abs(loss - rl) <= 1e-5 * max(1.0, abs(rl))
    pn.backward()
    g = pn.get_grads()
    acts = [pn.activation(l, (N, H, W)) for l in range(4)]
    from paper_2106_07136_amd import net
    ref = onet.Net(ol).backward(acts, rg, round_grad=True)
    gl = net.unflatten(g.astype(np.float64), C)
    assert _rel(gl[3][0], ref[3][0]) <= 1e-3
    # one Adam step from these gradients
    pn.adam_step(lr=1e-2, step=1)
    w1 = pn.get_params().astype(np.float64)
    exp, _, _ = onet.adam(flat.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr=1e-2)
    assert np.max(np.abs(w1 - exp)) <= 1e-6
