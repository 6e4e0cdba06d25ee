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


def _train_steps(torch, pn, X, T, V, steps, first=1):
    for s in range(first, first + steps):
        pn.forward(X)
        pn.loss(T, V, delta=1.0, conf_tol=1.0, conf_weight=0.1)
        pn.backward()
        pn.adam_step(1e-3 * (1.0 + 0.1 * s), s)
    torch.cuda.synchronize()


def _rand_batch(torch, N=4, H=12, W=16, seed=3):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = (torch.rand((N, H, W, 16), generator=g) * 2 - 1).to(torch.bfloat16).cuda().contiguous()
    T = (torch.rand((N, H, W), generator=g) * 4).cuda().contiguous()
    V = (torch.rand((N, H, W), generator=g) > 0.2).to(torch.uint8).cuda().contiguous()
    return X, T, V


def _parse_checkpoint(blob):
    """The checkpoint layout include/bdis.h documents."""
    assert blob[:8] == b"BDISNET\0"
    ver, C = np.frombuffer(blob[8:16], np.int32)
    n, step = np.frombuffer(blob[16:32], np.int64)
    arr = np.frombuffer(blob[32:], np.float32)
    assert arr.size == 3 * n
    return dict(version=int(ver), channels=int(C), n=int(n), step=int(step), w=arr[:n], m=arr[n:2 * n],
                v=arr[2 * n:])


def test_checkpoint_resume_is_bitwise(torch_cuda):
    """Six Adam steps in one go against three, a checkpoint, a new network
    loaded from it and three more: weights, both moments and the step count
    equal bit for bit (forward, backward and Adam are deterministic)."""
    from paper_2106_07136_amd import net
    torch = torch_cuda
    X, T, V = _rand_batch(torch)
    flat = net.init_params(32, 1)
    a = net.ProposalNet(32)
    a.set_params(flat)
    _train_steps(torch, a, X, T, V, 6)
    b = net.ProposalNet(32)
    b.set_params(flat)
    _train_steps(torch, b, X, T, V, 3)
    blob = b.save_checkpoint()
    ck = _parse_checkpoint(blob)
    assert (ck["version"], ck["channels"], ck["n"], ck["step"]) == (1, 32, b.nparam, 3)
    np.testing.assert_array_equal(ck["w"], b.get_params())
    assert np.all(ck["v"] >= 0) and np.any(ck["m"] != 0)
    b.close()
    c = net.ProposalNet(32)
    c.load_checkpoint(blob)
    assert c.step == 3
    _train_steps(torch, c, X, T, V, 3, first=4)
    assert a.save_checkpoint() == c.save_checkpoint()


def test_training_run_resumes_bitwise(torch_cuda):
    """train.train stopped after 5 of 9 steps (mid-epoch) and resumed from
    its state ends where the uninterrupted run ends, bit for bit; the state
    survives a round trip through its .npz file."""
    import os
    import tempfile

    from paper_2106_07136_amd import train
    torch = torch_cuda
    X, T, V = _rand_batch(torch, N=24, seed=4)
    data = [(X, T, V)]
    full = {}
    train.train(data, channels=32, epochs=3, batch=8, lr=2e-3, log_every=100, state_out=full)
    part = {}
    train.train(data, channels=32, epochs=3, batch=8, lr=2e-3, log_every=100, stop_after=5, state_out=part)
    assert part["step"] == 5 and part["epoch"] == 1 and part["pos"] == 2
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "state.npz")
        train.save_state(path, part)
        resumed_from = train.load_state(path)
    rest = {}
    train.train(data, channels=32, epochs=3, batch=8, lr=2e-3, log_every=100, resume=resumed_from, state_out=rest)
    assert rest["step"] == full["step"] == 9
    assert rest["net"] == full["net"]


def test_set_net_weights_equals_attached_network(torch_cuda):
    """A handle that loads a checkpoint into a network of its own computes
    the same learned-init disparity, bit for bit, as one given the network
    object; wrong checkpoints are refused."""
    from paper_2106_07136_amd import bdis, net, synth
    torch = torch_cuda
    pair = synth.make_pair(640, 480, 64.0, 52)
    L, R = torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda()
    pn = net.ProposalNet(32)
    pn.set_params(net.init_params(32, 7))
    gp = bdis.Params(levels=5, init=1, learned_iters=8)
    h1 = bdis.Bdis(gp)
    h1.set_net(pn)
    d1 = h1.compute(L, R).cpu().numpy()
    h2 = bdis.Bdis(gp)
    h2.set_net_weights(pn.save_checkpoint())
    d2 = h2.compute(L, R).cpu().numpy()
    np.testing.assert_array_equal(d1.view(np.uint32), d2.view(np.uint32))
    bad = bytearray(pn.save_checkpoint())
    bad[0:1] = b"X"
    with pytest.raises(bdis.BdisError) as e:
        h2.set_net_weights(bytes(bad))
    assert e.value.status == bdis.E_INVALID_ARG
    p48 = net.ProposalNet(48)
    with pytest.raises(bdis.BdisError) as e:
        p48.load_checkpoint(pn.save_checkpoint())
    assert e.value.status == bdis.E_INVALID_ARG
    # the owned network stays usable after the refusals
    d3 = h2.compute(L, R).cpu().numpy()
    np.testing.assert_array_equal(d1.view(np.uint32), d3.view(np.uint32))
