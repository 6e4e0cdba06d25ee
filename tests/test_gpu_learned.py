"""Learned-init path on the GPU: network input against the oracle, the gate
(learned field and plain fallback), and the fine levels against the oracle
run from the same initial field.  Networks here are built by hand so that
their outputs are known: constant outputs come from the last layer's bias,
and a spatially varying confidence follows the left image."""
import numpy as np
import pytest

from oracle import net as onet
from paper_2106_07136_amd import synth
from tests.parity_util import assert_parity, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _const_net(C, d, logit):
    from paper_2106_07136_amd import net
    layers = [(np.zeros((3, 3, ci, co)), np.zeros(co)) for ci, co in net.layer_dims(C)]
    layers[3] = (layers[3][0], np.array([d, logit]))
    pn = net.ProposalNet(C)
    pn.set_params(net.flatten(layers))
    return pn


def _varying_net(C, d, gain, offset):
    """logit = gain * relu((L - 128) / 64) + offset, disparity d."""
    from paper_2106_07136_amd import net
    layers = [(np.zeros((3, 3, ci, co)), np.zeros(co)) for ci, co in net.layer_dims(C)]
    w0 = layers[0][0].copy()
    w0[1, 1, 0, 0] = 1.0
    layers[0] = (w0, layers[0][1])
    for li in (1, 2):
        w = layers[li][0].copy()
        w[1, 1, 0, 0] = 1.0
        layers[li] = (w, layers[li][1])
    w3 = layers[3][0].copy()
    w3[1, 1, 0, 1] = gain
    layers[3] = (w3, np.array([d, offset]))
    pn = net.ProposalNet(C)
    pn.set_params(net.flatten(layers))
    return pn


def _gpu(torch, pair):
    return torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda()


def test_net_input_matches_oracle(torch_cuda, ref):
    from paper_2106_07136_amd import bdis
    pairs = [synth.make_pair(640, 480, 64.0, s) for s in (21, 22)]
    h = bdis.Bdis(bdis.Params(levels=5))
    L = [torch_cuda.from_numpy(p.left).cuda() for p in pairs]
    R = [torch_cuda.from_numpy(p.right).cuda() for p in pairs]
    x = h.net_input(L, R).float().cpu().numpy().astype(np.float64)
    assert x.shape == (2, 30, 40, 16)
    for i, p in enumerate(pairs):
        _, tr = ref.compute(p.left, p.right, ref.Params(levels=5), trace=True)
        exp = onet.bf16(onet.net_input(tr[4]["pyr_l"], tr[4]["pyr_r"]))
        np.testing.assert_array_equal(x[i], exp)


def test_all_fallback_equals_plain(torch_cuda):
    """Confidence ~0 everywhere: every coarse level runs and replaces the
    whole initial field, so with learned_iters = iters the result is the
    plain path's, bit for bit."""
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, 31)
    L, R = _gpu(torch_cuda, pair)
    plain = bdis.Bdis(bdis.Params(levels=5)).compute(L, R).cpu().numpy()
    net = _const_net(32, 0.7, -10.0)
    h = bdis.Bdis(bdis.Params(levels=5, init=1, learned_iters=12))
    h.set_net(net)
    got = h.compute(L, R).cpu().numpy()
    np.testing.assert_array_equal(got.view(np.uint32), plain.view(np.uint32))


@pytest.mark.parametrize("iters", [12, 4])
def test_confident_proposal_matches_oracle(torch_cuda, ref, iters):
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, 32)
    L, R = _gpu(torch_cuda, pair)
    net = _const_net(32, 1.5, 10.0)
    gp = bdis.Params(levels=5, init=1, learned_iters=iters)
    h = bdis.Bdis(gp)
    h.set_net(net)
    got = h.compute(L, R).cpu().numpy()
    U2 = h.debug_stage(bdis.STAGE_FIELD, 2)
    # gate: u = -4 * 1.5 everywhere (the bias is exact in bfloat16 and FP32)
    np.testing.assert_array_equal(U2, np.full_like(U2, -6.0))
    exp = ref.compute_init(pair.left, pair.right, oracle_params(ref, gp), 2, U2, iters)
    assert_parity(got, exp, f"learned confident iters={iters}")


def test_partial_fallback_matches_oracle(torch_cuda, ref):
    """Confidence follows the left image: where it is low the plain coarse
    levels' field is used, elsewhere the learned one."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    pair = synth.make_pair(640, 480, 64.0, 33)
    L, R = _gpu(torch, pair)
    net = _varying_net(32, 2.0, 2000.0, -3.0)
    gp = bdis.Params(levels=5, init=1, learned_iters=12)
    h = bdis.Bdis(gp)
    h.set_net(net)
    got = h.compute(L, R).cpu().numpy()
    U2 = h.debug_stage(bdis.STAGE_FIELD, 2)
    _, tr = ref.compute(pair.left, pair.right, oracle_params(ref, bdis.Params(levels=5)), trace=True)
    plain2 = tr[2]["field"]
    learned = np.abs(U2 - (-8.0)) == 0
    from_plain = np.abs(U2 - plain2) <= 1e-6
    assert np.all(learned | from_plain)
    frac = learned.mean()
    assert 0.05 < frac < 0.95, frac
    exp = ref.compute_init(pair.left, pair.right, oracle_params(ref, gp), 2, U2, 12)
    assert_parity(got, exp, "learned partial fallback")


@pytest.mark.parametrize("mode", [0, 1])
def test_learned_batch_equals_single(torch_cuda, mode):
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [(640, 480, 64.0, 41), (320, 240, 32.0, 42), (640, 480, 64.0, 43)]
    pairs = [synth.make_pair(*s) for s in spec]
    net = _varying_net(32, 1.0, 2000.0, -3.0)
    gp = bdis.Params(levels=0, init=1, learned_iters=8)
    singles = []
    import dataclasses
    for p, s in zip(pairs, spec):
        h1 = bdis.Bdis(dataclasses.replace(gp, max_disparity=s[2]))
        h1.set_net(net)
        singles.append(h1.compute(*_gpu(torch, p)).cpu().numpy())
    h = bdis.Bdis(gp)
    h.set_net(net)
    h.set_batch_mode(mode)
    Ls = [torch.from_numpy(p.left).cuda() for p in pairs]
    Rs = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = h.compute_batch(Ls, Rs, max_disparity=[s[2] for s in spec])
    for o, r in zip(outs, singles):
        np.testing.assert_array_equal(o.cpu().numpy().view(np.uint32), r.view(np.uint32))


def test_learned_errors(torch_cuda):
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, 34)
    L, R = _gpu(torch_cuda, pair)
    h = bdis.Bdis(bdis.Params(levels=5, init=1))
    with pytest.raises(bdis.BdisError) as e:
        h.compute(L, R)
    assert e.value.status == bdis.E_STATE
    h.set_net(_const_net(32, 0.0, 10.0))
    h.set_batch_mode(2)
    with pytest.raises(bdis.BdisError) as e:
        h.compute_batch([L], [R])
    assert e.value.status == bdis.E_UNSUPPORTED
    small = synth.make_pair(24, 24, 2.0, 35)  # two LK levels: nothing below the injection level
    with pytest.raises(bdis.BdisError) as e:
        h.compute(*_gpu(torch_cuda, small))
    assert e.value.status == bdis.E_INVALID_ARG


def _epe_cov(outs, pairs):
    epe, cov = [], []
    for o, p in zip(outs, pairs):
        d = o.cpu().numpy()
        m = np.isfinite(d) & p.valid
        epe.append(float(np.abs(d[m] - p.disp[m]).mean()))
        cov.append(float(m.sum() / p.valid.sum()))
    return float(np.mean(epe)), float(np.mean(cov))


def test_trained_net_gains_over_plain(torch_cuda):
    """The shipped 32-channel network, on held-out 640x480 pairs it never saw
    (training used seeds 10000-31499): the learned init lowers the end-point
    error against the generator's ground truth at equal coverage."""
    import os

    from paper_2106_07136_amd import bdis, net, train
    torch = torch_cuda
    pairs = [synth.make_pair(640, 480, 64.0, 90000 + i) for i in range(8)]
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    flat, C, meta = train.load(os.path.join(os.path.dirname(bdis.__file__), "weights", "proposal_c32.npz"))
    assert C == 32 and meta["epochs"] > 0
    pn = net.ProposalNet(C)
    pn.set_params(flat)
    plain = bdis.Bdis(bdis.Params(levels=0)).compute_batch(L, R, max_disparity=[64.0] * 8)
    hl = bdis.Bdis(bdis.Params(levels=0, init=1, learned_iters=12))
    hl.set_net(pn)
    learned = hl.compute_batch(L, R, max_disparity=[64.0] * 8)
    e_p, c_p = _epe_cov(plain, pairs)
    e_l, c_l = _epe_cov(learned, pairs)
    print(f"plain EPE {e_p:.3f} coverage {c_p:.4f}; learned EPE {e_l:.3f} coverage {c_l:.4f}", flush=True)
    assert e_l < 0.9 * e_p
    assert c_l >= 0.98 * c_p


def test_training_reduces_loss(torch_cuda):
    """A few Adam steps of the GPU training loop (forward, loss, backward,
    Adam through the bdisnet kernels) on 32 generated 320x240 pairs with
    the plain method's targets lower the loss from its initial value."""
    from paper_2106_07136_amd import train
    data = train.build_dataset([(320, 240, 32.0, 32, 70000)], workers=1, chunk=32)
    X, T, V = data[0]
    assert X.shape == (32, 15, 20, 16) and T.shape == (32, 15, 20)
    assert int(V.sum().item()) > 0.5 * V.numel()
    _, hist = train.train(data, channels=32, epochs=20, batch=16, lr=2e-3, log_every=1)
    losses = [l for _, l in hist]
    assert len(losses) == 40 and all(np.isfinite(losses))
    print(f"loss {losses[0]:.4f} -> {np.mean(losses[-5:]):.4f}", flush=True)
    assert np.mean(losses[-5:]) < 0.8 * losses[0]
