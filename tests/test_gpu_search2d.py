"""GPU 2-D (x, y) patch search (bdis_compute_2d) against the FP64 oracle's
compute_2d: disparity and vertical offset, element by element, to the same
bar as the 1-D path (RMS <= 1e-3 px, |diff| <= 1e-2 px on >= 99.9 % of the
pixels, NaN masks equal on >= 99.9 %)."""
import numpy as np
import pytest

from paper_2106_07136_amd import synth
from tests.parity_util import assert_parity, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _shift2d(img, sx, sy):
    """R(x, y) = L(x + sx, y + sy), border replicated."""
    H, W = img.shape
    ys = np.clip(np.arange(H) + sy, 0, H - 1)
    xs = np.clip(np.arange(W) + sx, 0, W - 1)
    return img[ys][:, xs].copy()


def _run2d(torch, gp, left, right, pitch_pad=0, out_pad=0):
    from paper_2106_07136_amd import bdis
    h = bdis.Bdis(gp)
    H, W = left.shape
    Lb = torch.zeros((H, W + pitch_pad), dtype=torch.uint8, device="cuda")
    Rb = torch.zeros((H, W + pitch_pad), dtype=torch.uint8, device="cuda")
    Lb[:, :W] = torch.from_numpy(np.ascontiguousarray(left)).cuda()
    Rb[:, :W] = torch.from_numpy(np.ascontiguousarray(right)).cuda()
    ob = torch.full((H, W + out_pad), 7.0, dtype=torch.float32, device="cuda")
    vb = torch.full((H, W + out_pad), 7.0, dtype=torch.float32, device="cuda")
    d, v = h.compute_2d(Lb[:, :W], Rb[:, :W], ob[:, :W], vb[:, :W])
    torch.cuda.synchronize()
    if out_pad:
        assert torch.all(ob[:, W:] == 7.0).item() and torch.all(vb[:, W:] == 7.0).item()
    return h, d.cpu().numpy(), v.cpu().numpy()


def _both(torch, ref, gp, left, right, what, **kw):
    print(f"case {what}", flush=True)
    _, d, v = _run2d(torch, gp, left, right, **kw)
    ed, ev = ref.compute_2d(left, right, oracle_params(ref, gp))
    assert_parity(d, ed, what + " d")
    assert_parity(v, ev, what + " v")
    # a pixel has both components or neither
    np.testing.assert_array_equal(np.isfinite(d), np.isfinite(v))
    return d, v, ed, ev


@pytest.mark.parametrize("sx,sy", [(0, 2), (3, -2), (5, 1)])
def test_integer_2d_shift(torch_cuda, ref, sx, sy):
    """R(x, y) = L(x + sx, y + sy): d = sx and v = -sy away from the
    borders, on both sides."""
    from paper_2106_07136_amd import bdis
    L = synth.integer_shift_pair(128, 96, 0, seed=21).left
    R = _shift2d(L, sx, sy)
    gp = bdis.Params(levels=3, iters=12)
    d, v, _, _ = _both(torch_cuda, ref, gp, L, R, f"shift ({sx}, {sy})")
    m = 12
    di, vi = d[m:-m, m + abs(sx):-m - abs(sx)], v[m:-m, m + abs(sx):-m - abs(sx)]
    assert np.isfinite(di).mean() > 0.99
    assert np.nanmax(np.abs(di - sx)) <= 1e-3 and np.nanmax(np.abs(vi + sy)) <= 1e-3


# (W, H, d_max, seed, levels, iters, patch, stride, v_max)
MISALIGNED = {
    "160x120": (160, 120, 16.0, 1, 3, 8, 8, 4, 1.5),
    "640x480": (640, 480, 64.0, 2, 5, 12, 8, 4, 6.0),
    # ragged: 16 px patch columns do not tile 203 px; patches of 6 and 4
    "203x97_p6": (203, 97, 20.0, 7, 3, 10, 6, 3, 3.0),
    "150x77_p4": (150, 77, 12.0, 8, 2, 10, 4, 2, 2.0),
}


@pytest.mark.parametrize("name", sorted(MISALIGNED))
def test_misaligned_pair_parity(torch_cuda, ref, name):
    from paper_2106_07136_amd import bdis
    W, H, dm, seed, lv, it, P, st, vm = MISALIGNED[name]
    pair, _ = synth.misaligned_pair(W, H, dm, seed, v_max=vm)
    gp = bdis.Params(levels=lv, iters=it, patch=P, stride=st)
    _both(torch_cuda, ref, gp, pair.left, pair.right, name)


def test_large_pair_parity(torch_cuda, ref):
    """1280 x 720, six levels, up to 3 px of vertical offset: element parity
    beyond the headline size."""
    from paper_2106_07136_amd import bdis
    pair, _ = synth.misaligned_pair(1280, 720, 128.0, 3001, v_max=4.0)
    gp = bdis.Params(levels=6, iters=12)
    _both(torch_cuda, ref, gp, pair.left, pair.right, "1280x720")


def test_without_convergence_test_parity(torch_cuda, ref):
    """conv_tol = 0: only a non-finite translation or one that moved more
    than a patch side is discarded (the convergence test switched off)."""
    from paper_2106_07136_amd import bdis
    pair, _ = synth.misaligned_pair(160, 120, 16.0, 5, v_max=1.5)
    gp = bdis.Params(levels=3, iters=8, conv_tol=0.0)
    _both(torch_cuda, ref, gp, pair.left, pair.right, "conv_tol 0")


def test_wide_window_parity(torch_cuda, ref):
    """Nine window samples 0.25 px apart (the kernel's wider window bound)
    and s = patch side in eq. (4)."""
    from paper_2106_07136_amd import bdis
    pair, _ = synth.misaligned_pair(160, 120, 16.0, 3, v_max=2.0)
    gp = bdis.Params(levels=3, iters=10, window=9, window_step=0.25, s_mode=1)
    _both(torch_cuda, ref, gp, pair.left, pair.right, "window 9")


@pytest.mark.parametrize("sx,sy", [(3, -2), (0, 1)])
def test_fp32_recovers_integer_2d_shift(torch_cuda, sx, sy):
    """FP32 (precision = 1, not held to the parity bar, as for the 1-D path):
    the 2-D search still recovers a whole-pixel 2-D shift away from the
    borders."""
    from paper_2106_07136_amd import bdis
    L = synth.integer_shift_pair(128, 96, 0, seed=21).left
    R = _shift2d(L, sx, sy)
    _, d, v = _run2d(torch_cuda, bdis.Params(levels=3, iters=12, precision=1), L, R)
    m = 12
    di, vi = d[m:-m, m + abs(sx):-m - abs(sx)], v[m:-m, m + abs(sx):-m - abs(sx)]
    fin = np.isfinite(di)
    assert fin.mean() > 0.98
    assert (np.abs(di[fin] - sx) <= 1e-3).mean() >= 0.98 and (np.abs(vi[fin] + sy) <= 1e-3).mean() >= 0.98


def test_one_level_padded_pitch(torch_cuda, ref):
    """A single level (level 0 is also the coarsest: zero initial field)
    with padded input rows and output rows, whose padding stays untouched."""
    from paper_2106_07136_amd import bdis
    pair, _ = synth.misaligned_pair(96, 64, 3.0, 11, v_max=1.0)
    gp = bdis.Params(levels=1, iters=16)
    _both(torch_cuda, ref, gp, pair.left, pair.right, "one level", pitch_pad=40, out_pad=24)


def test_full_size_sampled_against_ground_truth(torch_cuda):
    """1920 x 1080 with up to 4.5 px of vertical offset, the size the oracle
    takes a minute on: the GPU's estimates against the generator's ground
    truth (a property at any size; element parity runs at 640 x 480),
    beside the 1-D search on the same pair, whose assumption of no vertical
    offset no longer holds."""
    from paper_2106_07136_amd import bdis
    pair, vg = synth.misaligned_pair(1920, 1080, 192.0, 50000, v_max=6.0)
    gp = bdis.Params(levels=7, iters=12)
    _, d, v = _run2d(torch_cuda, gp, pair.left, pair.right)
    h1 = bdis.Bdis(gp)
    L, R = torch_cuda.from_numpy(pair.left).cuda(), torch_cuda.from_numpy(pair.right).cuda()
    d1 = h1.compute(L, R).cpu().numpy()
    m = np.isfinite(d) & pair.valid
    m1 = np.isfinite(d1) & pair.valid
    e2 = np.abs(d - pair.disp)[m]
    e1 = np.abs(d1 - pair.disp)[m1]
    ev = np.abs(v - vg)[m]
    print(f"2-D: coverage {m.mean():.3f} median |d err| {np.median(e2):.3f} median |v err| {np.median(ev):.3f}; "
          f"1-D: coverage {m1.mean():.3f} median |d err| {np.median(e1):.3f}", flush=True)
    assert m.mean() > 0.7
    assert np.median(e2) < 0.5 and np.median(ev) < 0.35
    assert np.median(e2) < np.median(e1)


def test_without_vertical_output(torch_cuda, ref):
    """A null vertical output: the disparity is the same bits."""
    from paper_2106_07136_amd import bdis
    pair, _ = synth.misaligned_pair(160, 120, 16.0, 1, v_max=1.5)
    gp = bdis.Params(levels=3, iters=8)
    h = bdis.Bdis(gp)
    L, R = torch_cuda.from_numpy(pair.left).cuda(), torch_cuda.from_numpy(pair.right).cuda()
    d_a, v_a = h.compute_2d(L, R)
    d_b, v_b = h.compute_2d(L, R, with_v=False)
    assert v_b is None
    np.testing.assert_array_equal(d_a.cpu().numpy().view(np.uint32), d_b.cpu().numpy().view(np.uint32))


def _batch_inputs(torch, spec):
    pairs = [synth.misaligned_pair(W, H, dm, seed, v_max=vm)[0] for (W, H, dm, seed, vm) in spec]
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    return pairs, L, R


def test_batch_equals_single_pairs_and_oracle(torch_cuda, ref):
    """bdis_compute_batch_2d on pairs of mixed sizes (one without a vertical
    output) equals bdis_compute_2d pair by pair, bit for bit, and the oracle
    to the parity bar."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [(160, 120, 16.0, 1, 1.5), (203, 97, 20.0, 7, 3.0), (320, 240, 32.0, 9, 4.0), (96, 64, 6.0, 11, 1.0)]
    pairs, L, R = _batch_inputs(torch, spec)
    gp = bdis.Params(levels=3, iters=10)
    h = bdis.Bdis(gp)
    vouts = [torch.empty(l.shape, dtype=torch.float32, device="cuda") for l in L]
    vouts[3] = None
    D, V = h.compute_batch_2d(L, R, vouts=vouts)
    torch.cuda.synchronize()
    assert V[3] is None
    for i, p in enumerate(pairs):
        d1, v1 = h.compute_2d(L[i], R[i])
        np.testing.assert_array_equal(D[i].cpu().numpy().view(np.uint32), d1.cpu().numpy().view(np.uint32))
        if V[i] is not None:
            np.testing.assert_array_equal(V[i].cpu().numpy().view(np.uint32), v1.cpu().numpy().view(np.uint32))
        ed, ev = ref.compute_2d(p.left, p.right, oracle_params(ref, gp))
        assert_parity(D[i].cpu().numpy(), ed, f"batch pair {i} d")
        if V[i] is not None:
            assert_parity(V[i].cpu().numpy(), ev, f"batch pair {i} v")


def test_batch_over_one_pack(torch_cuda):
    """30 pairs, more than one launch's pack of jobs, each with its own
    max_disparity hint and so its own level count (1 to 4): bit for bit the
    single-pair results."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [(96 + 8 * (i % 3), 64 + 4 * (i % 2), 6.0, 100 + i, 1.0) for i in range(30)]
    pairs, L, R = _batch_inputs(torch, spec)
    dm = [4.0 + i for i in range(30)]
    h = bdis.Bdis(bdis.Params(levels=0, iters=8))
    D, V = h.compute_batch_2d(L, R, max_disparity=dm)
    torch.cuda.synchronize()
    for i in range(30):
        hs = bdis.Bdis(bdis.Params(levels=0, iters=8, max_disparity=dm[i]))
        d1, v1 = hs.compute_2d(L[i], R[i])
        np.testing.assert_array_equal(D[i].cpu().numpy().view(np.uint32), d1.cpu().numpy().view(np.uint32))
        np.testing.assert_array_equal(V[i].cpu().numpy().view(np.uint32), v1.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_groups_and_graph_same_bits(torch_cuda, mode):
    """30 pairs: as pair groups on streams of their own or on one stream,
    replayed from the level graph (mode 0, twice) or launched directly (mode
    1), the batched 2-D search gives the same d and v bits."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [(96 + 8 * (i % 3), 64 + 4 * (i % 2), 6.0, 300 + i, 1.0) for i in range(30)]
    pairs, L, R = _batch_inputs(torch, spec)
    dm = [4.0 + i for i in range(30)]
    res = {}
    for groups in (True, False):
        h = bdis.Bdis(bdis.Params(levels=0, iters=8))
        h.set_batch_mode(mode)
        h.set_batch_groups(groups)
        runs = []
        for _ in range(2):
            D, V = h.compute_batch_2d(L, R, max_disparity=dm)
            runs.append(([d.cpu().numpy() for d in D], [v.cpu().numpy() for v in V]))
        h.close()
        for a, b in zip(runs[0][0] + runs[0][1], runs[1][0] + runs[1][1]):
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
        res[groups] = runs[0]
    for a, b in zip(res[True][0] + res[True][1], res[False][0] + res[False][1]):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def test_bench_batch_matches_oracle(torch_cuda, ref):
    """The batched 2-D workload the bench times: the 64 mixed pairs (24 x
    320x240, 24 x 640x480, 16 x 1280x720, seeds from 3000), levels from each
    pair's max_disparity, in one call: every pair's d and v at the parity
    bar against the oracle."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    with ThreadPoolExecutor(16) as ex:
        pairs = list(ex.map(lambda a: synth.make_pair(*a), synth.mixed_batch_spec(3000)))
    h = bdis.Bdis(bdis.Params(levels=0, iters=12))
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    D, V = h.compute_batch_2d(L, R, max_disparity=[p.d_max for p in pairs])
    D = [d.cpu().numpy() for d in D]
    V = [v.cpu().numpy() for v in V]

    def oracle_of(p):
        H, W = p.left.shape
        lv = bdis.plan(bdis.Params(levels=0, max_disparity=p.d_max), W, H)["levels"]
        return ref.compute_2d(p.left, p.right, oracle_params(ref, bdis.Params(levels=lv, iters=12)))

    with ThreadPoolExecutor(16) as ex:
        exp = list(ex.map(oracle_of, pairs))
    for i, (p, d, v, (ed, ev)) in enumerate(zip(pairs, D, V, exp)):
        assert_parity(d, ed, f"2-D bench batch pair {i} d")
        assert_parity(v, ev, f"2-D bench batch pair {i} v")


@pytest.mark.parametrize("name,W,H,dmax,kw", [
    ("640x480", 640, 480, 64.0, dict(levels=5)),
    ("160x120_level0_folds", 160, 120, 16.0, dict(levels=3)),
    ("203x97_p6", 203, 97, 20.0, dict(levels=3, patch=6, stride=3)),
    ("150x77_p4_w9", 150, 77, 15.0, dict(levels=3, patch=4, stride=2, window=9, window_step=0.25)),
])
def test_folded_densify_same_bits(torch_cuda, name, W, H, dmax, kw):
    """The small LK launches densify the level above them (both fields)
    in place of that level's densify launch: the same d and v bits as one
    densify launch per level, on a single pair and in a batch."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    print(f"case {name}", flush=True)
    mis, _ = synth.misaligned_pair(W, H, dmax, W + H, v_max=3.0)
    L = torch.from_numpy(mis.left).cuda()
    R = torch.from_numpy(mis.right).cuda()
    res = {}
    for fold in (True, False):
        h = bdis.Bdis(bdis.Params(**kw))
        h.set_fold_densify(fold)
        d = torch.empty(L.shape, dtype=torch.float32, device="cuda")
        v = torch.empty_like(d)
        h.compute_2d(L, R, d, v)
        ds, vs = h.compute_batch_2d([L, L], [R, R], max_disparity=[dmax] * 2)
        res[fold] = (d.cpu().numpy(), v.cpu().numpy(), [(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(ds, vs)])
        h.close()
    for a, b in zip(res[True][:2], res[False][:2]):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    assert np.isfinite(res[True][0]).mean() > 0.3
    for (a1, b1), (a2, b2) in zip(res[True][2], res[False][2]):
        np.testing.assert_array_equal(a1.view(np.uint32), a2.view(np.uint32))
        np.testing.assert_array_equal(b1.view(np.uint32), b2.view(np.uint32))


def test_rejections(torch_cuda):
    """Patch sides above 8, eq. (2)'s fusion and the learned init are
    refused before any launch; the handle still runs afterwards."""
    from paper_2106_07136_amd import bdis
    L = torch_cuda.zeros((64, 64), dtype=torch_cuda.uint8, device="cuda")
    for kw in (dict(patch=12, stride=6), dict(fusion=1)):
        h = bdis.Bdis(bdis.Params(levels=2, **kw))
        with pytest.raises(bdis.BdisError) as e:
            h.compute_2d(L, L)
        assert e.value.status == bdis.E_UNSUPPORTED
    h = bdis.Bdis(bdis.Params(levels=2))
    with pytest.raises(bdis.BdisError) as e:
        h.compute_2d(L[:, :3], L[:, :3])
    assert e.value.status == bdis.E_INVALID_ARG
    d, v = h.compute_2d(L, L)
    torch_cuda.cuda.synchronize()
    assert d.shape == (64, 64)
