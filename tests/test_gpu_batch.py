"""Batched execution: per-level launches replayed from a hipGraph (mode 0),
the same launches issued directly (mode 1) and one persistent launch
replayed from a hipGraph (mode 2) must all give, bit for bit, what
bdis_compute gives on each pair alone, for pairs of mixed sizes and pyramid
depths.  Graph replays with new buffers and repeated replays with eager
work in between are checked replay by replay."""
import numpy as np
import pytest

from paper_2106_07136_amd import synth
from tests.parity_util import assert_parity, oracle_params, shifted_right

pytestmark = pytest.mark.gpu

# (width, height, max disparity, seed): levels come from the disparity
MIXED = [(160, 120, 16.0, 1), (320, 240, 32.0, 2), (97, 61, 8.0, 3), (160, 120, 16.0, 4),
         (200, 150, 20.0, 5), (64, 48, 6.0, 6), (640, 480, 64.0, 7)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pairs(torch, spec, seed_shift=0):
    out = []
    for (W, H, d, s) in spec:
        p = synth.make_pair(W, H, d, s + seed_shift)
        out.append((p, torch.from_numpy(p.left).cuda(), torch.from_numpy(p.right).cuda(), d))
    return out


def _single(torch, base, pairs, patch=None, stride=None):
    """Reference: each pair alone through bdis_compute with its own max disparity."""
    import dataclasses

    from paper_2106_07136_amd import bdis
    res = []
    for (p, L, R, d) in pairs:
        prm = dataclasses.replace(base, max_disparity=d, patch=patch or base.patch,
                                  stride=stride or base.stride)
        h = bdis.Bdis(prm)
        res.append(h.compute(L, R).cpu().numpy())
        h.close()
    return res


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def _run_batch(h, pairs, outs=None):
    lefts = [q[1] for q in pairs]
    rights = [q[2] for q in pairs]
    outs = h.compute_batch(lefts, rights, outs, max_disparity=[q[3] for q in pairs])
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_equals_single(torch_cuda, mode):
    from paper_2106_07136_amd import bdis
    base = bdis.Params(levels=0, iters=10)
    pairs = _pairs(torch_cuda, MIXED)
    ref = _single(torch_cuda, base, pairs)
    h = bdis.Bdis(base)
    h.set_batch_mode(mode)
    got = _run_batch(h, pairs)
    assert h.batch_error() == 0
    for i, (g, r) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(_bits(g), _bits(r), err_msg=f"pair {i} mode {mode}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_outside_staged_span_equals_single(torch_cuda, mode):
    """The shifted 1920x1080 pairs whose iterates leave the LK blocks'
    staged columns (160 px against a max_disparity of 4, -80 px against
    1000), batched with two ordinary pairs: every execution gives what
    bdis_compute gives on each pair alone, bit for bit.  Their fallback
    reads then run in the batch's larger launches and, in mode 2, in the
    persistent kernel."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    left = synth.make_pair(1920, 1080, 192.0, 61).left
    pairs = [(None, torch.from_numpy(left).cuda(), torch.from_numpy(shifted_right(left, s)).cuda(), d)
             for s, d in ((160, 4.0), (-80, 1000.0))]
    pairs += _pairs(torch, [(640, 480, 64.0, 7), (320, 240, 32.0, 2)])
    base = bdis.Params(levels=7, iters=12)
    ref = _single(torch, base, pairs)
    h = bdis.Bdis(base)
    h.set_batch_mode(mode)
    got = _run_batch(h, pairs)
    assert h.batch_error() == 0
    for i, (g, r) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(_bits(g), _bits(r), err_msg=f"pair {i} mode {mode}")


def test_batch_pair_matches_oracle(torch_cuda, ref):
    from paper_2106_07136_amd import bdis
    base = bdis.Params(levels=0, iters=10)
    pairs = _pairs(torch_cuda, MIXED[:3])
    h = bdis.Bdis(base)
    got = _run_batch(h, pairs)
    for (p, _, _, d), g in zip(pairs, got):
        H, W = p.left.shape
        L = bdis.plan(bdis.Params(levels=0, max_disparity=d), W, H)["levels"]
        exp = ref.compute(p.left, p.right, oracle_params(ref, bdis.Params(levels=L, iters=10)))
        assert_parity(g, exp, f"batch {W}x{H}")


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_groups_same_bits(torch_cuda, mode):
    """60 pairs (more than one job pack): the batch as three pair groups on
    their own streams gives the same bits as on one stream, in the graph and
    in direct launches, and again on a second call with new outputs."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [((64, 48), (97, 61), (160, 120), (320, 240))[i % 4] + (6.0 + (i % 5), 700 + i) for i in range(60)]
    pairs = _pairs(torch, spec)
    res = {}
    for groups in (True, False):
        h = bdis.Bdis(bdis.Params(levels=0, iters=10))
        h.set_batch_mode(mode)
        h.set_batch_groups(groups)
        first = _run_batch(h, pairs)
        second = _run_batch(h, pairs)
        for a, b in zip(first, second):
            np.testing.assert_array_equal(_bits(a), _bits(b))
        res[groups] = first
        h.close()
    for a, b in zip(res[True], res[False]):
        np.testing.assert_array_equal(_bits(a), _bits(b))


def test_bench_batch_matches_oracle(torch_cuda, ref):
    """The batched workload as the bench times it: the 64 pairs of mixed
    sizes (24 x 320x240, 24 x 640x480, 16 x 1280x720, seeds from 3000,
    disparity up to 10 % of the width) in one level-graph call at patch 8,
    stride 4, 12 iterations, levels from each pair's max_disparity: every
    pair's whole disparity map at the parity bar against the oracle."""
    from concurrent.futures import ThreadPoolExecutor

    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = synth.mixed_batch_spec(3000)
    with ThreadPoolExecutor(16) as ex:
        pairs = list(ex.map(lambda a: synth.make_pair(*a), spec))
    base = bdis.Params(levels=0, iters=12)
    h = bdis.Bdis(base)
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    outs = h.compute_batch(L, R, max_disparity=[p.d_max for p in pairs])
    got = [o.cpu().numpy() for o in outs]

    def oracle_of(p):
        H, W = p.left.shape
        lv = bdis.plan(bdis.Params(levels=0, max_disparity=p.d_max), W, H)["levels"]
        return ref.compute(p.left, p.right, oracle_params(ref, bdis.Params(levels=lv, iters=12)))

    with ThreadPoolExecutor(16) as ex:
        exp = list(ex.map(oracle_of, pairs))
    for i, (p, g, e) in enumerate(zip(pairs, got, exp)):
        assert_parity(g, e, f"bench batch pair {i} {p.left.shape[1]}x{p.left.shape[0]}")


@pytest.mark.parametrize("mode", [0, 2])
def test_graph_replay_with_new_buffers(torch_cuda, mode):
    """Graph modes: mode 0 updates its graph for new buffers, mode 2 keeps
    its graph and re-uploads the task tables.  Every replay is checked
    against the eager per-pair results, with unrelated torch work between
    replays."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    base = bdis.Params(levels=0, iters=8)
    spec = MIXED[:4]
    A = _pairs(torch, spec)
    B = _pairs(torch, spec, seed_shift=100)
    refA = _single(torch, base, A)
    refB = _single(torch, base, B)
    h = bdis.Bdis(base)
    h.set_batch_mode(mode)
    outs = [torch.empty(q[1].shape, dtype=torch.float32, device="cuda") for q in A]
    for rep in range(3):
        for pairs, ref in ((A, refA), (B, refB)):
            got = _run_batch(h, pairs, outs)
            assert h.batch_error() == 0
            for i, (g, r) in enumerate(zip(got, ref)):
                np.testing.assert_array_equal(_bits(g), _bits(r), err_msg=f"replay {rep} pair {i}")
            x = torch.randn(512, 512, device="cuda")
            (x @ x).sum().item()  # eager work between replays
    # the same buffers again: no table upload, plain replay
    for rep in range(3):
        got = _run_batch(h, B, outs)
        for g, r in zip(got, refB):
            np.testing.assert_array_equal(_bits(g), _bits(r))


def test_tuning_table_selects_patch_and_stride(torch_cuda):
    from paper_2106_07136_amd import bdis
    base = bdis.Params(levels=0, iters=8, autotune=1)
    small = [q for q in MIXED if q[0] <= 160][:3]
    large = [q for q in MIXED if q[0] > 160][:2]
    S = _pairs(torch_cuda, small)
    Lg = _pairs(torch_cuda, large)
    refS = _single(torch_cuda, bdis.Params(levels=0, iters=8), S, patch=12, stride=3)
    refL = _single(torch_cuda, bdis.Params(levels=0, iters=8), Lg, patch=8, stride=6)
    for mode in (0, 1, 2):
        h = bdis.Bdis(base)
        h.set_batch_mode(mode)
        h.set_tuning([(160, 12, 3), (100000, 8, 6)])
        got = _run_batch(h, S + Lg)
        for g, r in zip(got, refS + refL):
            np.testing.assert_array_equal(_bits(g), _bits(r))


def test_persistent_mode_patch_limits(torch_cuda):
    from paper_2106_07136_amd import bdis
    pairs = _pairs(torch_cuda, MIXED[:2])
    h = bdis.Bdis(bdis.Params(levels=0, patch=16, stride=8))
    h.set_batch_mode(2)
    with pytest.raises(bdis.BdisError) as e:
        _run_batch(h, pairs)
    assert e.value.status == bdis.E_UNSUPPORTED
    for mode in (0, 1):
        h.set_batch_mode(mode)
        got = _run_batch(h, pairs)
        assert all(np.isfinite(g).any() for g in got)


def test_batch_fp32(torch_cuda):
    from paper_2106_07136_amd import bdis
    base = bdis.Params(levels=0, iters=8, precision=1)
    pairs = _pairs(torch_cuda, MIXED[:4])
    ref = _single(torch_cuda, base, pairs)
    for mode in (0, 2):
        h = bdis.Bdis(base)
        h.set_batch_mode(mode)
        got = _run_batch(h, pairs)
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(_bits(g), _bits(r))


def test_wgs_per_cu_setting(torch_cuda):
    from paper_2106_07136_amd import bdis
    base = bdis.Params(levels=0, iters=8)
    pairs = _pairs(torch_cuda, MIXED[:3])
    ref = _single(torch_cuda, base, pairs)
    h = bdis.Bdis(base)
    for w in (1, 2):
        h.set_batch_mode(2, w)
        got = _run_batch(h, pairs)
        assert h.batch_error() == 0
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(_bits(g), _bits(r))


@pytest.mark.parametrize("fusion", [0, 1])
def test_folded_densify_matches_separate_launches(torch_cuda, fusion):
    """Densifying level l+1 inside the LK launch of level l (the default)
    gives every level's field and the output of one densify launch per
    level, bit for bit (eq. (2)'s fusion keeps its own launches: same
    result by construction)."""
    from paper_2106_07136_amd import bdis
    pair = synth.make_pair(640, 480, 64.0, 61)
    L, R = torch_cuda.from_numpy(pair.left).cuda(), torch_cuda.from_numpy(pair.right).cuda()
    res = []
    for fold in (True, False):
        h = bdis.Bdis(bdis.Params(levels=5, fusion=fusion))
        h.set_fold_densify(fold)
        out = h.compute(L, R).cpu().numpy()
        fields = [h.debug_stage(bdis.STAGE_FIELD, l) for l in range(1, 5)]
        res.append((out, fields))
    np.testing.assert_array_equal(_bits(res[0][0]), _bits(res[1][0]))
    for a, b in zip(res[0][1], res[1][1]):
        np.testing.assert_array_equal(np.ascontiguousarray(a).view(np.uint64), np.ascontiguousarray(b).view(np.uint64))


def test_batch_beyond_one_job_pack(torch_cuda):
    """60 pairs: every level's launch holds at most 24 jobs, so the batch is
    split over several launches per level; each pair still equals its own
    bdis_compute, in all three executions."""
    from paper_2106_07136_amd import bdis
    spec = [((64, 48), (97, 61), (160, 120))[i % 3] + (6.0 + (i % 5), 500 + i) for i in range(60)]
    pairs = _pairs(torch_cuda, spec)
    base = bdis.Params(levels=0, iters=8)
    ref = _single(torch_cuda, base, pairs)
    for mode in (0, 1, 2):
        h = bdis.Bdis(base)
        h.set_batch_mode(mode)
        got = _run_batch(h, pairs)
        assert h.batch_error() == 0
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(_bits(g), _bits(r))


def test_batch_size_limits(torch_cuda):
    from paper_2106_07136_amd import bdis
    h = bdis.Bdis(bdis.Params(levels=0))
    with pytest.raises(bdis.BdisError) as e:
        h.compute_batch([], [])
    assert e.value.status == bdis.E_INVALID_ARG
