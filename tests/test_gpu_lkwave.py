"""The one-wave-per-patch LK kernel (k_lkw) against the one-lane-per-row
kernel (k_lk): both form every patch sum in one fixed order, so the library
must give the same bits whichever of them a launch takes.  Each case runs
with every eligible LK launch on k_lkw (patch sides up to 8) and with none,
and compares the disparity maps bit for bit; the parity tests check the
default mix (coarse levels on k_lkw) against the oracle."""
import numpy as np
import pytest

from paper_2106_07136_amd import synth

pytestmark = pytest.mark.gpu

ALL = 1 << 20  # patches per CU: every eligible launch on k_lkw


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def _compute(torch, params, pair, wave, fold=True):
    from paper_2106_07136_amd import bdis
    h = bdis.Bdis(params)
    h.set_wave_lk(wave)
    h.set_fold_densify(fold)
    L = torch.from_numpy(np.ascontiguousarray(pair.left)).cuda()
    R = torch.from_numpy(np.ascontiguousarray(pair.right)).cuda()
    out = torch.empty(L.shape, dtype=torch.float32, device="cuda")
    h.compute(L, R, out)
    res = out.cpu().numpy()
    h.close()
    return res


CASES = {
    "p8_640x480": (640, 480, 64.0, dict(levels=5, iters=12), True),
    "p8_odd_203x97": (203, 97, 20.0, dict(levels=3), True),
    "p8_fold_off": (320, 240, 32.0, dict(levels=4), False),
    "p4_st2": (96, 64, 9.6, dict(levels=3, patch=4, stride=2), True),
    "p6_st6": (96, 64, 9.6, dict(levels=3, patch=6, stride=6), True),
    "p6_st3_150x77": (150, 77, 15.0, dict(levels=3, patch=6, stride=3), True),
    "window9": (160, 120, 16.0, dict(levels=3, window=9, window_step=0.25), True),
    "window3_s_is_patch": (128, 96, 12.8, dict(levels=2, window=3, window_step=1.0, s_mode=1), True),
    "valid_band": (128, 96, 12.8, dict(levels=2, valid_lo=90, valid_hi=160), True),
    "dis_fusion": (128, 96, 12.8, dict(levels=3, fusion=1), True),
    "conv_tol_0": (640, 480, 64.0, dict(levels=5, conv_tol=0.0), True),
    "fp32": (640, 480, 64.0, dict(levels=5, precision=1), True),
    "stride8": (640, 480, 64.0, dict(levels=5, stride=8), True),
    "no_iters": (96, 64, 9.6, dict(levels=2, iters=0), True),
    "gamma_025": (160, 120, 16.0, dict(levels=3, gamma=0.25), True),
    "min_8x8": (8, 8, 2.0, dict(levels=3), True),
    "auto_levels_1280x720": (1280, 720, 128.0, dict(levels=0, max_disparity=128.0), True),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_wave_kernel_same_bits(torch_cuda, name):
    from paper_2106_07136_amd import bdis
    W, H, dmax, kw, fold = CASES[name]
    print(f"case {name}", flush=True)
    pair = synth.make_pair(W, H, dmax, seed=W * 3 + H)
    gp = bdis.Params(**kw)
    rows = _compute(torch_cuda, gp, pair, 0, fold)
    waves = _compute(torch_cuda, gp, pair, ALL, fold)
    dflt = _compute(torch_cuda, gp, pair, 8, fold)
    assert np.isfinite(rows).mean() > 0.3 or name in ("min_8x8", "no_iters")
    np.testing.assert_array_equal(_bits(waves), _bits(rows))
    np.testing.assert_array_equal(_bits(dflt), _bits(rows))


def test_wave_kernel_batch_same_bits(torch_cuda):
    """30 mixed pairs in one call (more than one job pack per launch): all
    LK launches on the row kernel, the default mix, and every eligible one
    on k_lkw give the same bits, each pair equal to its single-pair result."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    spec = [((64, 48), (97, 61), (160, 120), (320, 240), (203, 97))[i % 5] + (6.0 + (i % 4), 900 + i)
            for i in range(30)]
    pairs = [synth.make_pair(*s) for s in spec]
    L = [torch.from_numpy(p.left).cuda() for p in pairs]
    R = [torch.from_numpy(p.right).cuda() for p in pairs]
    res = {}
    for wave in (0, 8, ALL):
        h = bdis.Bdis(bdis.Params(levels=0, iters=10))
        h.set_wave_lk(wave)
        res[wave] = [o.cpu().numpy() for o in h.compute_batch(L, R, max_disparity=[s[2] for s in spec])]
        h.close()
    for i in range(len(pairs)):
        np.testing.assert_array_equal(_bits(res[8][i]), _bits(res[0][i]))
        np.testing.assert_array_equal(_bits(res[ALL][i]), _bits(res[0][i]))
    for i in (0, 3, 7):
        import dataclasses
        single = _compute(torch, dataclasses.replace(bdis.Params(levels=0, iters=10), max_disparity=spec[i][2]),
                          pairs[i], 8)
        np.testing.assert_array_equal(_bits(single), _bits(res[0][i]))


def test_wave_knob_rejects_negative(torch_cuda):
    from paper_2106_07136_amd import bdis
    h = bdis.Bdis(bdis.Params())
    with pytest.raises(bdis.BdisError):
        h.set_wave_lk(-1)
    h.close()
