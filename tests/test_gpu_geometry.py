"""The steps around the matcher on the GPU (rectification and undistortion
before it, depth after it) against the FP64 oracle, and the whole chain raw
pair -> rectified pair -> disparity -> depth.  Inputs: seeded synthetic
pairs taken as raw captures, and a seeded synthetic rig calibration."""
import numpy as np
import pytest

from paper_2106_07136_amd import synth
from tests.parity_util import ABS_TOL, assert_parity, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cams(ref, rig):
    from paper_2106_07136_amd import bdis
    return ([bdis.Camera(**rig[s]) for s in ("left", "right")],
            [ref.Camera(**rig[s]) for s in ("left", "right")])


@pytest.mark.parametrize("seed", [1, 2])
def test_rectify_pair_matches_oracle(torch_cuda, ref, seed):
    """Both images of a 640x480 pair in one launch, each with its own lens,
    rotation and camera matrix: every output pixel equals the oracle's (the
    source position and the interpolation are the same FP64 operations)."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    print(f"case rectify 640x480 rig seed {seed}", flush=True)
    pair = synth.make_pair(640, 480, 64.0, 40 + seed)
    rig = synth.stereo_rig(640, 480, seed)
    gcams, ocams = _cams(ref, rig)
    srcs = [torch.from_numpy(pair.left).cuda(), torch.from_numpy(pair.right).cuda()]
    outs = bdis.rectify(srcs, gcams)
    torch.cuda.synchronize()
    for o, raw, oc in zip(outs, (pair.left, pair.right), ocams):
        exp = ref.rectify(oc, raw)
        got = o.cpu().numpy()
        assert (exp != raw).mean() > 0.5  # the rig moves the image
        np.testing.assert_array_equal(got, exp)


def test_rectify_sizes_and_pitches(torch_cuda, ref):
    """A 1280x720 raw image with a padded pitch into a 637x481 output whose
    pitch is not a multiple of 4 (byte stores), and a 3x5 output (tails)."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    raw = synth.make_pair(1280, 720, 32.0, 44).left
    rig = synth.stereo_rig(1280, 720, 3)
    cam = dict(rig["left"], nfx=rig["left"]["nfx"] / 2, nfy=rig["left"]["nfy"] / 2, ncx=318.0, ncy=240.0)
    buf = torch.zeros((720, 1291), dtype=torch.uint8, device="cuda")
    buf[:, :1280] = torch.from_numpy(raw).cuda()
    src = buf[:, :1280]
    obuf = torch.full((481, 639), 7, dtype=torch.uint8, device="cuda")
    out = obuf[:, :637]
    small = torch.full((3, 5), 7, dtype=torch.uint8, device="cuda")
    bdis.rectify([src, src], [bdis.Camera(**cam), bdis.Camera(**cam)], outs=[out, small])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.rectify(ref.Camera(**cam), raw, (481, 637)))
    np.testing.assert_array_equal(small.cpu().numpy(), ref.rectify(ref.Camera(**cam), raw, (3, 5)))
    assert torch.all(obuf[:, 637:] == 7).item()


def test_depth_matches_oracle(torch_cuda, ref):
    """Z = f B / d on a disparity grid with NaNs, zeros and negatives: the
    float32 output is the FP64 value rounded once, as the oracle's."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    rng = np.random.default_rng(5)
    d = rng.uniform(-2.0, 80.0, (480, 640)).astype(np.float32)
    d[rng.uniform(size=d.shape) < 0.05] = np.nan
    d[0, :10] = 0.0
    z = bdis.depth_from_disparity(torch.from_numpy(d).cuda(), 512.5, 4.8, min_disparity=0.5)
    exp = ref.depth(d.astype(np.float64), 512.5, 4.8, d_min=np.float64(np.float32(0.5)))
    got = z.cpu().numpy()
    np.testing.assert_array_equal(np.isnan(got), np.isnan(exp))
    fin = np.isfinite(exp)
    np.testing.assert_array_equal(got[fin], exp[fin].astype(np.float32))


def test_rectified_pipeline_matches_oracle(torch_cuda, ref):
    """Raw pair -> rectify (both cameras) -> BDIS -> depth in mm, against the
    oracle's chain on the same raw pair: the disparity at the parity bar, the
    depth to the relative error that bar allows where d >= 2 px.  The raw
    pair is what the synthetic rig would record of a generated rectified
    pair, so rectifying it recovers that pair."""
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    pair = synth.make_pair(640, 480, 64.0, 46)
    rig = synth.stereo_rig(640, 480, 4)
    raw = [synth.raw_capture(pair.left, rig["left"]), synth.raw_capture(pair.right, rig["right"])]
    gcams, ocams = _cams(ref, rig)
    srcs = [torch.from_numpy(r).cuda() for r in raw]
    rl, rr = bdis.rectify(srcs, gcams)
    gp = bdis.Params(levels=5, iters=12)
    disp = bdis.Bdis(gp).compute(rl, rr)
    z = bdis.depth_from_disparity(disp, rig["focal"], rig["baseline"])
    torch.cuda.synchronize()
    ol, orr = ref.rectify(ocams[0], raw[0]), ref.rectify(ocams[1], raw[1])
    od = ref.compute(ol, orr, oracle_params(ref, gp))
    assert_parity(disp.cpu().numpy(), od, "rectified pipeline disparity")
    oz = ref.depth(od, rig["focal"], rig["baseline"])
    gz = z.cpu().numpy()
    m = np.isfinite(oz) & np.isfinite(gz) & (od >= 2.0)
    rel = np.abs(gz[m] - oz[m]) / oz[m]
    assert (rel <= ABS_TOL / 2.0 + 1e-6).mean() >= 0.999


def test_geometry_argument_errors(torch_cuda):
    from paper_2106_07136_amd import bdis
    torch = torch_cuda
    lib = bdis.lib()
    img = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    cam = bdis.Camera(10.0, 10.0, 4.0, 4.0)
    bad = bdis.Camera(0.0, 10.0, 4.0, 4.0)
    with pytest.raises(bdis.BdisError) as e:
        bdis.rectify([img], [bad])
    assert e.value.status == bdis.E_INVALID_ARG and b"focal" in lib.bdis_last_error(None)
    arr = (bdis.CRectifyJob * 9)()
    assert lib.bdis_rectify(arr, 9, None) == bdis.E_INVALID_ARG
    arr1 = (bdis.CRectifyJob * 1)()
    arr1[0] = bdis.CRectifyJob(img.data_ptr(), img.data_ptr(), 8, 8, 4, 8, 8, 8, cam.to_c())
    assert lib.bdis_rectify(arr1, 1, None) == bdis.E_INVALID_ARG  # pitch < width
    d = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(bdis.BdisError):
        bdis.depth_from_disparity(d, -1.0, 5.0)
    with pytest.raises(bdis.BdisError):
        bdis.depth_from_disparity(d, 500.0, 5.0, min_disparity=-1.0)
