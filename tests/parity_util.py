"""Shared helpers for the GPU parity tests (not a test module)."""
import numpy as np

# Tolerances of the GPU path against the FP64 oracle, per output pixel:
# RMS <= 1e-3 px over pixels both sides estimate, |d_gpu - d_ref| <= 1e-2 px
# on >= 99.9 % of all pixels (a pixel one side leaves NaN and the other does
# not counts as a miss), and the NaN masks agree on >= 99.9 % of pixels.
RMS_TOL = 1e-3
ABS_TOL = 1e-2
FRAC_TOL = 0.999


def parity(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    fg, fr = np.isfinite(gpu), np.isfinite(ref)
    both = fg & fr
    err = np.abs(gpu[both] - ref[both])
    rms = float(np.sqrt(np.mean(err ** 2))) if err.size else 0.0
    ok = np.zeros(gpu.shape, bool)
    ok[both] = np.abs(gpu[both] - ref[both]) <= ABS_TOL
    ok[~fg & ~fr] = True
    return dict(agree=float((fg == fr).mean()), rms=rms, frac=float(ok.mean()),
                max=float(err.max()) if err.size else 0.0, coverage=float(fg.mean()))


def assert_parity(gpu, ref, what=""):
    m = parity(gpu, ref)
    print(f"parity {what}: {m}", flush=True)
    assert m["agree"] >= FRAC_TOL, (what, m)
    assert m["rms"] <= RMS_TOL, (what, m)
    assert m["frac"] >= FRAC_TOL, (what, m)
    return m


def oracle_params(ref, gp):
    """Oracle parameters equal to a bdis.Params (levels resolved by the caller)."""
    return ref.Params(levels=gp.levels, patch=gp.patch, stride=gp.stride, iters=gp.iters,
                      sigma_r=gp.sigma_r, sigma_s=gp.sigma_s, window=gp.window,
                      window_step=gp.window_step, gamma=gp.gamma, s_mode=gp.s_mode,
                      fusion=gp.fusion, valid_lo=gp.valid_lo, valid_hi=gp.valid_hi,
                      eps_h=float(np.float32(gp.eps_h)), conv_tol=float(np.float32(gp.conv_tol)))


def shifted_right(left, shift):
    """Right image whose pixel x is the left image's x + shift (border
    column repeated): disparity `shift` everywhere."""
    right = np.empty_like(left)
    if shift > 0:
        right[:, :-shift] = left[:, shift:]
        right[:, -shift:] = left[:, -1:]
    else:
        s = -shift
        right[:, s:] = left[:, :-s]
        right[:, :s] = left[:, :1]
    return right
