"""The oracle's pins must catch plausible mistakes.  Each case below plants
one mistake in a copy of the oracle's C source (on the CPU), builds it, and
runs the pin suite against it in a subprocess: the suite has to fail."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bdis_ref.c")

MUTATIONS = {
    "update_sign": ("u = u - b / Hs;", "u = u + b / Hs;"),
    # (dropping the mean from the LK residual is not a mistake: the Jacobian
    # sums to zero, so the step is unchanged; the energy's mean is another matter)
    "no_mean_in_energy": ("- L[i] - mean;", "- L[i];"),
    "no_mean_in_jacobian": ("double J = G[i] - gmean;", "double J = G[i];"),
    "gradient_sign": ("0.5 * (img[(size_t)y * W + xp] - img[(size_t)y * W + xm])",
                      "0.5 * (img[(size_t)y * W + xm] - img[(size_t)y * W + xp])"),
    "blur_weights": ("4.0 / 16, 6.0 / 16, 4.0 / 16", "4.0 / 16, 5.0 / 16, 5.0 / 16"),
    "reflect_border": ("i = 2 * (n - 1) - i;", "i = 2 * n - 1 - i;"),
    "decimate_odd": ("int y = 2 * yc, x = 2 * xc;", "int y = 2 * yc + 1 < H ? 2 * yc + 1 : 2 * yc, x = 2 * xc;"),
    "sampler_weights": ("return (1.0 - f) * row[m] + f * row[m + 1];",
                        "return f * row[m] + (1.0 - f) * row[m + 1];"),
    "posterior_sign": ("s += exp(-(E[i] - E[centre]) / tau);", "s += exp((E[i] - E[centre]) / tau);"),
    "energy_no_square": ("E += d * d;", "E += fabs(d);"),
    "spatial_centre": ("double cy = (p - 1) * 0.5, cx = (p - 1) * 0.5;",
                       "double cy = p * 0.5, cx = p * 0.5;"),
    "fusion_drops_posterior": ("w = post[k] * ref_spatial_weight(r, c, p, P->sigma_s);",
                               "w = ref_spatial_weight(r, c, p, P->sigma_s);"),
    "init_not_doubled": ("u0 = 2.0 * ref_bilinear(", "u0 = 1.0 * ref_bilinear("),
    "init_transposed": ("0.5 * cx, 0.5 * cy);", "0.5 * cy, 0.5 * cx);"),
    "grid_no_snap": ("return x < n - patch ? x : n - patch;", "return x;"),
    "gate_ignores_right_mask": ("if (MR[rr + m] && MR[rr + m1])", "if (1)"),
    "mask_or_pool": ("if (y < H && x < W && !m[(size_t)y * W + x])\n                        ok = 0;",
                     "if (y < H && x < W && m[(size_t)y * W + x])\n                        ok = 2;"),
    "dis_weight_inverse": ("w = 1.0 / (q > 1.0 ? q : 1.0);", "w = (q > 1.0 ? q : 1.0);"),
    "uncovered_zero": ("v = NAN; /* Sec. 3.2", "v = 0.0; /* Sec. 3.2"),
    "convergence_test_off": ("(P->conv_tol > 0 && P->iters > 0 &&", "(0 && P->iters > 0 &&"),
    "divergence_bound_off": ("fabs(o->u - u0) > (double)p ||", "0 ||"),
    # learned initial field (gate and merge)
    "gate_disparity_sign": ("U[i] = -(double)scale * ref_bilinear(", "U[i] = (double)scale * ref_bilinear("),
    "gate_no_logistic": ("c[i] = 1.0 / (1.0 + exp(-net[2 * i + 1]));", "c[i] = net[2 * i + 1];"),
    "gate_transposed": ("ref_bilinear(d, W4, H4, X, Y)", "ref_bilinear(d, W4, H4, Y, X)"),
    "gate_strict_threshold": ("ref_bilinear(c, W4, H4, X, Y) >= thr", "ref_bilinear(c, W4, H4, X, Y) > thr"),
    "gate_coordinate_scale": ("double X = (double)x / scale, Y = (double)y / scale;",
                              "double X = (double)x / (2 * scale), Y = (double)y / (2 * scale);"),
    "merge_inverted": ("if (keep[i])\n                    U[l][i] = Ug[i];",
                       "if (!keep[i])\n                    U[l][i] = Ug[i];"),
    "fine_iters_ignored": ("Pl.iters = lrn->fine_iters;", "Pl.iters = P->iters;"),
    # rectification and depth
    "rotation_not_transposed": ("double X = c->R[0] * a + c->R[3] * b + c->R[6];",
                                "double X = c->R[0] * a + c->R[1] * b + c->R[2];"),
    "tangential_swapped": ("double xd = x * radial + 2.0 * c->p1 * x * y + c->p2 * (r2 + 2.0 * x * x);",
                           "double xd = x * radial + 2.0 * c->p2 * x * y + c->p1 * (r2 + 2.0 * x * x);"),
    "radial_k2_power": ("c->k2 * r2 * r2 +", "c->k2 * r2 +"),
    "tangential_no_2x2": ("c->p2 * (r2 + 2.0 * x * x)", "c->p2 * (r2 + x * x)"),
    "rectify_truncates": ("double q = floor(val + 0.5);", "double q = floor(val);"),
    "rectify_outside_kept": ("if (xs >= 0.0 && ys >= 0.0 && xs <= (double)(sw - 1) && ys <= (double)(sh - 1)) {",
                             "if (1) {"),
    "depth_inverted": ("f * B / d : NAN;", "d / (f * B) : NAN;"),
    # 2-D search
    "grad_y_sign": ("0.5 * (img[(size_t)yp * W + x] - img[(size_t)ym * W + x])",
                    "0.5 * (img[(size_t)ym * W + x] - img[(size_t)yp * W + x])"),
    "lk2d_cross_term_sign": ("double du = (hyy * bx - hxy * by) / det, dv = (hxx * by - hxy * bx) / det;",
                             "double du = (hyy * bx + hxy * by) / det, dv = (hxx * by + hxy * bx) / det;"),
    "lk2d_solve_swapped": ("double du = (hyy * bx - hxy * by) / det, dv = (hxx * by - hxy * bx) / det;",
                           "double du = (hxx * bx - hxy * by) / det, dv = (hyy * by - hxy * bx) / det;"),
    "energy2d_transposed": ("sum += ref_bilinear(R, W, H, x0 + c + u, y0 + r + v) - L[i];",
                            "sum += ref_bilinear(R, W, H, x0 + c + v, y0 + r + u) - L[i];"),
    "ratio2d_bottom_taps_ignored": ("MR[(size_t)my1 * W + mx] &&\n                MR[(size_t)my1 * W + mx1])",
                                    "1 &&\n                1)"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(mut), "-lm"])
    env = dict(os.environ, BDIS_REF_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch mutation {name}:\n{r.stdout[-2000:]}"
