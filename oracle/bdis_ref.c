/*
 * bdis_ref.c -- FP64 CPU oracle for Bayesian Dense Inverse Search stereo.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
 * statement of what the GPU path computes.  It is used by the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark, and by nothing in
 * the product path.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * Method: J. Song, Q. Zhu, J. Lin, M. Ghaffari, "Bayesian dense inverse
 * searching algorithm for real-time stereo matching in minimally invasive
 * surgery" (arXiv 2106.07136).
 *   - Sec. 2.1, eq. (1): per-patch inverse-compositional Lucas-Kanade search,
 *     Hessian taken once on the left (template) patch; coarse-to-fine.
 *   - Sec. 2.1, eq. (2): the DIS inverse-residual fusion (ablation mode).
 *   - Sec. 2.2, eqs. (3)-(4): patch posterior, Boltzmann likelihood normalised
 *     over a small window of candidate disparities.
 *   - Sec. 2.3, eq. (5) and the unnumbered final equation: spatial Gaussian
 *     mask times the patch posterior as the per-pixel fusion weight.
 *   - Sec. 3, first paragraph: sigma_r = sigma_s = 4, five window samples at
 *     offsets 0.5 and 1 px, valid-pixel ratio gamma.
 *   - Sec. 3.2, second paragraph: discard non-converged patches, lower the
 *     weight of patches with invalid pixels, leave uncovered pixels unestimated.
 *
 * Readings of points the paper leaves open are stated where they are used.
 * Everything is FP64, single-threaded, plain loops, in the paper's order.
 * Sign convention of eq. (1): u is the shift with I_r(x + u) ~ I_l(x); the
 * returned disparity is d = -u (left x matches right x - d).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_MAX_LEVELS 12

/* Patch outcome codes. */
enum { REF_KEPT = 0, REF_DEGENERATE = 1, REF_DIVERGED = 2, REF_GATED = 3 };

typedef struct {
    int levels;          /* pyramid levels requested (capped by size)          */
    int patch;           /* p: square patch side                               */
    int stride;          /* st: patch grid spacing                             */
    int iters;           /* K: LK iterations per level, no early exit          */
    double sigma_r;      /* eq. (4) brightness spread                          */
    double sigma_s;      /* eq. (5) spatial spread, level pixels               */
    int window;          /* number of window samples in P' (odd)               */
    double window_step;  /* spacing of the window samples, level pixels        */
    double gamma;        /* valid-pixel ratio gate                             */
    int s_mode;          /* 0: s = window samples; 1: s = patch side           */
    int fusion;          /* 0: Bayesian (Sec. 2.3); 1: DIS eq. (2)             */
    int valid_lo;        /* pixel valid iff valid_lo <= v <= valid_hi          */
    int valid_hi;
    double eps_h;        /* degenerate patch: H <= eps_h * n                   */
    double conv_tol;     /* not converged: |last LK step| > conv_tol (<= 0: off) */
} ref_params;

typedef struct {
    /* Optional per-level taps, caller-allocated, any entry may be NULL. */
    double *pyr_l[REF_MAX_LEVELS], *pyr_r[REF_MAX_LEVELS];
    uint8_t *mask_l[REF_MAX_LEVELS], *mask_r[REF_MAX_LEVELS];
    double *u_init[REF_MAX_LEVELS];   /* per patch, row-major (ny, nx) */
    double *u_final[REF_MAX_LEVELS];  /* per patch after K iterations  */
    double *post[REF_MAX_LEVELS];     /* per patch posterior p_k       */
    int8_t *status[REF_MAX_LEVELS];   /* per patch outcome code        */
    double *field[REF_MAX_LEVELS];    /* dense U_l, level pixels       */
} ref_trace;

/* ------------------------------------------------------------------------ */
/* Sizes                                                                     */
/* ------------------------------------------------------------------------ */

/* Level sizes: each coarser level halves with rounding up. */
void ref_level_dims(int W, int H, int level, int *Wl, int *Hl)
{
    int w = W, h = H;
    for (int l = 0; l < level; l++) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
    *Wl = w;
    *Hl = h;
}

/* Levels actually used: the request, cut so the coarsest level still holds
 * a whole patch in both directions. */
int ref_num_levels(int W, int H, int patch, int requested)
{
    int n = 0;
    for (int l = 0; l < requested && l < REF_MAX_LEVELS; l++) {
        int w, h;
        ref_level_dims(W, H, l, &w, &h);
        if (w < patch || h < patch)
            break;
        n = l + 1;
    }
    return n;
}

/* Patch grid along one axis: positions j*st, the last one snapped so the
 * patch ends at the border (Sec. 1: patches are square segments on a grid). */
int ref_grid_count(int n, int patch, int stride)
{
    if (n < patch)
        return 0;
    return (n - patch + stride - 1) / stride + 1;
}

int ref_grid_pos(int j, int n, int patch, int stride)
{
    int x = j * stride;
    return x < n - patch ? x : n - patch;
}

/* ------------------------------------------------------------------------ */
/* Pyramid (Sec. 1 and Fig. 1: left and right resized to coarser scales).    */
/* Reading: binomial [1 4 6 4 1]/16 blur in x then y, reflect-101 border,    */
/* keep even indices, coarse size = ceil(fine / 2).                          */
/* ------------------------------------------------------------------------ */

static int reflect101(int i, int n)
{
    if (n == 1)
        return 0;
    while (i < 0 || i >= n) {
        if (i < 0)
            i = -i;
        if (i >= n)
            i = 2 * (n - 1) - i;
    }
    return i;
}

void ref_blur_decimate(const double *src, int W, int H, double *dst)
{
    static const double w5[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    double *tmp = (double *)malloc(sizeof(double) * (size_t)W * H);
    /* blur along x */
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            double s = 0.0;
            for (int a = -2; a <= 2; a++)
                s += w5[a + 2] * src[(size_t)y * W + reflect101(x + a, W)];
            tmp[(size_t)y * W + x] = s;
        }
    /* blur along y, then keep even rows and columns */
    int Wc = (W + 1) / 2, Hc = (H + 1) / 2;
    for (int yc = 0; yc < Hc; yc++)
        for (int xc = 0; xc < Wc; xc++) {
            int y = 2 * yc, x = 2 * xc;
            double s = 0.0;
            for (int a = -2; a <= 2; a++)
                s += w5[a + 2] * tmp[(size_t)reflect101(y + a, H) * W + x];
            dst[(size_t)yc * Wc + xc] = s;
        }
    free(tmp);
}

/* Validity (Sec. 3.2: invalid, dark and bright pixels break photometric
 * consistency).  Level 0: intensity inside [lo, hi].  Coarser levels: a pixel
 * is valid iff every existing one of its 2x2 fine children is valid. */
void ref_mask_base(const uint8_t *img, int W, int H, int pitch, int lo, int hi, uint8_t *m)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int v = img[(size_t)y * pitch + x];
            m[(size_t)y * W + x] = (uint8_t)(v >= lo && v <= hi);
        }
}

void ref_mask_down(const uint8_t *m, int W, int H, uint8_t *mc)
{
    int Wc = (W + 1) / 2, Hc = (H + 1) / 2;
    for (int yc = 0; yc < Hc; yc++)
        for (int xc = 0; xc < Wc; xc++) {
            int ok = 1;
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) {
                    int y = 2 * yc + dy, x = 2 * xc + dx;
                    if (y < H && x < W && !m[(size_t)y * W + x])
                        ok = 0;
                }
            mc[(size_t)yc * Wc + xc] = (uint8_t)ok;
        }
}

/* Template-side gradient for eq. (1): the inverse-compositional form needs
 * only the left patch's derivative along the search direction (x).
 * Reading: central difference, replicate border. */
void ref_grad_x(const double *img, int W, int H, double *g)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int xp = x + 1 < W ? x + 1 : W - 1;
            int xm = x - 1 > 0 ? x - 1 : 0;
            g[(size_t)y * W + x] = 0.5 * (img[(size_t)y * W + xp] - img[(size_t)y * W + xm]);
        }
}

/* ------------------------------------------------------------------------ */
/* Samplers                                                                  */
/* ------------------------------------------------------------------------ */

/* I_r(x + u) on one image row.  Rows are integer in a rectified pair, so the
 * bilinear sampler reduces to linear interpolation in x; the coordinate is
 * clamped to the row. */
double ref_sample_row(const double *row, int W, double X)
{
    if (W == 1)
        return row[0];
    if (X < 0.0)
        X = 0.0;
    if (X > (double)(W - 1))
        X = (double)(W - 1);
    int m = (int)floor(X);
    if (m > W - 2)
        m = W - 2;
    double f = X - (double)m;
    return (1.0 - f) * row[m] + f * row[m + 1];
}

/* Bilinear read of a coarse field at (X, Y), coordinates clamped. */
double ref_bilinear(const double *F, int W, int H, double X, double Y)
{
    if (X < 0.0) X = 0.0;
    if (X > (double)(W - 1)) X = (double)(W - 1);
    if (Y < 0.0) Y = 0.0;
    if (Y > (double)(H - 1)) Y = (double)(H - 1);
    int mx = (int)floor(X), my = (int)floor(Y);
    if (mx > W - 2) mx = W - 2;
    if (my > H - 2) my = H - 2;
    if (mx < 0) mx = 0;
    if (my < 0) my = 0;
    double fx = W > 1 ? X - mx : 0.0, fy = H > 1 ? Y - my : 0.0;
    int mx1 = W > 1 ? mx + 1 : mx, my1 = H > 1 ? my + 1 : my;
    double a = (1.0 - fx) * F[(size_t)my * W + mx] + fx * F[(size_t)my * W + mx1];
    double b = (1.0 - fx) * F[(size_t)my1 * W + mx] + fx * F[(size_t)my1 * W + mx1];
    return (1.0 - fy) * a + fy * b;
}

/* ------------------------------------------------------------------------ */
/* One patch: eq. (1) then eqs. (3)-(4) and the gates.                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    double u0, u, H, post, valid_ratio;
    int n, status;
} ref_patch_out;

/* Mean-normalised residual energy of the patch at shift u:
 * E(u) = sum over left-valid pixels of (d_j - mean d)^2, d_j = I_r(x_j+u) - I_l(x_j).
 * The same residual drives the LK update (eq. (1)) and the likelihood (eq. (4)). */
double ref_patch_energy(const double *L, const double *R, const uint8_t *ML, int W, int H,
                        int x0, int y0, int p, double u)
{
    (void)H;
    double sum = 0.0;
    int n = 0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (!ML[i])
                continue;
            sum += ref_sample_row(R + (size_t)(y0 + r) * W, W, x0 + c + u) - L[i];
            n++;
        }
    if (n == 0)
        return 0.0;
    double mean = sum / n, E = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (!ML[i])
                continue;
            double d = ref_sample_row(R + (size_t)(y0 + r) * W, W, x0 + c + u) - L[i] - mean;
            E += d * d;
        }
    return E;
}

/* Posterior of the converged disparity, eqs. (3)-(4): Boltzmann likelihood of
 * each window sample, normalised over the window P' (the ratio r is the same
 * for every patch and cancels in the normalised fusion).  Written with the
 * centre energy factored out, p = 1 / sum_i exp(-(E_i - E_c)/tau), which is
 * the same number without underflow. */
double ref_posterior(const double *E, int n, int centre, double tau)
{
    double s = 0.0;
    for (int i = 0; i < n; i++)
        s += exp(-(E[i] - E[centre]) / tau);
    return 1.0 / s;
}

/* Inverse-compositional LK on one patch (Sec. 2.1, eq. (1)).  The update is
 * taken on the template (left) side, so its Jacobian and Hessian come from
 * the left patch once: J_j = g_j - mean g (the mean-normalised template
 * gradient), H = sum J_j^2.  Each iteration samples the right image at the
 * current shift, forms the mean-normalised residual e_j and moves
 * u <- u - (sum J_j e_j) / H.  Only left-valid pixels enter the sums. */
int ref_patch_lk(const double *L, const double *R, const double *G, const uint8_t *ML,
                 int W, int H, int x0, int y0, int p, int iters, double u0, double eps_h,
                 double *u_out, double *H_out, int *n_out, double *step_hist)
{
    (void)H;
    int n = 0;
    double gsum = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (ML[i]) {
                gsum += G[i];
                n++;
            }
        }
    *n_out = n;
    *u_out = u0;
    *H_out = 0.0;
    if (n == 0)
        return REF_DEGENERATE;
    double gmean = gsum / n, Hs = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (ML[i]) {
                double J = G[i] - gmean;
                Hs += J * J;
            }
        }
    *H_out = Hs;
    if (!(Hs > eps_h * n))
        return REF_DEGENERATE;
    double u = u0;
    for (int t = 0; t < iters; t++) {
        double dsum = 0.0;
        for (int r = 0; r < p; r++)
            for (int c = 0; c < p; c++) {
                size_t i = (size_t)(y0 + r) * W + (x0 + c);
                if (ML[i])
                    dsum += ref_sample_row(R + (size_t)(y0 + r) * W, W, x0 + c + u) - L[i];
            }
        double dmean = dsum / n, b = 0.0;
        for (int r = 0; r < p; r++)
            for (int c = 0; c < p; c++) {
                size_t i = (size_t)(y0 + r) * W + (x0 + c);
                if (!ML[i])
                    continue;
                double e = ref_sample_row(R + (size_t)(y0 + r) * W, W, x0 + c + u) - L[i] - dmean;
                b += (G[i] - gmean) * e;
            }
        if (step_hist)
            step_hist[t] = b / Hs;
        u = u - b / Hs;
    }
    *u_out = u;
    return REF_KEPT;
}

/* Fraction of the patch that gives usable evidence at shift u: left pixel
 * valid, its right sample inside the row, and both right taps valid
 * (Sec. 3 gamma; Sec. 3.2 invalid pixels lower a patch's weight). */
double ref_valid_ratio(const uint8_t *ML, const uint8_t *MR, int W, int x0, int y0, int p, double u)
{
    int cnt = 0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            double X = x0 + c + u;
            if (!ML[i] || X < 0.0 || X > (double)(W - 1))
                continue;
            int m = (int)floor(X);
            if (W > 1 && m > W - 2)
                m = W - 2;
            int m1 = W > 1 ? m + 1 : m;
            size_t rr = (size_t)(y0 + r) * W;
            if (MR[rr + m] && MR[rr + m1])
                cnt++;
        }
    return (double)cnt / ((double)p * p);
}

/* Whole per-patch pipeline at one level. */
static void ref_patch(const ref_params *P, const double *L, const double *R, const double *G,
                      const uint8_t *ML, const uint8_t *MR, int W, int H, int x0, int y0,
                      double u0, ref_patch_out *o)
{
    int p = P->patch;
    o->u0 = u0;
    o->post = 0.0;
    o->valid_ratio = 0.0;
    double steps[1024];
    o->status = ref_patch_lk(L, R, G, ML, W, H, x0, y0, p, P->iters, u0, P->eps_h,
                             &o->u, &o->H, &o->n, steps);
    if (o->status != REF_KEPT)
        return;
    if (P->fusion == 1) { /* DIS eq. (2): no window, no gate, no discard */
        if (!isfinite(o->u))
            o->status = REF_DIVERGED;
        else
            o->post = 1.0;
        return;
    }
    /* Sec. 3.2: the patch that does not converge is discarded.  Reading:
     * a non-finite shift, or one that left the initial estimate by more
     * than a patch side. */
    if (!isfinite(o->u) || fabs(o->u - u0) > (double)p ||
        (P->conv_tol > 0 && P->iters > 0 && !(fabs(steps[P->iters - 1]) <= P->conv_tol))) {
        o->status = REF_DIVERGED;
        return;
    }
    /* eqs. (3)-(4) over the window P' = {u + (i - c) * step}. */
    double E[64];
    int nw = P->window, c = (P->window - 1) / 2;
    for (int i = 0; i < nw; i++)
        E[i] = ref_patch_energy(L, R, ML, W, H, x0, y0, p, o->u + (i - c) * P->window_step);
    double s = P->s_mode == 0 ? (double)P->window : (double)p;
    double tau = 2.0 * P->sigma_r * P->sigma_r * s * s;
    o->post = ref_posterior(E, nw, c, tau);
    o->valid_ratio = ref_valid_ratio(ML, MR, W, x0, y0, p, o->u);
    if (o->valid_ratio < P->gamma) {
        o->status = REF_GATED;
        o->post = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Densification (Sec. 2.3): written as a scatter over patches.              */
/* ------------------------------------------------------------------------ */

/* Spatial Gaussian mask of eq. (5): weight of pixel (r, c) of a patch is
 * exp(-|x - centre|^2 / (2 sigma_s^2)); it depends on the offset inside the
 * patch only, so it is the same for every patch. */
double ref_spatial_weight(int r, int c, int p, double sigma_s)
{
    double cy = (p - 1) * 0.5, cx = (p - 1) * 0.5;
    double d2 = (r - cy) * (r - cy) + (c - cx) * (c - cx);
    return exp(-d2 / (2.0 * sigma_s * sigma_s));
}

/* Per-pixel posterior-weighted mean over the kept covering patches
 * (final equation of Sec. 2.3 used as weights).  acc_w and acc_wu are
 * caller buffers of W*H.  In DIS mode the weight is eq. (2)'s inverse
 * residual 1/max((I_r(x+u_k) - I_l(x))^2, 1). */
void ref_densify(const ref_params *P, int W, int H, int nx, int ny, const double *u,
                 const double *post, const int8_t *status, const double *L, const double *R,
                 double *acc_w, double *acc_wu)
{
    int p = P->patch;
    for (size_t i = 0; i < (size_t)W * H; i++) {
        acc_w[i] = 0.0;
        acc_wu[i] = 0.0;
    }
    for (int jy = 0; jy < ny; jy++)
        for (int jx = 0; jx < nx; jx++) {
            int k = jy * nx + jx;
            if (status[k] != REF_KEPT)
                continue;
            int x0 = ref_grid_pos(jx, W, p, P->stride), y0 = ref_grid_pos(jy, H, p, P->stride);
            for (int r = 0; r < p; r++)
                for (int c = 0; c < p; c++) {
                    size_t i = (size_t)(y0 + r) * W + (x0 + c);
                    double w;
                    if (P->fusion == 1) {
                        double res = ref_sample_row(R + (size_t)(y0 + r) * W, W, x0 + c + u[k]) - L[i];
                        double q = res * res;
                        w = 1.0 / (q > 1.0 ? q : 1.0);
                    } else {
                        w = post[k] * ref_spatial_weight(r, c, p, P->sigma_s);
                    }
                    acc_w[i] += w;
                    acc_wu[i] += w * u[k];
                }
        }
}

/* ------------------------------------------------------------------------ */
/* Whole pair, coarse to fine (Sec. 2.1, Fig. 1).                            */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Learned initial field (an added serving pattern, not in the paper).       */
/* A proposal network gives, on a coarse pyramid level, a disparity d (in    */
/* that level's pixels) and a confidence logit per pixel.  Read at a finer   */
/* "injection" level that is `scale` times larger, pixel (x, y) takes the    */
/* network values bilinearly at (x / scale, y / scale) (the sampler of        */
/* ref_bilinear, coordinates clamped); the confidence is the logistic        */
/* function of the logit, taken at the four taps before the interpolation.   */
/* The proposal is the shift u = -scale * d (eq. (1)'s sign: d = -u), kept   */
/* where the confidence is at least thr.                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *net;   /* H4 x W4 x 2, row-major: (disparity, confidence logit) */
    int W4, H4;          /* size of the network level                           */
    int scale;           /* network level -> injection level size ratio (2^k)   */
    int level;           /* injection level (>= 1)                              */
    double thr;          /* confidence gate                                     */
    int fine_iters;      /* LK iterations of the levels below the injection level */
    double *field_out;   /* optional: merged field at the injection level       */
    uint8_t *keep_out;   /* optional: 1 where the proposal is kept              */
} ref_learned;

void ref_gate(const double *net, int W4, int H4, int Wi, int Hi, int scale, double thr,
              double *U, uint8_t *keep)
{
    double *d = (double *)malloc(sizeof(double) * (size_t)W4 * H4);
    double *c = (double *)malloc(sizeof(double) * (size_t)W4 * H4);
    if (!d || !c) {
        free(d);
        free(c);
        return;
    }
    for (size_t i = 0; i < (size_t)W4 * H4; i++) {
        d[i] = net[2 * i];
        c[i] = 1.0 / (1.0 + exp(-net[2 * i + 1]));
    }
    for (int y = 0; y < Hi; y++)
        for (int x = 0; x < Wi; x++) {
            double X = (double)x / scale, Y = (double)y / scale;
            size_t i = (size_t)y * Wi + x;
            U[i] = -(double)scale * ref_bilinear(d, W4, H4, X, Y);
            keep[i] = (uint8_t)(ref_bilinear(c, W4, H4, X, Y) >= thr);
        }
    free(d);
    free(c);
}

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * disp: W*H doubles, row-major, d = -U_0, NaN where no patch covered the
 * pixel (Sec. 3.2: such pixels are not estimated). */
static int ref_compute_impl(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W,
                            int H, int pitch, double *disp, ref_trace *trace, int init_level,
                            const double *U_init, int init_iters, const ref_learned *lrn);

int ref_compute(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W, int H,
                int pitch, double *disp, ref_trace *trace)
{
    return ref_compute_impl(P, Limg, Rimg, W, H, pitch, disp, trace, -1, NULL, 0, NULL);
}

/* Learned-init pipeline with the network output as an input.  The plain
 * method runs from the coarsest level down to the injection level (it is
 * the fallback); there its dense field is replaced by the proposal wherever
 * the gate keeps it (ref_gate), and the finer levels start from that merged
 * field with fine_iters LK iterations.  net: the network output on level
 * net_level (H4 x W4 x 2, the sizes of that level).  field_out (merged
 * field, injection-level size) and keep_out may be NULL. */
int ref_compute_learned(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W,
                        int H, int pitch, const double *net, int net_level, int inj_level,
                        double thr, int fine_iters, double *disp, double *field_out,
                        uint8_t *keep_out)
{
    if (!net || inj_level < 1 || net_level <= inj_level || net_level >= 30 || fine_iters < 0 ||
        fine_iters > 1000)
        return -1;
    ref_learned g;
    g.net = net;
    ref_level_dims(W, H, net_level, &g.W4, &g.H4);
    g.scale = 1 << (net_level - inj_level);
    g.level = inj_level;
    g.thr = thr;
    g.fine_iters = fine_iters;
    g.field_out = field_out;
    g.keep_out = keep_out;
    return ref_compute_impl(P, Limg, Rimg, W, H, pitch, disp, NULL, -1, NULL, 0, &g);
}

/* The fine levels only, from a given initial field: U_init is the dense
 * field of level init_level (level pixels, row-major, that level's size);
 * levels init_level-1 .. 0 run as in ref_compute with init_iters LK
 * iterations.  This is the learned-init pipeline with the proposal taken as
 * an input. */
int ref_compute_init(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W, int H,
                     int pitch, int init_level, const double *U_init, int init_iters, double *disp)
{
    if (!U_init || init_level < 1 || init_iters < 0 || init_iters > 1000)
        return -1;
    return ref_compute_impl(P, Limg, Rimg, W, H, pitch, disp, NULL, init_level, U_init, init_iters, NULL);
}

static int ref_compute_impl(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W,
                            int H, int pitch, double *disp, ref_trace *trace, int init_level,
                            const double *U_init, int init_iters, const ref_learned *lrn)
{
    if (!P || !Limg || !Rimg || !disp || W < 1 || H < 1 || pitch < W || P->patch < 1 ||
        P->stride < 1 || P->iters < 0 || P->iters > 1000 || P->window < 1 || (P->window % 2) == 0 ||
        P->window > 63 || W < P->patch || H < P->patch)
        return -1;
    int NL = ref_num_levels(W, H, P->patch, P->levels);
    if (NL < 1 || (init_level >= 0 && init_level >= NL) || (lrn && lrn->level >= NL))
        return -1;

    double *pl[REF_MAX_LEVELS], *pr[REF_MAX_LEVELS], *gl[REF_MAX_LEVELS], *U[REF_MAX_LEVELS];
    uint8_t *ml[REF_MAX_LEVELS], *mr[REF_MAX_LEVELS];
    int Ws[REF_MAX_LEVELS], Hs[REF_MAX_LEVELS];
    memset(pl, 0, sizeof pl); memset(pr, 0, sizeof pr); memset(gl, 0, sizeof gl);
    memset(U, 0, sizeof U); memset(ml, 0, sizeof ml); memset(mr, 0, sizeof mr);
    int rc = 0;
    double *aw = NULL, *awu = NULL;

    for (int l = 0; l < NL; l++) {
        ref_level_dims(W, H, l, &Ws[l], &Hs[l]);
        size_t n = (size_t)Ws[l] * Hs[l];
        pl[l] = (double *)malloc(n * sizeof(double));
        pr[l] = (double *)malloc(n * sizeof(double));
        gl[l] = (double *)malloc(n * sizeof(double));
        U[l] = (double *)malloc(n * sizeof(double));
        ml[l] = (uint8_t *)malloc(n);
        mr[l] = (uint8_t *)malloc(n);
        if (!pl[l] || !pr[l] || !gl[l] || !U[l] || !ml[l] || !mr[l]) {
            rc = -2;
            goto done;
        }
    }
    aw = (double *)malloc((size_t)W * H * sizeof(double));
    awu = (double *)malloc((size_t)W * H * sizeof(double));
    if (!aw || !awu) {
        rc = -2;
        goto done;
    }

    /* Intensities stay in gray levels 0..255: sigma_r is in those units. */
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            pl[0][(size_t)y * W + x] = Limg[(size_t)y * pitch + x];
            pr[0][(size_t)y * W + x] = Rimg[(size_t)y * pitch + x];
        }
    ref_mask_base(Limg, W, H, pitch, P->valid_lo, P->valid_hi, ml[0]);
    ref_mask_base(Rimg, W, H, pitch, P->valid_lo, P->valid_hi, mr[0]);
    for (int l = 1; l < NL; l++) {
        ref_blur_decimate(pl[l - 1], Ws[l - 1], Hs[l - 1], pl[l]);
        ref_blur_decimate(pr[l - 1], Ws[l - 1], Hs[l - 1], pr[l]);
        ref_mask_down(ml[l - 1], Ws[l - 1], Hs[l - 1], ml[l]);
        ref_mask_down(mr[l - 1], Ws[l - 1], Hs[l - 1], mr[l]);
    }
    for (int l = 0; l < NL; l++)
        ref_grad_x(pl[l], Ws[l], Hs[l], gl[l]);

    int top = NL - 1;
    if (init_level >= 0) {
        memcpy(U[init_level], U_init, (size_t)Ws[init_level] * Hs[init_level] * sizeof(double));
        top = init_level - 1;
    }
    ref_params Pl = *P;
    if (init_level >= 0)
        Pl.iters = init_iters;
    for (int l = top; l >= 0; l--) {
        int w = Ws[l], h = Hs[l], p = P->patch;
        if (lrn && l < lrn->level)
            Pl.iters = lrn->fine_iters;
        int nx = ref_grid_count(w, p, P->stride), ny = ref_grid_count(h, p, P->stride);
        size_t np = (size_t)nx * ny;
        double *pu = (double *)malloc(np * sizeof(double));
        double *pp = (double *)malloc(np * sizeof(double));
        int8_t *ps = (int8_t *)malloc(np);
        if (!pu || !pp || !ps) {
            free(pu); free(pp); free(ps);
            rc = -2;
            goto done;
        }
        for (int jy = 0; jy < ny; jy++)
            for (int jx = 0; jx < nx; jx++) {
                int k = jy * nx + jx;
                int x0 = ref_grid_pos(jx, w, p, P->stride), y0 = ref_grid_pos(jy, h, p, P->stride);
                /* Sec. 2.1: the fine level starts from the optimised coarse
                 * field, read bilinearly at the patch centre and doubled. */
                double u0 = 0.0;
                if (l < NL - 1) {
                    double cx = x0 + 0.5 * (p - 1), cy = y0 + 0.5 * (p - 1);
                    u0 = 2.0 * ref_bilinear(U[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * cx, 0.5 * cy);
                }
                ref_patch_out o;
                ref_patch(&Pl, pl[l], pr[l], gl[l], ml[l], mr[l], w, h, x0, y0, u0, &o);
                pu[k] = o.u;
                pp[k] = o.status == REF_KEPT ? o.post : 0.0;
                ps[k] = (int8_t)o.status;
                if (trace && trace->u_init[l]) trace->u_init[l][k] = u0;
            }
        ref_densify(P, w, h, nx, ny, pu, pp, ps, pl[l], pr[l], aw, awu);
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t i = (size_t)y * w + x;
                double v;
                if (aw[i] > 0.0)
                    v = awu[i] / aw[i];
                else if (l == 0)
                    v = NAN; /* Sec. 3.2: uncovered pixels stay unestimated */
                else if (l == NL - 1)
                    v = 0.0;
                else
                    v = 2.0 * ref_bilinear(U[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * x, 0.5 * y);
                U[l][i] = v;
            }
        if (lrn && l == lrn->level) {
            /* the proposal replaces the plain field where the gate keeps it */
            double *Ug = (double *)malloc((size_t)w * h * sizeof(double));
            uint8_t *keep = (uint8_t *)malloc((size_t)w * h);
            if (!Ug || !keep) {
                free(Ug); free(keep); free(pu); free(pp); free(ps);
                rc = -2;
                goto done;
            }
            ref_gate(lrn->net, lrn->W4, lrn->H4, w, h, lrn->scale, lrn->thr, Ug, keep);
            for (size_t i = 0; i < (size_t)w * h; i++)
                if (keep[i])
                    U[l][i] = Ug[i];
            if (lrn->field_out) memcpy(lrn->field_out, U[l], (size_t)w * h * sizeof(double));
            if (lrn->keep_out) memcpy(lrn->keep_out, keep, (size_t)w * h);
            free(Ug);
            free(keep);
        }
        if (trace) {
            if (trace->u_final[l]) memcpy(trace->u_final[l], pu, np * sizeof(double));
            if (trace->post[l]) memcpy(trace->post[l], pp, np * sizeof(double));
            if (trace->status[l]) memcpy(trace->status[l], ps, np);
        }
        free(pu); free(pp); free(ps);
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            disp[(size_t)y * W + x] = -U[0][(size_t)y * W + x];
    if (trace)
        for (int l = 0; l < NL; l++) {
            size_t n = (size_t)Ws[l] * Hs[l];
            if (trace->pyr_l[l]) memcpy(trace->pyr_l[l], pl[l], n * sizeof(double));
            if (trace->pyr_r[l]) memcpy(trace->pyr_r[l], pr[l], n * sizeof(double));
            if (trace->mask_l[l]) memcpy(trace->mask_l[l], ml[l], n);
            if (trace->mask_r[l]) memcpy(trace->mask_r[l], mr[l], n);
            if (trace->field[l]) memcpy(trace->field[l], U[l], n * sizeof(double));
        }
done:
    for (int l = 0; l < NL; l++) {
        free(pl[l]); free(pr[l]); free(gl[l]); free(U[l]); free(ml[l]); free(mr[l]);
    }
    free(aw);
    free(awu);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* The steps around the matcher (Sec. 1: stereo follows the pinhole camera  */
/* model with rectification and undistortion before disparity estimation;  */
/* Sec. 3: the data are rectified and undistorted from the calibration;    */
/* Sec. 3.2: depth errors in mm, and the invalid pixels undistortion leaves */
/* at the image edges).  Not part of the paper's algorithm: standard        */
/* pinhole geometry with the radial-tangential (Brown-Conrady) lens model.  */
/* ------------------------------------------------------------------------ */

typedef struct {
    double fx, fy, cx, cy;          /* raw camera matrix                                */
    double k1, k2, p1, p2, k3;      /* radial (k) and tangential (p) distortion          */
    double R[9];                    /* rectifying rotation, row-major: rectified = R raw */
    double nfx, nfy, ncx, ncy;      /* camera matrix of the rectified image             */
} ref_camera;

/* Where rectified pixel (u, v) comes from in the raw image.  The rectified
 * pixel's ray in the rectified frame is ((u - ncx) / nfx, (v - ncy) / nfy, 1);
 * the raw frame sees it rotated back by R^T; projected to the raw normalised
 * plane (x, y), the lens moves it to
 *   x_d = x (1 + k1 r^2 + k2 r^4 + k3 r^6) + 2 p1 x y + p2 (r^2 + 2 x^2)
 *   y_d = y (1 + k1 r^2 + k2 r^4 + k3 r^6) + p1 (r^2 + 2 y^2) + 2 p2 x y
 * with r^2 = x^2 + y^2, and the raw camera matrix maps it to pixels. */
void ref_rectify_source(const ref_camera *c, double u, double v, double *xs, double *ys)
{
    double a = (u - c->ncx) / c->nfx, b = (v - c->ncy) / c->nfy;
    /* R^T (a, b, 1): column j of R dotted with (a, b, 1) */
    double X = c->R[0] * a + c->R[3] * b + c->R[6];
    double Y = c->R[1] * a + c->R[4] * b + c->R[7];
    double Z = c->R[2] * a + c->R[5] * b + c->R[8];
    double x = X / Z, y = Y / Z;
    double r2 = x * x + y * y;
    double radial = 1.0 + c->k1 * r2 + c->k2 * r2 * r2 + c->k3 * r2 * r2 * r2;
    double xd = x * radial + 2.0 * c->p1 * x * y + c->p2 * (r2 + 2.0 * x * x);
    double yd = y * radial + c->p1 * (r2 + 2.0 * y * y) + 2.0 * c->p2 * x * y;
    *xs = c->fx * xd + c->cx;
    *ys = c->fy * yd + c->cy;
}

/* Rectified, undistorted image: each output pixel takes the raw image
 * bilinearly at its source position, rounded to the nearest gray level
 * (halves up).  A source position outside the raw image (beyond its pixel
 * centres) gives 0, below the validity band: the matcher treats those edge
 * pixels as invalid (Sec. 3.2). */
void ref_rectify(const ref_camera *c, const uint8_t *src, int sw, int sh, int spitch, uint8_t *dst,
                 int dw, int dh, int dpitch)
{
    for (int v = 0; v < dh; v++)
        for (int u = 0; u < dw; u++) {
            double xs, ys;
            ref_rectify_source(c, (double)u, (double)v, &xs, &ys);
            uint8_t out = 0;
            if (xs >= 0.0 && ys >= 0.0 && xs <= (double)(sw - 1) && ys <= (double)(sh - 1)) {
                int mx = (int)floor(xs), my = (int)floor(ys);
                if (mx > sw - 2) mx = sw - 2;
                if (my > sh - 2) my = sh - 2;
                if (mx < 0) mx = 0;
                if (my < 0) my = 0;
                double fx = sw > 1 ? xs - mx : 0.0, fy = sh > 1 ? ys - my : 0.0;
                int mx1 = sw > 1 ? mx + 1 : mx, my1 = sh > 1 ? my + 1 : my;
                double top = (1.0 - fx) * src[(size_t)my * spitch + mx] + fx * src[(size_t)my * spitch + mx1];
                double bot = (1.0 - fx) * src[(size_t)my1 * spitch + mx] + fx * src[(size_t)my1 * spitch + mx1];
                double val = (1.0 - fy) * top + fy * bot;
                double q = floor(val + 0.5);
                out = (uint8_t)(q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q));
            }
            dst[(size_t)v * dpitch + u] = out;
        }
}

/* Depth along the optical axis from disparity in a rectified pair with
 * focal length f (pixels) and baseline B: Z = f B / d, in the unit of B.
 * Unestimated (NaN) and disparities at or below d_min give NaN. */
void ref_depth(const double *disp, int W, int H, double f, double B, double d_min, double *depth)
{
    for (size_t i = 0; i < (size_t)W * H; i++) {
        double d = disp[i];
        depth[i] = (isfinite(d) && d > d_min) ? f * B / d : NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* 2-D search: the DIS patch search the method builds on (Sec. 2.1: the     */
/* inverse-compositional LK of DIS, restricted by the paper to the epipolar */
/* direction; Fig. 1) estimates a full translation (u, v) per patch, which  */
/* tolerates imperfect rectification.  Everything else is the 1-D method:   */
/* mean-normalised residuals, the window posterior along the disparity      */
/* direction at the converged v (eqs. (3)-(4)), the gates, and the spatial  */
/* Gaussian fusion (eq. (5)) applied to u and to v with the same weights.   */
/* Sign convention: I_r(x + u, y + v) ~ I_l(x, y); outputs d = -u and v.    */
/* ------------------------------------------------------------------------ */

/* Template-side gradient along y: central difference, replicate border. */
void ref_grad_y(const double *img, int W, int H, double *g)
{
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int yp = y + 1 < H ? y + 1 : H - 1;
            int ym = y - 1 > 0 ? y - 1 : 0;
            g[(size_t)y * W + x] = 0.5 * (img[(size_t)yp * W + x] - img[(size_t)ym * W + x]);
        }
}

/* Mean-normalised energy at (u, v): sum over left-valid pixels of
 * (d_j - mean d)^2, d_j = I_r(x_j + u, y_j + v) - I_l(x_j, y_j), I_r read
 * bilinearly with clamped coordinates. */
double ref_patch_energy2d(const double *L, const double *R, const uint8_t *ML, int W, int H, int x0, int y0, int p,
                          double u, double v)
{
    double sum = 0.0;
    int n = 0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (!ML[i])
                continue;
            sum += ref_bilinear(R, W, H, x0 + c + u, y0 + r + v) - L[i];
            n++;
        }
    if (n == 0)
        return 0.0;
    double mean = sum / n, E = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (!ML[i])
                continue;
            double d = ref_bilinear(R, W, H, x0 + c + u, y0 + r + v) - L[i] - mean;
            E += d * d;
        }
    return E;
}

/* Inverse-compositional LK on one patch in 2-D.  J_j = (gx_j, gy_j) - mean,
 * H = sum J J^T (2 x 2); each step solves H (du, dv) = sum J_j e_j and moves
 * (u, v) <- (u, v) - (du, dv).  Degenerate if n = 0 or the smaller
 * eigenvalue of H is at most eps_h n (no 2-D texture: the aperture problem).
 * step_hist receives max(|du|, |dv|) per iteration. */
int ref_patch_lk2d(const double *L, const double *R, const double *GX, const double *GY, const uint8_t *ML,
                   int W, int H, int x0, int y0, int p, int iters, double u0, double v0, double eps_h,
                   double *u_out, double *v_out, double *step_hist)
{
    int n = 0;
    double sx = 0.0, sy = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (ML[i]) {
                sx += GX[i];
                sy += GY[i];
                n++;
            }
        }
    *u_out = u0;
    *v_out = v0;
    if (n == 0)
        return REF_DEGENERATE;
    double mx = sx / n, my = sy / n, hxx = 0.0, hxy = 0.0, hyy = 0.0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            if (!ML[i])
                continue;
            double jx = GX[i] - mx, jy = GY[i] - my;
            hxx += jx * jx;
            hxy += jx * jy;
            hyy += jy * jy;
        }
    double tr = hxx + hyy, det = hxx * hyy - hxy * hxy;
    double disc = 0.25 * (hxx - hyy) * (hxx - hyy) + hxy * hxy;
    double lmin = 0.5 * tr - sqrt(disc);
    if (!(lmin > eps_h * n))
        return REF_DEGENERATE;
    double u = u0, v = v0;
    for (int t = 0; t < iters; t++) {
        double dsum = 0.0;
        for (int r = 0; r < p; r++)
            for (int c = 0; c < p; c++) {
                size_t i = (size_t)(y0 + r) * W + (x0 + c);
                if (ML[i])
                    dsum += ref_bilinear(R, W, H, x0 + c + u, y0 + r + v) - L[i];
            }
        double dmean = dsum / n, bx = 0.0, by = 0.0;
        for (int r = 0; r < p; r++)
            for (int c = 0; c < p; c++) {
                size_t i = (size_t)(y0 + r) * W + (x0 + c);
                if (!ML[i])
                    continue;
                double e = ref_bilinear(R, W, H, x0 + c + u, y0 + r + v) - L[i] - dmean;
                bx += (GX[i] - mx) * e;
                by += (GY[i] - my) * e;
            }
        /* (du, dv) = H^-1 (bx, by) */
        double du = (hyy * bx - hxy * by) / det, dv = (hxx * by - hxy * bx) / det;
        if (step_hist)
            step_hist[t] = fabs(du) > fabs(dv) ? fabs(du) : fabs(dv);
        u -= du;
        v -= dv;
    }
    *u_out = u;
    *v_out = v;
    return REF_KEPT;
}

/* Valid fraction at (u, v): left pixel valid, its sample inside the image,
 * and all four bilinear taps valid in the right mask. */
double ref_valid_ratio2d(const uint8_t *ML, const uint8_t *MR, int W, int H, int x0, int y0, int p, double u,
                         double v)
{
    int cnt = 0;
    for (int r = 0; r < p; r++)
        for (int c = 0; c < p; c++) {
            size_t i = (size_t)(y0 + r) * W + (x0 + c);
            double X = x0 + c + u, Y = y0 + r + v;
            if (!ML[i] || X < 0.0 || X > (double)(W - 1) || Y < 0.0 || Y > (double)(H - 1))
                continue;
            int mx = (int)floor(X), my = (int)floor(Y);
            if (W > 1 && mx > W - 2) mx = W - 2;
            if (H > 1 && my > H - 2) my = H - 2;
            int mx1 = W > 1 ? mx + 1 : mx, my1 = H > 1 ? my + 1 : my;
            if (MR[(size_t)my * W + mx] && MR[(size_t)my * W + mx1] && MR[(size_t)my1 * W + mx] &&
                MR[(size_t)my1 * W + mx1])
                cnt++;
        }
    return (double)cnt / ((double)p * p);
}

/* Whole pair with the 2-D search, coarse to fine.  disp = -U_0 and vout = V_0
 * (W*H doubles each, NaN where no kept patch covers the pixel).  The
 * posterior window is along x at the converged v.  Returns 0, -1 (bad
 * arguments) or -2 (allocation). */
int ref_compute_2d(const ref_params *P, const uint8_t *Limg, const uint8_t *Rimg, int W, int H, int pitch,
                   double *disp, double *vout)
{
    if (!P || !Limg || !Rimg || !disp || !vout || W < 1 || H < 1 || pitch < W || P->patch < 1 ||
        P->stride < 1 || P->iters < 0 || P->iters > 1000 || P->window < 1 || (P->window % 2) == 0 ||
        P->window > 63 || W < P->patch || H < P->patch || P->fusion != 0)
        return -1;
    int NL = ref_num_levels(W, H, P->patch, P->levels);
    if (NL < 1)
        return -1;
    double *pl[REF_MAX_LEVELS], *pr[REF_MAX_LEVELS], *gx[REF_MAX_LEVELS], *gy[REF_MAX_LEVELS];
    double *U[REF_MAX_LEVELS], *V[REF_MAX_LEVELS];
    uint8_t *ml[REF_MAX_LEVELS], *mr[REF_MAX_LEVELS];
    int Ws[REF_MAX_LEVELS], Hs[REF_MAX_LEVELS];
    memset(pl, 0, sizeof pl); memset(pr, 0, sizeof pr); memset(gx, 0, sizeof gx); memset(gy, 0, sizeof gy);
    memset(U, 0, sizeof U); memset(V, 0, sizeof V); memset(ml, 0, sizeof ml); memset(mr, 0, sizeof mr);
    int rc = 0;
    double *aw = NULL, *awu = NULL, *awv = NULL;
    for (int l = 0; l < NL; l++) {
        ref_level_dims(W, H, l, &Ws[l], &Hs[l]);
        size_t n = (size_t)Ws[l] * Hs[l];
        pl[l] = (double *)malloc(n * sizeof(double));
        pr[l] = (double *)malloc(n * sizeof(double));
        gx[l] = (double *)malloc(n * sizeof(double));
        gy[l] = (double *)malloc(n * sizeof(double));
        U[l] = (double *)malloc(n * sizeof(double));
        V[l] = (double *)malloc(n * sizeof(double));
        ml[l] = (uint8_t *)malloc(n);
        mr[l] = (uint8_t *)malloc(n);
        if (!pl[l] || !pr[l] || !gx[l] || !gy[l] || !U[l] || !V[l] || !ml[l] || !mr[l]) {
            rc = -2;
            goto done2;
        }
    }
    aw = (double *)malloc((size_t)W * H * sizeof(double));
    awu = (double *)malloc((size_t)W * H * sizeof(double));
    awv = (double *)malloc((size_t)W * H * sizeof(double));
    if (!aw || !awu || !awv) {
        rc = -2;
        goto done2;
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            pl[0][(size_t)y * W + x] = Limg[(size_t)y * pitch + x];
            pr[0][(size_t)y * W + x] = Rimg[(size_t)y * pitch + x];
        }
    ref_mask_base(Limg, W, H, pitch, P->valid_lo, P->valid_hi, ml[0]);
    ref_mask_base(Rimg, W, H, pitch, P->valid_lo, P->valid_hi, mr[0]);
    for (int l = 1; l < NL; l++) {
        ref_blur_decimate(pl[l - 1], Ws[l - 1], Hs[l - 1], pl[l]);
        ref_blur_decimate(pr[l - 1], Ws[l - 1], Hs[l - 1], pr[l]);
        ref_mask_down(ml[l - 1], Ws[l - 1], Hs[l - 1], ml[l]);
        ref_mask_down(mr[l - 1], Ws[l - 1], Hs[l - 1], mr[l]);
    }
    for (int l = 0; l < NL; l++) {
        ref_grad_x(pl[l], Ws[l], Hs[l], gx[l]);
        ref_grad_y(pl[l], Ws[l], Hs[l], gy[l]);
    }
    for (int l = NL - 1; l >= 0; l--) {
        int w = Ws[l], h = Hs[l], p = P->patch;
        int nx = ref_grid_count(w, p, P->stride), ny = ref_grid_count(h, p, P->stride);
        size_t np = (size_t)nx * ny;
        double *pu = (double *)malloc(np * sizeof(double));
        double *pv = (double *)malloc(np * sizeof(double));
        double *pp = (double *)malloc(np * sizeof(double));
        int8_t *ps = (int8_t *)malloc(np);
        double steps[1024];
        if (!pu || !pv || !pp || !ps) {
            free(pu); free(pv); free(pp); free(ps);
            rc = -2;
            goto done2;
        }
        for (int jy = 0; jy < ny; jy++)
            for (int jx = 0; jx < nx; jx++) {
                int k = jy * nx + jx;
                int x0 = ref_grid_pos(jx, w, p, P->stride), y0 = ref_grid_pos(jy, h, p, P->stride);
                double u0 = 0.0, v0 = 0.0;
                if (l < NL - 1) {
                    double cx = x0 + 0.5 * (p - 1), cy = y0 + 0.5 * (p - 1);
                    u0 = 2.0 * ref_bilinear(U[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * cx, 0.5 * cy);
                    v0 = 2.0 * ref_bilinear(V[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * cx, 0.5 * cy);
                }
                double u, v, post = 0.0;
                int st = ref_patch_lk2d(pl[l], pr[l], gx[l], gy[l], ml[l], w, h, x0, y0, p, P->iters, u0, v0,
                                        P->eps_h, &u, &v, steps);
                if (st == REF_KEPT) {
                    if (!isfinite(u) || !isfinite(v) || fabs(u - u0) > (double)p || fabs(v - v0) > (double)p ||
                        (P->conv_tol > 0 && P->iters > 0 && !(steps[P->iters - 1] <= P->conv_tol))) {
                        st = REF_DIVERGED;
                    } else {
                        double E[64];
                        int nw = P->window, cw = (P->window - 1) / 2;
                        for (int i = 0; i < nw; i++)
                            E[i] = ref_patch_energy2d(pl[l], pr[l], ml[l], w, h, x0, y0, p,
                                                      u + (i - cw) * P->window_step, v);
                        double s = P->s_mode == 0 ? (double)P->window : (double)p;
                        post = ref_posterior(E, nw, cw, 2.0 * P->sigma_r * P->sigma_r * s * s);
                        if (ref_valid_ratio2d(ml[l], mr[l], w, h, x0, y0, p, u, v) < P->gamma) {
                            st = REF_GATED;
                            post = 0.0;
                        }
                    }
                }
                pu[k] = u;
                pv[k] = v;
                pp[k] = st == REF_KEPT ? post : 0.0;
                ps[k] = (int8_t)st;
            }
        /* eq. (5) fusion of u, then of v, with the same weights */
        ref_densify(P, w, h, nx, ny, pu, pp, ps, pl[l], pr[l], aw, awu);
        ref_densify(P, w, h, nx, ny, pv, pp, ps, pl[l], pr[l], aw, awv);
        for (int y = 0; y < h; y++)
            for (int x = 0; x < w; x++) {
                size_t i = (size_t)y * w + x;
                double a, b;
                if (aw[i] > 0.0) {
                    a = awu[i] / aw[i];
                    b = awv[i] / aw[i];
                } else if (l == 0) {
                    a = b = NAN;
                } else if (l == NL - 1) {
                    a = b = 0.0;
                } else {
                    a = 2.0 * ref_bilinear(U[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * x, 0.5 * y);
                    b = 2.0 * ref_bilinear(V[l + 1], Ws[l + 1], Hs[l + 1], 0.5 * x, 0.5 * y);
                }
                U[l][i] = a;
                V[l][i] = b;
            }
        free(pu); free(pv); free(pp); free(ps);
    }
    for (size_t i = 0; i < (size_t)W * H; i++) {
        disp[i] = -U[0][i];
        vout[i] = V[0][i];
    }
done2:
    for (int l = 0; l < NL; l++) {
        free(pl[l]); free(pr[l]); free(gx[l]); free(gy[l]); free(U[l]); free(V[l]); free(ml[l]); free(mr[l]);
    }
    free(aw); free(awu); free(awv);
    return rc;
}
