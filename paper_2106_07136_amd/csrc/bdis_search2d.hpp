// bdis_search2d.hpp -- the 2-D (x, y) patch search: the DIS patch search the
// method builds on (Sec. 2.1, Fig. 1) estimates a full translation (u, v)
// per patch, which tolerates imperfect rectification; the paper restricts it
// to the epipolar direction.  Everything else is the method as in the 1-D
// kernels: mean-normalised residuals, the window posterior along the
// disparity direction at the converged v (eqs. (3)-(4)), the discard gates,
// and the spatial-Gaussian fusion (eq. (5)) of u and of v with the same
// weights.
//
// Mapping: one wave per patch, one lane per patch pixel (P * P <= 64; the
// other lanes idle).  The right image is sampled bilinearly from global
// memory (rows vary with v, so no row staging); the patch's taps are reused
// across the iterations through L1.  Per-patch sums are wave reductions:
// DPP inside each row of 16 lanes, then the four row sums combined by two
// DPP row broadcasts and read from the last lane.
#pragma once
#include "bdis_kernels.hpp"
#include "bdis_lkwave.hpp"

namespace bdis {

struct Lk2Job {
    const void *L, *R;              // this level's images (uint8 at level 0)
    void *Uc, *Vc;                  // fields of level + 1 (null at the coarsest): read for the
                                    // initial (u, v), or -- when the job densifies level + 1
                                    // itself (rec_w1 set) -- written (this launch's share)
    void *rec_u, *rec_v, *rec_w;    // per-patch records (arithmetic type)
    int8_t *rec_st;                 // per-patch outcome
    // Densification of level + 1 folded into this launch: its records, the
    // spatial weights and the fallback fields (level + 2, null when level + 1
    // is the coarsest); rec_w1 null: Uc and Vc are read as they are
    const void *rec_u1, *rec_v1, *rec_w1, *gtab1, *U2, *V2;
    int pitch, W, H, Wc, Hc, nx, ny, stride;
    int block0;
    int pad_;
};
static_assert(sizeof(Lk2Job) == 14 * 8 + 10 * 4, "Lk2Job must have no padding");

// The two fusions of one level: same weights, records and fallback fields
// of u or of v.
struct Dense2Job {
    DenseView du, dv;
    void *Uo, *Vo;         // level fields out (levels >= 1), or null
    float *out_d, *out_v;  // level 0: -U and V (out_v may be null), or null
    int out_pitch, vout_pitch;
    int block0, pad_;
};
static_assert(sizeof(DenseView) == 6 * 8 + 10 * 4, "DenseView must have no padding");
static_assert(sizeof(Dense2Job) == 2 * sizeof(DenseView) + 4 * 8 + 4 * 4, "Dense2Job must have no padding");
template <> struct PackCap<Lk2Job> { static constexpr int value = 24; };
template <> struct PackCap<Dense2Job> { static constexpr int value = 16; };

constexpr int kLk2PatchesPerBlock = kBlock / 64;

__host__ __device__ constexpr int lk2_blocks(int nx, int ny) {
    return (nx * ny + kLk2PatchesPerBlock - 1) / kLk2PatchesPerBlock;
}

// Sum over the 64 lanes of a wave, every lane receiving the same bits: DPP
// sums inside each row of 16 lanes, then the four row sums s0..s3 added as
// (s3 + s2) + (s1 + s0) by two row broadcasts, and lane 63's total read.
// All 64 lanes must be active.
__device__ __forceinline__ double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <int N, typename T>
__device__ __forceinline__ void wave_sum_n(T *v) {
    seg_sum_n<16, N>(v);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_bcast<kDppRowBcast15, 0xA>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_bcast<kDppRowBcast31, 0xC>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] = lane_value(v[i], 63);
}
__device__ __forceinline__ int wave_sum_i(int v) {
    v = seg_sum_i<16>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

// Image value (|x| above level 0) and validity at (x, y), in the row.
template <typename T, bool U8>
__device__ __forceinline__ T pix2(const void *img, int pitch, int x, int y, const KParams &kp, bool &valid) {
    return pix<T, U8>(img, (size_t)y * pitch + x, kp, valid);
}

// Bilinear read of the right image at (X, Y), coordinates clamped to the
// image (as the coarse-field reader); ok: all four taps valid.
template <typename T, bool U8>
__device__ __forceinline__ T sample2(const void *img, int pitch, int W, int H, T X, T Y, const KParams &kp,
                                     bool &ok) {
    int mx, my, mx1, my1;
    T fx, fy;
    bilinear_taps<T>(W, H, X, Y, mx, my, mx1, my1, fx, fy);
    bool v00, v01, v10, v11;
    const T f00 = pix2<T, U8>(img, pitch, mx, my, kp, v00), f01 = pix2<T, U8>(img, pitch, mx1, my, kp, v01);
    const T f10 = pix2<T, U8>(img, pitch, mx, my1, kp, v10), f11 = pix2<T, U8>(img, pitch, mx1, my1, kp, v11);
    ok = v00 && v01 && v10 && v11;
    return bilinear_mix<T>(f00, f01, f10, f11, fx, fy);
}

// FOLD compiles the densification of level + 1 in (used when J.rec_w1 is
// set; the small launches): its gathers cost registers, so the large
// launches take the build without it.
template <typename T, int P, bool U8, int WN, bool FOLD>
__global__ __launch_bounds__(kBlock) void k_lk2d(const JobPack<Lk2Job> pk, KParams kp) {
    static_assert(P * P <= 64, "one lane per patch pixel");
    const Lk2Job &J = pk.j[find_job(pk, (int)blockIdx.x)];
    const int lane = (int)threadIdx.x & 63;
    const int lb = (int)blockIdx.x - J.block0;
    const int kraw = lb * kLk2PatchesPerBlock + (int)threadIdx.x / 64;
    const bool live = kraw < J.nx * J.ny;  // uniform per wave
    const int k = live ? kraw : J.nx * J.ny - 1;
    const int jy = k / J.nx, jx = k - jy * J.nx;
    const int x0 = grid_pos(jx, J.W, P, J.stride), y0 = grid_pos(jy, J.H, P, J.stride);
    const bool on = lane < P * P;
    const int r = on ? lane / P : 0, c = on ? lane % P : 0;
    const int x = x0 + c, y = y0 + r;
    const int W = J.W, H = J.H;
    // template value, validity and the two central differences (replicate border)
    bool vl, d0, d1, d2, d3;
    const T Tv = pix2<T, U8>(J.L, J.pitch, x, y, kp, vl);
    const T gx = T(0.5) * (pix2<T, U8>(J.L, J.pitch, min(x + 1, W - 1), y, kp, d0) -
                           pix2<T, U8>(J.L, J.pitch, max(x - 1, 0), y, kp, d1));
    const T gy = T(0.5) * (pix2<T, U8>(J.L, J.pitch, x, min(y + 1, H - 1), kp, d2) -
                           pix2<T, U8>(J.L, J.pitch, x, max(y - 1, 0), kp, d3));
    const bool val = on && vl;
    // initial translation: twice the coarse fields at the patch centre,
    // those fields densified here when this launch densifies level + 1
    T u0 = 0, v0 = 0;
    if (J.Uc) {
        const T cx = (T)x0 + T(0.5) * (T)(P - 1), cy = (T)y0 + T(0.5) * (T)(P - 1);
        if (!FOLD || !J.rec_w1) {
            u0 = T(2) * bilinear<T>(static_cast<const T *>(J.Uc), J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy);
            v0 = T(2) * bilinear<T>(static_cast<const T *>(J.Vc), J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy);
        } else if constexpr (FOLD) {
            // the 1-D fold's arithmetic for both fields: the same weights,
            // the records and fallback of u or of v
            DenseView Du;
            Du.L = Du.R = nullptr;
            Du.rec_u = J.rec_u1; Du.rec_w = J.rec_w1; Du.gtab = J.gtab1; Du.Uc = J.U2;
            Du.pitch = 0; Du.W = J.Wc; Du.H = J.Hc; Du.patch = P; Du.stride = J.stride;
            Du.nx = J.Wc < P ? 0 : (J.Wc - P + J.stride - 1) / J.stride + 1;
            Du.ny = J.Hc < P ? 0 : (J.Hc - P + J.stride - 1) / J.stride + 1;
            Du.Wc = (J.Wc + 1) / 2; Du.Hc = (J.Hc + 1) / 2;
            Du.mode = J.U2 ? 0 : 1;
            DenseView Dv = Du;
            Dv.rec_u = J.rec_v1; Dv.Uc = J.V2;
            int mx, my, mx1, my1;
            T fx, fy;
            bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy, mx, my, mx1, my1, fx, fy);
            const int tap = lane & 3, tx = (tap & 1) ? mx1 : mx, ty = (tap & 2) ? my1 : my;
            const T Fu = dense_value<T, false, 3>(Du, tx, ty, kp);
            const T Fv = dense_value<T, false, 3>(Dv, tx, ty, kp);
            if constexpr (!U8) {
                // this block's share of both level + 1 fields (the next finer
                // level's fallback reads them); no finer level reads level 1
                // of a level-0 launch
                const int n1 = J.Wc * J.Hc, nblk = lk2_blocks(J.nx, J.ny), chunk = (n1 + nblk - 1) / nblk;
                const int i1 = min(n1, (lb + 1) * chunk);
                const double inv_wc = 1.0 / (double)J.Wc;
                for (int i = lb * chunk + (int)threadIdx.x; i < i1; i += kBlock) {
                    const int yy = div_exact(i, inv_wc), xx = i - yy * J.Wc;
                    static_cast<T *>(J.Uc)[i] = dense_value<T, false, 3>(Du, xx, yy, kp);
                    static_cast<T *>(J.Vc)[i] = dense_value<T, false, 3>(Dv, xx, yy, kp);
                }
            }
            u0 = T(2) * bilinear_mix<T>(dpp_v<0x00>(Fu), dpp_v<0x55>(Fu), dpp_v<0xAA>(Fu), dpp_v<0xFF>(Fu), fx, fy);
            v0 = T(2) * bilinear_mix<T>(dpp_v<0x00>(Fv), dpp_v<0x55>(Fv), dpp_v<0xAA>(Fv), dpp_v<0xFF>(Fv), fx, fy);
        }
    }
    if (!live) return;  // uniform per wave; no block-wide step follows
    const int n = wave_sum_i(val ? 1 : 0);
    T g[2] = {val ? gx : T(0), val ? gy : T(0)};
    wave_sum_n<2>(g);
    const T mx = n > 0 ? g[0] / (T)n : T(0), my = n > 0 ? g[1] / (T)n : T(0);
    const T jxv = val ? gx - mx : T(0), jyv = val ? gy - my : T(0);
    T hs[3] = {jxv * jxv, jxv * jyv, jyv * jyv};
    wave_sum_n<3>(hs);
    const T hxx = hs[0], hxy = hs[1], hyy = hs[2];
    const T det = hxx * hyy - hxy * hxy;
    const T disc = T(0.25) * (hxx - hyy) * (hxx - hyy) + hxy * hxy;
    const T lmin = T(0.5) * (hxx + hyy) - sqrt(disc);
    int status = ST_KEPT;
    T u = u0, v = v0, post = 0;
    if (n == 0 || !(lmin > (T)kp.eps_h * (T)n)) {
        status = ST_DEGENERATE;
    } else {
        T step = 0;
        const T idet = T(1) / det;
        for (int t = 0; t < kp.iters; t++) {
            bool ok;
            const T I = sample2<T, U8>(J.R, J.pitch, W, H, (T)x + u, (T)y + v, kp, ok);
            const T d = val ? I - Tv : T(0);
            // sum J d equals sum J (d - mean d): the Jacobian sums to zero
            T b[2] = {jxv * d, jyv * d};
            wave_sum_n<2>(b);
            const T du = (hyy * b[0] - hxy * b[1]) * idet, dv = (hxx * b[1] - hxy * b[0]) * idet;
            step = fmax(fabs(du), fabs(dv));
            u -= du;
            v -= dv;
        }
        const bool unconverged = kp.conv_tol > 0 && kp.iters > 0 && !(step <= (T)kp.conv_tol);
        if (!isfinite(u) || !isfinite(v) || fabs(u - u0) > (T)P || fabs(v - v0) > (T)P || unconverged) {
            status = ST_DIVERGED;
        } else {
            // window posterior along x at the converged v (two passes: the
            // mean of each sample's residuals, then the centred energies)
            const int cw = (kp.window - 1) / 2;
            T dres[WN], s[WN];
#pragma unroll
            for (int i = 0; i < WN; i++) {
                dres[i] = 0;
                if (i < kp.window) {
                    bool ok;
                    const T I = sample2<T, U8>(J.R, J.pitch, W, H, (T)x + u + (T)(i - cw) * (T)kp.window_step,
                                               (T)y + v, kp, ok);
                    dres[i] = val ? I - Tv : T(0);
                }
                s[i] = dres[i];
            }
            wave_sum_n<WN>(s);
            const T ninv = T(1) / (T)n;
#pragma unroll
            for (int i = 0; i < WN; i++) {
                const T q = val ? dres[i] - s[i] * ninv : T(0);
                s[i] = q * q;
            }
            wave_sum_n<WN>(s);
            // lane i < window evaluates the term of sample i (one exponential
            // per lane); the centre term is 1
            T Ec = s[0], Ei = s[0];
#pragma unroll
            for (int i = 1; i < WN; i++) {
                if (i == cw) Ec = s[i];
                if (i == lane) Ei = s[i];
            }
            const T e = exp(-(Ei - Ec) * (T)kp.inv_tau);
            const T term = lane < kp.window ? (lane == cw ? T(1) : e) : T(0);
            T tsum[1] = {term};
            wave_sum_n<1>(tsum);
            post = T(1) / tsum[0];
            // gamma gate: left valid, sample inside the image, four taps valid
            bool ok;
            const T X = (T)x + u, Y = (T)y + v;
            (void)sample2<T, U8>(J.R, J.pitch, W, H, X, Y, kp, ok);
            const bool inside = X >= T(0) && Y >= T(0) && X <= (T)(W - 1) && Y <= (T)(H - 1);
            const int cnt = wave_sum_i(val && inside && ok ? 1 : 0);
            if (cnt < kp.min_valid) {
                status = ST_GATED;
                post = 0;
            }
        }
    }
    if (lane == 0) {
        static_cast<T *>(J.rec_u)[k] = u;
        static_cast<T *>(J.rec_v)[k] = v;
        static_cast<T *>(J.rec_w)[k] = status == ST_KEPT ? post : T(0);
        J.rec_st[k] = (int8_t)status;
    }
}

// One pixel of both fields: the 1-D path's gather with the records of u and
// then of v (the weights are the same); level 0 writes -U and V.
template <typename T, bool U8>
__global__ __launch_bounds__(kBlock) void k_dense2d(const JobPack<Dense2Job> pk, KParams kp) {
    const int bid = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const Dense2Job &J = pk.j[find_job(pk, bid)];
    const int i = (bid - J.block0) * kBlock + (int)threadIdx.x;
    if (i >= J.du.W * J.du.H) return;
    const int y = i / J.du.W, x = i - y * J.du.W;
    const T U = dense_value<T, U8>(J.du, x, y, kp);
    const T V = dense_value<T, U8>(J.dv, x, y, kp);
    if (J.out_d) {
        J.out_d[(size_t)y * J.out_pitch + x] = (float)(-U);
        if (J.out_v) J.out_v[(size_t)y * J.vout_pitch + x] = (float)V;
    } else {
        static_cast<T *>(J.Uo)[i] = U;
        static_cast<T *>(J.Vo)[i] = V;
    }
}

}  // namespace bdis
