// bdis_lkwave.hpp -- the LK search and window posterior (Sec. 2.1, eqs.
// (3)-(4), the gates of Sec. 3 and 3.2) with one wave per patch and one lane
// per patch pixel, for the small launches of the coarse levels.  There a
// block of the row kernel (one lane per patch row) is a long chain of
// dependent steps at one wave per SIMD; here every per-pixel step runs in
// parallel and only the patch sums are chains (lane swizzles).
//
// The results are the row kernel's, bit for bit: every patch sum takes the
// fixed order of row_sum8 / row_dot8 over a row's eight column slots, then
// the row kernel's segment order over the rows.  Lane 8 r + c holds column
// slot c of row r (patch sides up to 8; slots past the side hold zeros):
//   - DPP xor 1, xor 2 and the half-row mirror add the column slots in
//     row_sum8's order; a product sum first fuses each even slot's product
//     with its odd neighbour's, rounded, then copies that pair sum to the odd
//     lane, as row_dot8 does;
//   - the row mirror then adds rows (0, 1), and the four row-pair sums (one
//     per row of 16 lanes) are added as ((3 + 2) + (1 + 0)) by two DPP row
//     broadcasts: the row kernel's xor 1 / xor 2 / half-mirror order over its
//     eight row lanes, each add's operands swapped (the same bits).
// The right image is read from global memory (through L1) rather than
// staged in LDS: the same values as the row kernel's staged copy, and at
// these launch sizes staging measured no faster.
#pragma once
#include "bdis_kernels.hpp"

namespace bdis {

constexpr int kLkwPatchesPerBlock = kBlock / 64;

__host__ __device__ constexpr int lkw_blocks(int nx, int ny) {
    return (nx * ny + kLkwPatchesPerBlock - 1) / kLkwPatchesPerBlock;
}

constexpr int kDppEvenToOdd = 0xA0;  // quad_perm [0, 0, 2, 2]

__device__ __forceinline__ double lkw_lane(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ float lkw_lane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Row broadcasts across the rows of 16 lanes (rows not in ROWS keep 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

// Sums over the patch of N values whose column pairs are already formed
// (each lane of a pair holding the pair's sum): pairs of pairs, halves, row
// pairs, then the four row-pair sums s0..s3 (one per row of 16 lanes) as
// (s3 + s2) + (s1 + s0): row 1 adds row 0's and row 3 adds row 2's (row
// broadcast of lane 15), row 3 then adds row 1's (row broadcast of lane 31),
// and lane 63's total is read.  Every lane receives the total.  All 64 lanes
// must be active.
template <int N, typename T>
__device__ __forceinline__ void lkw_tail_n(T *v) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppXor2>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppHalfMirror>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppMirror>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_bcast<kDppRowBcast15, 0xA>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_bcast<kDppRowBcast31, 0xC>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] = lkw_lane(v[i], 63);
}
// row_sum8 per row, then over the rows
template <int N, typename T>
__device__ __forceinline__ void lkw_sum_n(T *v) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppXor1>(v[i]);
    lkw_tail_n<N>(v);
}
// row_dot8 per row, then over the rows: out[i] = sum a[i] b[i]
template <int N, typename T>
__device__ __forceinline__ void lkw_dot_n(const T *a, const T *b, T *out) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < N; i++) out[i] = fma(a[i], b[i], dpp_v<kDppXor1>(a[i] * b[i]));
#pragma unroll
    for (int i = 0; i < N; i++) out[i] = dpp_v<kDppEvenToOdd>(out[i]);
    lkw_tail_n<N>(out);
}
__device__ __forceinline__ int lkw_sum_i(int v) {
    v = seg_sum_i<16>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

// One patch per wave of an LK job (the row kernel's LkJob, same records).
// With J.rec_u1 set the launch also densifies level + 1 (its share of that
// field, and the four bilinear taps of each patch centre), as the row
// kernel's small builds do.  WN >= kp.window bounds the window samples.
template <typename T, int P, bool U8, int WN>
__global__ __launch_bounds__(kBlock) void k_lkw(const JobPack<LkJob> pk, KParams kp) {
#pragma clang fp contract(off)
    static_assert(P <= 8, "one lane per pixel of an 8 x 8 slot grid");
    const int bid = (int)blockIdx.x;
    const LkJob &J = pk.j[find_job(pk, bid)];
    const int lb = bid - J.block0;
    const int W = J.W;
    const int lane = (int)threadIdx.x & 63;
    const int npatch = J.nx * J.ny;
    const int kraw = lb * kLkwPatchesPerBlock + (int)threadIdx.x / 64;
    const bool live = kraw < npatch;  // uniform per wave
    const int k = live ? kraw : npatch - 1;
    const int jy = k / J.nx, jx = k - jy * J.nx;
    const int x0 = grid_pos(jx, W, P, J.stride), y0 = grid_pos(jy, J.H, P, J.stride);
    const int r = lane >> 3, c = lane & 7;
    const bool on = r < P && c < P;
    const int x = x0 + (on ? c : 0), y = y0 + (on ? r : 0);
    const size_t row0 = (size_t)y * J.pitch;
    // template value and central difference (replicate border), as the row
    // kernel's template read
    bool vl, vm, vp;
    const T Tv = pix<T, U8>(J.L, row0 + x, kp, vl);
    const T gm = pix<T, U8>(J.L, row0 + max(x - 1, 0), kp, vm);
    const T gp = pix<T, U8>(J.L, row0 + min(x + 1, W - 1), kp, vp);
    const T Jg = T(0.5) * (gp - gm);
    const bool val = on && vl;

    // initial shift: twice the level + 1 field at the patch centre, that
    // field densified here when this launch densifies it
    T u0 = 0;
    if (J.Uc) {
        const T cx = (T)x0 + T(0.5) * (T)(P - 1), cy = (T)y0 + T(0.5) * (T)(P - 1);
        if (!J.rec_u1) {
            u0 = T(2) * bilinear<T>(static_cast<const T *>(J.Uc), J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy);
        } else {
            DenseView D;
            D.L = D.R = nullptr;
            D.rec_u = J.rec_u1; D.rec_w = J.rec_w1; D.gtab = J.gtab1; D.Uc = J.U2;
            D.pitch = 0; D.W = J.Wc; D.H = J.Hc; D.patch = P; D.stride = J.stride;
            D.nx = J.Wc < P ? 0 : (J.Wc - P + J.stride - 1) / J.stride + 1;
            D.ny = J.Hc < P ? 0 : (J.Hc - P + J.stride - 1) / J.stride + 1;
            D.Wc = (J.Wc + 1) / 2; D.Hc = (J.Hc + 1) / 2;
            D.mode = J.U2 ? 0 : 1;
            int mx, my, mx1, my1;
            T fx, fy;
            bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy, mx, my, mx1, my1, fx, fy);
            const int tap = lane & 3, tx = (tap & 1) ? mx1 : mx, ty = (tap & 2) ? my1 : my;
            const T F = dense_value<T, false, 3>(D, tx, ty, kp);
            if constexpr (!U8) {
                // this block's share of the level + 1 field (the next finer
                // level's fallback reads it); no finer level reads level 1
                // of a level-0 launch
                const int n1 = J.Wc * J.Hc, nblk = lkw_blocks(J.nx, J.ny), chunk = (n1 + nblk - 1) / nblk;
                const int i1 = min(n1, (lb + 1) * chunk);
                const double inv_wc = 1.0 / (double)J.Wc;
                for (int i = lb * chunk + (int)threadIdx.x; i < i1; i += kBlock) {
                    const int yy = div_exact(i, inv_wc), xx = i - yy * J.Wc;
                    static_cast<T *>(J.Uc)[i] = dense_value<T, false, 3>(D, xx, yy, kp);
                }
            }
            const T f00 = dpp_v<0x00>(F), f01 = dpp_v<0x55>(F), f10 = dpp_v<0xAA>(F), f11 = dpp_v<0xFF>(F);
            u0 = T(2) * bilinear_mix<T>(f00, f01, f10, f11, fx, fy);
        }
    }
    if (!live) return;  // uniform per wave; no block-wide step follows

    // right value of column xc of this lane's row (clamped to the row):
    // |value| above level 0, as the row kernel's staged copy
    auto rv = [&](int xc) -> T {
        const size_t g = row0 + (size_t)min(max(xc, 0), W - 1);
        if constexpr (U8) return (T) static_cast<const uint8_t *>(J.R)[g];
        else return fabs(static_cast<const T *>(J.R)[g]);
    };
    auto ishift = [&](T v, T &uf) -> int {
        const T fl = floor(v);
        uf = v - fl;
        return min(max((int)fl, -(W + P + 2)), W + 2);
    };

    const int n = lkw_sum_i(val ? 1 : 0);
    T gs[1] = {val ? Jg : T(0)};
    lkw_sum_n<1>(gs);
    const T gmean = n > 0 ? gs[0] / (T)n : T(0);
    const T Jm = val ? Jg - gmean : T(0);
    const T Ts = on ? Tv : T(0);
    T ja[2] = {Jm, Jm}, jb[2] = {Jm, Ts}, hj[2];
    lkw_dot_n<2>(ja, jb, hj);
    const T Hs = hj[0], JT = hj[1];

    int status = ST_KEPT;
    T u = u0, post = 0;
    const T ulo = -(T)(W + P + 2), uhi = (T)(W + 2);
    if (n == 0 || !(Hs > (T)kp.eps_h * (T)n)) {
        status = ST_DEGENERATE;
    } else {
        T step = 0;
        const T invH = T(1) / Hs;
        // sum J e = SA + f SD within one cell of the shift (see the row
        // kernel); the shift is uniform, so is the cell test
        int xi_prev = INT_MIN;
        T SA = 0, SD = 0;
        for (int t = 0; t < kp.iters; t++) {
            T uf;
            const int xi0 = x0 + ishift(u, uf);
            if (xi0 != xi_prev) {
                xi_prev = xi0;
                const T va = on ? rv(xi0 + c) : T(0), vb = on ? rv(xi0 + c + 1) : T(0);
                T aa[2] = {Jm, Jm}, bb[2] = {va, vb}, ab[2];
                lkw_dot_n<2>(aa, bb, ab);
                SA = ab[0] - JT;
                SD = ab[1] - ab[0];
            }
            step = fma(uf, SD, SA) * invH;
            u = u - step;
        }
        const bool unconverged = kp.conv_tol > 0 && kp.iters > 0 && !(fabs(step) <= (T)kp.conv_tol);
        if (kp.fusion == 1) {
            if (!isfinite(u)) status = ST_DIVERGED;
            else post = 1;
        } else if (!isfinite(u) || fabs(u - u0) > (T)P || unconverged) {
            status = ST_DIVERGED;
        } else {
            // eqs. (3)-(4): E_i = sum d^2 - (sum d)^2 / n of the window
            // samples u + (i - c) step, the row kernel's arithmetic
            const int cw = (kp.window - 1) / 2;
            const T mv = val ? T(1) : T(0);
            // the gamma gate's taps at the final shift (Sec. 3, Sec. 3.2),
            // loaded here so that they arrive with the window's samples
            const T uc = fmin(fmax(u, ulo), uhi);
            const T ui = floor(uc), ufr = uc - ui;
            const int xc = x0 + (int)ui + c;
            using RawT = std::conditional_t<U8, uint8_t, T>;
            auto raw = [&](int xq) -> RawT {
                return static_cast<const RawT *>(J.R)[row0 + (size_t)min(max(xq, 0), W - 1)];
            };
            const RawT g0 = raw(xc), g1 = raw(xc + 1), e0 = raw(W - 2), e1 = raw(W - 1);
            T m[WN], q[WN], acc[2 * WN];
#pragma unroll
            for (int i = 0; i < WN; i++) {
                q[i] = 0;
                m[i] = 0;
                if (i < kp.window && on) {
                    T uf;
                    const T ud = u + (T)(i - cw) * (T)kp.window_step;
                    const int xi = x0 + ishift(ud, uf);
                    const T omf = T(1) - uf;
                    q[i] = fma(omf, rv(xi + c), uf * rv(xi + c + 1)) - Tv;
                    m[i] = mv * q[i];
                }
            }
            T sm[WN];
#pragma unroll
            for (int i = 0; i < WN; i++) sm[i] = m[i];
            lkw_sum_n<WN>(sm);
            T ee[WN];
            lkw_dot_n<WN>(m, q, ee);
#pragma unroll
            for (int i = 0; i < WN; i++) {
                acc[2 * i] = sm[i];
                acc[2 * i + 1] = ee[i];
            }
            const T ninv = T(1) / (T)n;
            auto energy = [&](int i) -> T {
                T E = T(0);
#pragma unroll
                for (int j = 0; j < WN; j++)
                    if (j == i) E = acc[2 * j + 1] - acc[2 * j] * acc[2 * j] * ninv;
                return E;
            };
            const T Ec = energy(cw);
            // the row kernel's term sum: lane r of each 8-lane group the
            // terms of samples r and r + 8, then the group's sum
            const int rr = lane & 7;
            T term = 0;
#pragma unroll
            for (int qq = 0; qq < (WN + 7) / 8; qq++) {
                const int i = rr + qq * 8;
                if (i < kp.window) term += i == cw ? T(1) : exp(-(energy(i) - Ec) * (T)kp.inv_tau);
            }
            post = T(1) / seg_sum<8>(term);
            // gamma gate at the final shift: left valid, sample inside the
            // row, both right taps valid
            auto tap_ok = [&](RawT v) -> bool {
                if constexpr (U8) return (int)v >= kp.vlo && (int)v <= kp.vhi;
                else return !signbit(v);
            };
            bool good = false;
            if (xc >= 0 && xc <= W - 2) good = tap_ok(g0) && tap_ok(g1);
            else if (ufr == T(0) && xc == W - 1) good = tap_ok(e0) && tap_ok(e1);
            const int cnt = lkw_sum_i(val && good ? 1 : 0);
            if (cnt < kp.min_valid) {
                status = ST_GATED;
                post = 0;
            }
        }
    }
    if (lane == 0) {
        static_cast<T *>(J.rec_u)[k] = u;
        static_cast<T *>(J.rec_w)[k] = status == ST_KEPT ? post : T(0);
        J.rec_st[k] = (int8_t)status;
        static_cast<T *>(J.rec_u0)[k] = u0;
    }
}

}  // namespace bdis
