// bdis_kernels.hpp -- gfx950 kernels of the BDIS stereo hot path.
//
// Paper: J. Song et al., "Bayesian dense inverse searching algorithm for
// real-time stereo matching in minimally invasive surgery", arXiv 2106.07136.
//
// Kernels, each launched once for every pair of a call (a "job" is one pair
// at one level):
//   k_pyr2   blur + decimate two levels of the left and right pyramids
//            (Sec. 1, Fig. 1), validity carried in the sign bit (the
//            persistent kernel runs one level per task: pyr_block);
//   k_lk     per-patch inverse-compositional LK along x (Sec. 2.1, eq. (1)),
//            then the windowed posterior (Sec. 2.2, eqs. (3)-(4)) and the
//            discard gates (Sec. 3 gamma, Sec. 3.2);
//   k_dense  per-pixel gather of the covering patches with the spatial
//            Gaussian mask times the posterior as weight (Sec. 2.3, eq. (5)
//            and the final equation), or eq. (2)'s inverse residual.
//
// Arithmetic type T: double (default; matches the FP64 reference to rounding)
// or float.  Data layout: level 0 is the caller's uint8 image (pitch in
// bytes); levels >= 1 are T images of the level size whose sign bit marks
// invalid pixels (value = |x|), so one load gives intensity and validity.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>
#include <type_traits>

namespace bdis {

constexpr int kBlock = 256;

// Method constants for one launch.
struct KParams {
    int iters;           // LK iterations, no early exit
    int window;          // posterior window samples (odd)
    double window_step;  // spacing of the samples, level px
    double inv_tau;      // 1 / (2 sigma_r^2 s^2), eq. (4)
    int min_valid;       // gamma gate: kept iff valid count >= min_valid
    int fusion;          // 0 Bayesian, 1 DIS eq. (2)
    int vlo, vhi;        // level-0 validity band
    double eps_h;        // degenerate iff H <= eps_h * n
    double conv_tol;     // not converged iff |last LK step| > conv_tol (<= 0: off)
};

static_assert(sizeof(KParams) == 56, "KParams has no padding: it is compared byte for byte");

// Job descriptors have no padding bytes (pointers first, ints after, an
// explicit pad where needed): they are copied and compared byte for byte.
struct PyrJob {
    const void *src_l, *src_r;  // level l-1 (uint8 when l-1 == 0)
    void *dst_l, *dst_r;        // level l (arithmetic type), pitch = wd
    int src_pitch;              // elements
    int ws, hs;                 // level l-1 size
    int wd, hd;                 // level l size
    int ppt;                    // coarse pixels per thread (block = ppt * kBlock)
    int block0;                 // first block of this job in its launch
    int pad_;
};
static_assert(sizeof(PyrJob) == 4 * 8 + 8 * 4, "PyrJob must have no padding");

// Two pyramid levels in one launch: level l+1 ("mid") and, when has2, level
// l+2 ("dst") from level l.  Tiles are kP2X x kP2Y pixels of level l+2 (of
// the virtual level l+2 when has2 == 0); each block also writes the level-
// (l+1) pixels under its tile.
struct Pyr2Job {
    const void *src_l, *src_r;  // level l (uint8 when l == 0)
    void *mid_l, *mid_r;        // level l+1, pitch = wm
    void *dst_l, *dst_r;        // level l+2, pitch = wd (unused when has2 == 0)
    int src_pitch;              // elements
    int ws, hs;                 // level l size
    int wm, hm;                 // level l+1 size
    int wd, hd;                 // level l+2 size: ceil(wm / 2) x ceil(hm / 2)
    int has2;                   // 1: write level l+2
    int tiles_x;                // tiles per row of level l+2
    int block0;
};
static_assert(sizeof(Pyr2Job) == 6 * 8 + 10 * 4, "Pyr2Job must have no padding");

struct LkJob {
    const void *L, *R;     // this level's images
    void *Uc;              // coarse field (level + 1), pitch Wc; null at coarsest.
                           // Read for the initial shifts, or -- when the job
                           // densifies level + 1 itself (rec_u1 set) -- written
    void *rec_u, *rec_w, *rec_u0;  // per-patch records, arithmetic type
    int8_t *rec_st;        // per-patch outcome
    // Densification of level + 1 folded into this launch (Bayesian fusion):
    // its patch records, spatial weights and fallback field (level + 2, null
    // when level + 1 is the coarsest); rec_u1 null: Uc is read as it is
    const void *rec_u1, *rec_w1, *gtab1, *U2;
    int pitch;             // image pitch, elements
    int W, H;
    int Wc, Hc;
    int nx, ny, stride;
    int reach;             // staged span reaches this many columns left of a
                           // patch (the level's largest expected disparity)
    int block0;
};
static_assert(sizeof(LkJob) == 11 * 8 + 10 * 4, "LkJob must have no padding");

struct DenseJob {
    const void *L, *R;     // images (DIS fusion only)
    const void *rec_u, *rec_w;
    const void *gtab;      // patch x patch spatial weights
    const void *Uc;        // fallback source (0 < l < L-1)
    void *U;               // level field out (pitch W), or null
    float *out;            // level 0: disparity out (= -U), or null
    const uint8_t *keep;   // non-null: pixels with keep[i] != 0 are left as they are
    int pitch;
    int W, H, patch, stride, nx, ny;
    int Wc, Hc;
    int mode;              // 0: fallback to 2*Uc, 1: zero (coarsest), 2: NaN (level 0)
    int out_pitch;
    int ppt;               // pixels per thread (block = ppt * kBlock pixels)
    int block0;
    int strip;             // > 1: one strip of this many pixels of a row per thread (ppt unused)
};
static_assert(sizeof(DenseJob) == 9 * 8 + 14 * 4, "DenseJob must have no padding");

// Input of the proposal network for one pair at its level (NHWC bfloat16,
// 16 channels).
struct NetInJob {
    const void *L, *R;     // pyramid level images (arithmetic type, sign = invalid)
    uint16_t *x;           // output, W * H * 16
    int W, H;
    int block0;
    int pad_;
};
static_assert(sizeof(NetInJob) == 3 * 8 + 4 * 4, "NetInJob must have no padding");

// Learned initial field of one pair at the injection level from the network
// output at the network level.
struct GateJob {
    const float *net;      // network output (H4 x W4 x 2: disparity, confidence logit)
    void *U;               // field at the injection level (arithmetic type), Wi x Hi
    uint8_t *keep;         // 1 where the learned value is kept (confident)
    int W4, H4, Wi, Hi;
    int block0;
    float thr;             // confidence threshold
    float sxy;             // injection-level pixel -> network-level coordinate
    float sd;              // network disparity -> shift u at the injection level
};
static_assert(sizeof(GateJob) == 3 * 8 + 8 * 4, "GateJob must have no padding");

// ---------------------------------------------------------------- helpers

// Jobs of one launch, passed by value as the kernel argument (read through
// the scalar path from the kernel-argument segment: no dependent load of a
// table).  A launch carries at most PackCap<Job> jobs (kMaxJobs, or more for
// the small records of the network input and the gate, whose packs stay
// within the same kernel-argument size); larger sets are split.
constexpr int kMaxJobs = 24;
template <typename Job> struct PackCap { static constexpr int value = kMaxJobs; };
template <> struct PackCap<NetInJob> { static constexpr int value = 96; };
template <> struct PackCap<GateJob> { static constexpr int value = 70; };
template <typename Job>
struct JobPack {
    int n;
    int pad_;
    Job j[PackCap<Job>::value];
};

template <typename Job>
__device__ __forceinline__ int find_job(const JobPack<Job> &pk, int b) {
    int lo = 0, hi = pk.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pk.j[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups of a launch are dealt to the chip's eight XCDs in turn (XCD =
// block id mod 8), and each XCD has its own L2.  Renumbering the blocks so
// that every XCD gets one contiguous range of tiles keeps the rows that
// neighbouring tiles share (filter halos, the patch records a pixel gathers)
// inside one L2 instead of fetching them from HBM once per XCD.  Bijective on
// [0, n) for any n.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int bid, int n) {
    const int q = n / kXcds, r = n % kXcds, x = bid % kXcds, k = bid / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// q / n for 0 <= q < 2^31 and n >= 1, given inv = 1.0 / n (correctly
// rounded double).  (q + 0.5) / n lies at least 0.5 / n from an integer, and
// the two roundings move it by at most (q + 0.5) / n * 2^-52 < 0.5 / n, so
// truncation gives the integer quotient: four full-rate instructions instead
// of an integer division's expansion.
__device__ __forceinline__ int div_exact(int q, double inv) {
    return (int)(((double)q + 0.5) * inv);
}

// reflect101 for -n < i < 2 n - 1 (one reflection suffices), n >= 2
__device__ __forceinline__ int reflect101_near(int i, int n) {
    i = i < 0 ? -i : i;
    return i >= n ? 2 * (n - 1) - i : i;
}

__device__ __forceinline__ int reflect101(int i, int n) {
    if (n == 1) return 0;
    while (i < 0 || i >= n) {
        if (i < 0) i = -i;
        if (i >= n) i = 2 * (n - 1) - i;
    }
    return i;
}

__device__ __forceinline__ int grid_pos(int j, int n, int p, int st) {
    int x = j * st;
    return x < n - p ? x : n - p;
}

// Value and validity of one pixel.  U8: the caller's image and the level-0
// intensity band; float: sign bit = invalid.
template <typename T, bool U8>
__device__ __forceinline__ T pix(const void *img, size_t idx, const KParams &kp, bool &valid) {
    if constexpr (U8) {
        int v = static_cast<const uint8_t *>(img)[idx];
        valid = v >= kp.vlo && v <= kp.vhi;
        return static_cast<T>(v);
    } else {
        T v = static_cast<const T *>(img)[idx];
        valid = !signbit(v);
        return fabs(v);
    }
}

template <typename T, bool U8>
__device__ __forceinline__ T pixv(const void *img, size_t idx) {
    if constexpr (U8) return static_cast<T>(static_cast<const uint8_t *>(img)[idx]);
    else return fabs(static_cast<const T *>(img)[idx]);
}

// Lane swizzles inside a row of 16 lanes (DPP): swap neighbours, swap pairs,
// mirror each half-row of 8, mirror the row of 16.
constexpr int kDppXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

// (every pattern stays inside its row and all lanes are active, so no lane
// reads out of bounds: bound_ctrl only spares the copy of an old value)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_v(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_v(double v) {
    int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Sum over aligned segments of SEG (8 or 16) lanes.  Every lane of a segment
// receives the bitwise-same total: each step adds a commuting pair.  All
// lanes of a segment must be active.
template <int SEG, typename T>
__device__ __forceinline__ T seg_sum(T v) {
    v += dpp_v<kDppXor1>(v);
    v += dpp_v<kDppXor2>(v);
    v += dpp_v<kDppHalfMirror>(v);
    if constexpr (SEG == 16) v += dpp_v<kDppMirror>(v);
    return v;
}
// seg_sum on N independent values at once (the DPP chains interleave)
template <int SEG, int N, typename T>
__device__ __forceinline__ void seg_sum_n(T *v) {
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppXor1>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppXor2>(v[i]);
#pragma unroll
    for (int i = 0; i < N; i++) v[i] += dpp_v<kDppHalfMirror>(v[i]);
    if constexpr (SEG == 16) {
#pragma unroll
        for (int i = 0; i < N; i++) v[i] += dpp_v<kDppMirror>(v[i]);
    }
}

template <int SEG>
__device__ __forceinline__ int seg_sum_i(int v) {
    v += dpp_i<kDppXor1>(v);
    v += dpp_i<kDppXor2>(v);
    v += dpp_i<kDppHalfMirror>(v);
    if constexpr (SEG == 16) v += dpp_i<kDppMirror>(v);
    return v;
}

// Sums over the eight column slots of a patch row (patch sides up to 8; the
// slots past the patch side hold zeros), in one fixed order: pairs (0, 1),
// (2, 3), (4, 5), (6, 7), then pairs of pairs, then the two halves.  A sum
// of products fuses each pair into one FMA, a0 b0 + round(a1 b1).  The
// one-lane-per-pixel LK kernel forms the same sums with lane swizzles, so
// both give the same bits.
template <typename T>
__device__ __forceinline__ T row_sum8(const T (&t)[8]) {
#pragma clang fp contract(off)
    return ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
}
template <typename T>
__device__ __forceinline__ T row_dot8(const T (&a)[8], const T (&b)[8]) {
#pragma clang fp contract(off)
    T q[4];
#pragma unroll
    for (int j = 0; j < 4; j++) q[j] = fma(a[2 * j], b[2 * j], a[2 * j + 1] * b[2 * j + 1]);
    return (q[0] + q[1]) + (q[2] + q[3]);
}

// Bilinear read of a coarse field, coordinates clamped to the field.
template <typename T>
__device__ __forceinline__ void bilinear_taps(int W, int H, T X, T Y, int &mx, int &my, int &mx1, int &my1, T &fx,
                                              T &fy) {
    X = fmin(fmax(X, T(0)), (T)(W - 1));
    Y = fmin(fmax(Y, T(0)), (T)(H - 1));
    mx = (int)floor(X), my = (int)floor(Y);
    mx = min(mx, W - 2); my = min(my, H - 2);
    mx = max(mx, 0); my = max(my, 0);
    fx = W > 1 ? X - (T)mx : T(0), fy = H > 1 ? Y - (T)my : T(0);
    mx1 = W > 1 ? mx + 1 : mx, my1 = H > 1 ? my + 1 : my;
}
template <typename T>
__device__ __forceinline__ T bilinear_mix(T f00, T f01, T f10, T f11, T fx, T fy) {
    // no contraction into FMAs: the value must not depend on the caller
    // (the densify kernel and the LK launch that densifies for itself)
#pragma clang fp contract(off)
    T a = (T(1) - fx) * f00 + fx * f01;
    T b = (T(1) - fx) * f10 + fx * f11;
    return (T(1) - fy) * a + fy * b;
}
template <typename T>
__device__ __forceinline__ T bilinear(const T *F, int W, int H, T X, T Y) {
    int mx, my, mx1, my1;
    T fx, fy;
    bilinear_taps<T>(W, H, X, Y, mx, my, mx1, my1, fx, fy);
    return bilinear_mix<T>(F[(size_t)my * W + mx], F[(size_t)my * W + mx1], F[(size_t)my1 * W + mx],
                           F[(size_t)my1 * W + mx1], fx, fy);
}

// Right-image sample at column xi + uf of one row (xi integer, 0 <= uf < 1),
// the coordinate clamped to [0, W-1] as in the linear sampler of eq. (1).
// Splitting the shift into integer and fraction keeps the fraction exact.
template <typename T, bool U8>
__device__ __forceinline__ T sample_row(const void *img, size_t row0, int W, int xi, T uf) {
    if (xi < 0) return pixv<T, U8>(img, row0);
    if (xi >= W - 1) return pixv<T, U8>(img, row0 + (W - 1));
    T a = pixv<T, U8>(img, row0 + xi), b = pixv<T, U8>(img, row0 + xi + 1);
    return (T(1) - uf) * a + uf * b;
}

// ---------------------------------------------------------------- pyramid

// One coarse pixel of both images: binomial [1 4 6 4 1]/16 in x then y with
// reflect-101 borders, taken at the even fine position; valid iff all
// existing 2x2 fine children are valid.  In double precision every level up
// to the fifth is exact (dyadic sums of 8-bit values).
constexpr double kBinom5[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};

// Validity of a coarse pixel at fine position (x, y) = 2 (xc, yc): all of
// its existing 2x2 fine children are valid.
template <typename T, bool U8>
__device__ __forceinline__ bool pyr_valid(const void *src, int pitch, int ws, int hs, int x, int y,
                                          const KParams &kp) {
    bool ok = true;
#pragma unroll
    for (int dy = 0; dy < 2; dy++)
#pragma unroll
        for (int dx = 0; dx < 2; dx++) {
            int yy = y + dy, xx = x + dx;
            if (yy < hs && xx < ws) {
                bool v;
                (void)pix<T, U8>(src, (size_t)yy * pitch + xx, kp, v);
                ok = ok && v;
            }
        }
    return ok;
}

// One coarse pixel of both images: binomial [1 4 6 4 1]/16 in x then y with
// reflect-101 borders, taken at the even fine position; valid iff all
// existing 2x2 fine children are valid.  In double precision every level up
// to the fifth is exact (dyadic sums of 8-bit values).
template <typename T, bool U8>
__device__ __forceinline__ void pyr_pixel(const PyrJob &J, int i, const KParams &kp) {
    int yc = i / J.wd, xc = i - yc * J.wd;
    int x = 2 * xc, y = 2 * yc;
    int cols[5], rows[5];
#pragma unroll
    for (int a = 0; a < 5; a++) {
        cols[a] = reflect101(x + a - 2, J.ws);
        rows[a] = reflect101(y + a - 2, J.hs);
    }
#pragma unroll
    for (int img = 0; img < 2; img++) {
        const void *src = img ? J.src_r : J.src_l;
        T acc = 0;
#pragma unroll
        for (int a = 0; a < 5; a++) {
            size_t r0 = (size_t)rows[a] * J.src_pitch;
            T h = 0;
#pragma unroll
            for (int b = 0; b < 5; b++) h += (T)kBinom5[b] * pixv<T, U8>(src, r0 + cols[b]);
            acc += (T)kBinom5[a] * h;
        }
        const bool ok = pyr_valid<T, U8>(src, J.src_pitch, J.ws, J.hs, x, y, kp);
        T *dst = static_cast<T *>(img ? J.dst_r : J.dst_l);
        dst[i] = ok ? acc : -acc;  // -0 keeps the invalid flag for a zero value
    }
}

// Block lb of a pyramid job: ppt coarse pixels per thread (1 for a launch
// per level, more for the coarser tasks of the persistent kernel).
__host__ __device__ constexpr int pyr_blocks(int wd, int hd, int ppt) {
    return (wd * hd + kBlock * ppt - 1) / (kBlock * ppt);
}

template <typename T, bool U8>
__device__ __forceinline__ void pyr_block(const PyrJob &J, int lb, const KParams &kp) {
    const int n = J.wd * J.hd;
    for (int q = 0; q < J.ppt; q++) {
        int i = (lb * J.ppt + q) * kBlock + (int)threadIdx.x;
        if (i < n) pyr_pixel<T, U8>(J, i, kp);
    }
}

// Two levels per launch, separable through LDS.  The block's level-(l+2)
// tile reads level l+1 at rows and columns 2 t - 2 .. 2 t + 2 (reflect-101);
// that region ("mid", virtual coordinates) holds, at each position, the
// level-(l+1) value of the reflected position.  Its in-image part is filtered
// from level l in two passes -- rows of level l in x into H, then H in y --
// the out-of-image part is copied from the reflected entries (always inside
// the region), and the tile is filtered from mid.  The sums run in the same
// order as pyr_pixel's, so both levels equal two single-level launches bit
// for bit; the level-(l+1) pixels under the tile are written out as well.
constexpr int kP2X = 16, kP2Y = 8;                         // level-(l+2) tile
constexpr int kP2MX = 2 * kP2X + 3, kP2MY = 2 * kP2Y + 3;  // level-(l+1) region
constexpr int kP2HY = 2 * (kP2MY - 1) + 5;                 // level-l rows of H
static_assert(2 * kP2X * kP2Y == kBlock, "one thread per (image, tile pixel)");

template <typename T, bool U8>
__global__ __launch_bounds__(kBlock) void k_pyr2(const JobPack<Pyr2Job> pk, KParams kp) {
    // from 8-bit pixels the row sums are multiples of 1/16 below 256: exact in
    // float, so H takes half the LDS (more blocks per CU) at no cost in bits
    using HT = std::conditional_t<U8, float, T>;
    __shared__ HT Hs[2][kP2HY][kP2MX];
    __shared__ uint8_t Vs[2][kP2HY][kP2MX];  // bits: source pixels xc, xc + 1 valid
    __shared__ T mid[2][kP2MY][kP2MX];       // signed: sign bit = validity
    const int bid = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const Pyr2Job &J = pk.j[find_job(pk, bid)];
    const int lb = bid - J.block0;
    const int ty = lb / J.tiles_x, tx = lb - ty * J.tiles_x;
    const int x2_0 = tx * kP2X, y2_0 = ty * kP2Y;
    const int vx0 = 2 * x2_0 - 2, vy0 = 2 * y2_0 - 2;  // virtual origin of mid
    // mid entries the tile reads (all of them are needed only with has2)
    const int vx_end = J.has2 ? min(vx0 + kP2MX, 2 * J.wd + 1) : min(2 * x2_0 + 2 * kP2X, J.wm);
    const int vy_end = J.has2 ? min(vy0 + kP2MY, 2 * J.hd + 1) : min(2 * y2_0 + 2 * kP2Y, J.hm);
    // in-image part [xa, xb) x [ya, yb) of level l+1
    const int xa = J.has2 ? max(vx0, 0) : 2 * x2_0, xb = min(vx_end, J.wm);
    const int ya = J.has2 ? max(vy0, 0) : 2 * y2_0, yb = min(vy_end, J.hm);
    const int ncol = xb - xa, nhrow = 2 * (yb - ya - 1) + 5;
    // pass 1: H[r][c] = sum_b w_b src(row(2 ya - 2 + r), col(2 (xa + c) + b - 2)).
    // A thread takes the entries c, c + 1 of a row together: their taps
    // overlap in three columns, so 7 loads serve both (the loads pass through
    // the compute unit's address unit one instruction at a time).  Fixed trip
    // count and clamped indices keep the loop one basic block, so every load
    // of the thread is in flight before the first sum.
    const int npr = (ncol + 1) / 2, np = nhrow * npr;  // entry pairs per row, in all
    constexpr int NP1 = (kP2HY * ((kP2MX + 1) / 2) + kBlock - 1) / kBlock;
    // q / n for the region's small indices without an integer division
    const double inv_ncol = 1.0 / (double)ncol, inv_npr = 1.0 / (double)npr;
    auto row_of = [&](int q) { return div_exact(q, inv_ncol); };
    T hv[NP1][2][2];
    uint32_t vb[NP1][2][2];  // validity of the source pixels at columns xc, xc + 1 of the row
    // every tap is within 2 of the image (one reflection) unless a side < 3:
    // one uniform branch picks a straight-line copy of the loop, so that
    // every load of the thread goes out back to back
    auto pass1 = [&](auto NEAR_) {
        constexpr bool NEAR = decltype(NEAR_)::value;
        auto refl = [&](int i, int n) {
            if constexpr (NEAR) return reflect101_near(i, n);
            else return reflect101(i, n);
        };
#pragma unroll
        for (int it = 0; it < NP1; it++) {
            const int pq = min((int)threadIdx.x + it * kBlock, np - 1);
            const int r = div_exact(pq, inv_npr), c = 2 * (pq - r * npr);
            const size_t r0 = (size_t)refl(2 * ya - 2 + r, J.hs) * J.src_pitch;
            const int xc = 2 * (xa + c);
#pragma unroll
            for (int img = 0; img < 2; img++) {
                const void *src = img ? J.src_r : J.src_l;
                T x[7];
                bool v[7];
#pragma unroll
                for (int k = 0; k < 7; k++) x[k] = pix<T, U8>(src, r0 + refl(xc + k - 2, J.ws), kp, v[k]);
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    T h = 0;
#pragma unroll
                    for (int b = 0; b < 5; b++) h += (T)kBinom5[b] * x[2 * e + b];
                    hv[it][e][img] = h;
                    // a missing child counts as valid
                    vb[it][e][img] = (v[2 * e + 2] ? 1u : 0u) | ((v[2 * e + 3] || xc + 2 * e + 1 >= J.ws) ? 2u : 0u);
                }
            }
        }
    };
    if (J.ws >= 3 && J.hs >= 3) pass1(std::true_type());
    else pass1(std::false_type());
#pragma unroll
    for (int it = 0; it < NP1; it++) {
        const int pq = (int)threadIdx.x + it * kBlock;
        if (pq < np) {
            const int r = div_exact(pq, inv_npr), c = 2 * (pq - r * npr);
#pragma unroll
            for (int e = 0; e < 2; e++) {
                if (c + e >= ncol) continue;
#pragma unroll
                for (int img = 0; img < 2; img++) {
                    Hs[img][r][c + e] = (HT)hv[it][e][img];
                    Vs[img][r][c + e] = (uint8_t)vb[it][e][img];
                }
            }
        }
    }
    __syncthreads();
    // pass 2: the level-(l+1) values, their validity (the 2 x 2 children:
    // rows 2 r + 2, 2 r + 3 of H) and the owned writes.  Without level l+2,
    // the in-image entries; with it, every entry of the mid region, an
    // out-of-image one computed at its reflected position (always inside the
    // region): the same value as a copy of that entry, without a second pass
    // and barrier.
    auto mid_value = [&](int img, int r, int c, int ym) -> T {
        const bool row2 = 2 * ym + 1 < J.hs;
        T acc = 0;
#pragma unroll
        for (int a = 0; a < 5; a++) acc += (T)kBinom5[a] * (T)Hs[img][2 * r + a][c];
        const bool ok = Vs[img][2 * r + 2][c] == 3u && (!row2 || Vs[img][2 * r + 3][c] == 3u);
        return ok ? acc : -acc;
    };
    constexpr int NQ2 = (kP2MY * kP2MX + kBlock - 1) / kBlock;
    if (!J.has2) {
        const int n2 = (yb - ya) * ncol;
#pragma unroll
        for (int it = 0; it < NQ2; it++) {
            const int q = (int)threadIdx.x + it * kBlock;
            if (q >= n2) continue;
            const int r = row_of(q), c = q - r * ncol;
            const int ym = ya + r, xm = xa + c;
            const bool own = ym >= 2 * y2_0 && ym < 2 * y2_0 + 2 * kP2Y && xm >= 2 * x2_0 && xm < 2 * x2_0 + 2 * kP2X;
#pragma unroll
            for (int img = 0; img < 2; img++)
                if (own) static_cast<T *>(img ? J.mid_r : J.mid_l)[(size_t)ym * J.wm + xm] = mid_value(img, r, c, ym);
        }
        return;  // uniform over the block
    }
    const bool nearm = J.wm >= 3 && J.hm >= 3;
#pragma unroll
    for (int it = 0; it < NQ2; it++) {
        const int q = (int)threadIdx.x + it * kBlock;
        const int t = q / kP2MX, cc = q - t * kP2MX;
        const int vy = vy0 + t, vx = vx0 + cc;
        if (q >= kP2MY * kP2MX || vy >= vy_end || vx >= vx_end) continue;
        const int ym = nearm ? reflect101_near(vy, J.hm) : reflect101(vy, J.hm);
        const int xm = nearm ? reflect101_near(vx, J.wm) : reflect101(vx, J.wm);
        const int r = ym - ya, c = xm - xa;
        const bool own = vy == ym && vx == xm && ym >= 2 * y2_0 && ym < 2 * y2_0 + 2 * kP2Y &&
                         xm >= 2 * x2_0 && xm < 2 * x2_0 + 2 * kP2X;
#pragma unroll
        for (int img = 0; img < 2; img++) {
            const T v = mid_value(img, r, c, ym);
            mid[img][t][cc] = v;
            if (own) static_cast<T *>(img ? J.mid_r : J.mid_l)[(size_t)ym * J.wm + xm] = v;
        }
    }
    __syncthreads();
    // level l+2: thread = (image, pixel of the kP2X x kP2Y tile)
    const int img = (int)threadIdx.x / (kP2X * kP2Y), pxl = (int)threadIdx.x % (kP2X * kP2Y);
    const int x2 = x2_0 + pxl % kP2X, y2 = y2_0 + pxl / kP2X;
    if (x2 >= J.wd || y2 >= J.hd) return;
    const int t0 = 2 * (y2 - y2_0), c0 = 2 * (x2 - x2_0);  // mid index of tap -2
    T acc = 0;
#pragma unroll
    for (int a = 0; a < 5; a++) {
        T h = 0;
#pragma unroll
        for (int b = 0; b < 5; b++) h += (T)kBinom5[b] * fabs(mid[img][t0 + a][c0 + b]);
        acc += (T)kBinom5[a] * h;
    }
    bool ok = true;
#pragma unroll
    for (int dy = 0; dy < 2; dy++)
#pragma unroll
        for (int dx = 0; dx < 2; dx++)
            if (2 * y2 + dy < J.hm && 2 * x2 + dx < J.wm) ok = ok && !signbit(mid[img][t0 + 2 + dy][c0 + 2 + dx]);
    static_cast<T *>(img ? J.dst_r : J.dst_l)[(size_t)y2 * J.wd + x2] = ok ? acc : -acc;
}

// ---------------------------------------------------------------- densify: value of one pixel

// The fields of a densification that dense_value reads.
struct DenseView {
    const void *L, *R, *rec_u, *rec_w, *gtab, *Uc;
    int pitch, W, H, patch, stride, nx, ny, Wc, Hc, mode;
};

// One pixel: kept covering patches in (row, column) order, weight = patch
// posterior x spatial Gaussian at the pixel's offset in the patch (Bayesian)
// or 1 / max(residual^2, 1) (DIS eq. (2)); U = sum(w u) / sum(w).  Uncovered:
// NaN at level 0, zero at the coarsest level, else twice the coarse field.
// V is a DenseJob or a DenseView: the fields the value needs.
template <typename T, bool U8, int NC = 2, typename V>
__device__ __forceinline__ T dense_value(const V &J, const int x, const int y, const KParams &kp) {
    // no contraction into FMAs: the value must be the same bits wherever it
    // is evaluated (densify kernel, LK launch, fast path or loop)
#pragma clang fp contract(off)
    const int P = J.patch, st = J.stride;
    const T *rec_u = static_cast<const T *>(J.rec_u);
    const T *rec_w = static_cast<const T *>(J.rec_w);
    const T *gtab = static_cast<const T *>(J.gtab);
    const double inv_st = 1.0 / (double)st;
    auto range = [&](int v, int n, int cnt, int &lo, int &hi, int &extra) {
        int t = v - P + 1;
        lo = t > 0 ? div_exact(t + st - 1, inv_st) : 0;
        hi = min(cnt - 1, div_exact(v, inv_st));
        extra = (hi < cnt - 1 && v >= n - P) ? cnt - 1 : -1;
    };
    int xlo, xhi, xex, ylo, yhi, yex;
    range(x, J.W, J.nx, xlo, xhi, xex);
    range(y, J.H, J.ny, ylo, yhi, yex);
    // The fallback field's taps are loaded here and mixed only at the end,
    // so that they go out with the patch records (one round trip): mixed
    // here, they would be waited for before the records' loads are issued.
    T f00 = 0, f01 = 0, f10 = 0, f11 = 0, ffx = 0, ffy = 0;
    if (J.mode == 0) {
        const T *Uc = static_cast<const T *>(J.Uc);
        int mx, my, mx1, my1;
        bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * (T)x, T(0.5) * (T)y, mx, my, mx1, my1, ffx, ffy);
        f00 = Uc[(size_t)my * J.Wc + mx];
        f01 = Uc[(size_t)my * J.Wc + mx1];
        f10 = Uc[(size_t)my1 * J.Wc + mx];
        f11 = Uc[(size_t)my1 * J.Wc + mx1];
    }
    T A = 0, B = 0;
    auto add = [&](int py, int px, T wk, T uk, T g) {
        T w;
        if (kp.fusion == 1) {
            size_t row0 = (size_t)y * J.pitch;
            T uc = fmin(fmax(uk, -(T)(J.W + 2)), (T)(J.W + 2));
            T ui = floor(uc), uf = uc - ui;
            T res = sample_row<T, U8>(J.R, row0, J.W, x + (int)ui, uf) - pixv<T, U8>(J.L, row0 + x);
            T q = res * res;
            w = T(1) / (q > T(1) ? q : T(1));
        } else {
            w = wk * g;
        }
        A += w;
        B += w * uk;
    };
    // Fast paths: at most 2 (or, with NC = 3, 3) candidate patches per axis
    // (lo .. hi, then the one snapped to the border), every record and mask
    // load issued before the sums, which run in the same (row, column) order
    // as the loop below.  Two per axis covers the interior at stride >= patch
    // / 2; three also the rows and columns next to a snapped border patch,
    // for the LK launches that densify (registers are free there, and one
    // slow block sets the launch time).  The densify kernel keeps NC = 2: a
    // wider path would cost occupancy, and it is bound by its gathers.
    const int ncx = xhi - xlo + 1 + (xex >= 0 ? 1 : 0), ncy = yhi - ylo + 1 + (yex >= 0 ? 1 : 0);
    auto fast = [&](auto M_) {
        constexpr int M = decltype(M_)::value;
        int px[M], py[M], jxs[M], jys[M];
        bool vx[M], vy[M];
#pragma unroll
        for (int i = 0; i < M; i++) {
            int jx = i <= xhi - xlo ? xlo + i : (i == xhi - xlo + 1 ? xex : -1);
            int jy = i <= yhi - ylo ? ylo + i : (i == yhi - ylo + 1 ? yex : -1);
            px[i] = jx >= 0 ? grid_pos(jx, J.W, P, st) : 0;
            py[i] = jy >= 0 ? grid_pos(jy, J.H, P, st) : 0;
            vx[i] = jx >= 0 && x >= px[i] && x < px[i] + P;
            vy[i] = jy >= 0 && y >= py[i] && y < py[i] + P;
            jxs[i] = vx[i] ? jx : 0;
            jys[i] = vy[i] ? jy : 0;
        }
        T wk[M][M], uk[M][M], g[M][M];
#pragma unroll
        for (int iy = 0; iy < M; iy++)
#pragma unroll
            for (int ix = 0; ix < M; ix++) {
                const bool v = vy[iy] && vx[ix];
                const int k = v ? jys[iy] * J.nx + jxs[ix] : 0;
                wk[iy][ix] = rec_w[k];
                uk[iy][ix] = rec_u[k];
                g[iy][ix] = gtab[v ? (y - py[iy]) * P + (x - px[ix]) : 0];
                if (!v) wk[iy][ix] = T(0);
            }
#pragma unroll
        for (int iy = 0; iy < M; iy++)
#pragma unroll
            for (int ix = 0; ix < M; ix++)
                if (wk[iy][ix] > T(0)) add(py[iy], px[ix], wk[iy][ix], uk[iy][ix], g[iy][ix]);
    };
    if (ncx <= 2 && ncy <= 2) {
        fast(std::integral_constant<int, 2>());
    } else if (NC >= 3 && ncx <= 3 && ncy <= 3) {
        fast(std::integral_constant<int, (NC >= 3 ? 3 : 2)>());
    } else {
    for (int jy = ylo; jy <= (yex >= 0 ? yex : yhi); jy++) {
        if (jy > yhi && jy != yex) continue;
        int py = grid_pos(jy, J.H, P, st);
        if (y < py || y >= py + P) continue;
        for (int jx = xlo; jx <= (xex >= 0 ? xex : xhi); jx++) {
            if (jx > xhi && jx != xex) continue;
            int px = grid_pos(jx, J.W, P, st);
            if (x < px || x >= px + P) continue;
            int k = jy * J.nx + jx;
            T wk = rec_w[k];
            if (!(wk > T(0))) continue;
            add(py, px, wk, rec_u[k], gtab[(y - py) * P + (x - px)]);
        }
    }
    }
    if (A > T(0)) return B / A;
    if (J.mode == 2) return (T)__builtin_nan("");
    if (J.mode == 1) return 0;
    return T(2) * bilinear_mix<T>(f00, f01, f10, f11, ffx, ffy);
}

// dense_value for the Bayesian fusion in two halves, so that the loads of
// several pixels go out together: dense_gather issues a pixel's loads (the
// fast path's records, spatial weights and fallback taps), dense_finish sums
// them with dense_value's arithmetic in its order, or calls dense_value for a
// pixel outside the fast path.
template <typename T, int NC = 2>
struct DenseG {
    T wk[NC][NC], uk[NC][NC], g[NC][NC];
    T f00, f01, f10, f11, ffx, ffy;
    bool fast;
};
template <typename T, int NC, typename V>
__device__ __forceinline__ void dense_gather(const V &J, const int x, const int y, DenseG<T, NC> &G) {
#pragma clang fp contract(off)
    const int P = J.patch, st = J.stride;
    const T *rec_u = static_cast<const T *>(J.rec_u);
    const T *rec_w = static_cast<const T *>(J.rec_w);
    const T *gtab = static_cast<const T *>(J.gtab);
    const double inv_st = 1.0 / (double)st;
    auto range = [&](int v, int n, int cnt, int &lo, int &hi, int &extra) {
        int t = v - P + 1;
        lo = t > 0 ? div_exact(t + st - 1, inv_st) : 0;
        hi = min(cnt - 1, div_exact(v, inv_st));
        extra = (hi < cnt - 1 && v >= n - P) ? cnt - 1 : -1;
    };
    int xlo, xhi, xex, ylo, yhi, yex;
    range(x, J.W, J.nx, xlo, xhi, xex);
    range(y, J.H, J.ny, ylo, yhi, yex);
    G.f00 = G.f01 = G.f10 = G.f11 = G.ffx = G.ffy = T(0);
    if (J.mode == 0) {
        const T *Uc = static_cast<const T *>(J.Uc);
        int mx, my, mx1, my1;
        bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * (T)x, T(0.5) * (T)y, mx, my, mx1, my1, G.ffx, G.ffy);
        G.f00 = Uc[(size_t)my * J.Wc + mx];
        G.f01 = Uc[(size_t)my * J.Wc + mx1];
        G.f10 = Uc[(size_t)my1 * J.Wc + mx];
        G.f11 = Uc[(size_t)my1 * J.Wc + mx1];
    }
    const int ncx = xhi - xlo + 1 + (xex >= 0 ? 1 : 0), ncy = yhi - ylo + 1 + (yex >= 0 ? 1 : 0);
    G.fast = ncx <= NC && ncy <= NC;
    int px[NC], py[NC], jxs[NC], jys[NC];
    bool vx[NC], vy[NC];
#pragma unroll
    for (int i = 0; i < NC; i++) {
        int jx = i <= xhi - xlo ? xlo + i : (i == xhi - xlo + 1 ? xex : -1);
        int jy = i <= yhi - ylo ? ylo + i : (i == yhi - ylo + 1 ? yex : -1);
        px[i] = jx >= 0 ? grid_pos(jx, J.W, P, st) : 0;
        py[i] = jy >= 0 ? grid_pos(jy, J.H, P, st) : 0;
        vx[i] = G.fast && jx >= 0 && x >= px[i] && x < px[i] + P;
        vy[i] = G.fast && jy >= 0 && y >= py[i] && y < py[i] + P;
        jxs[i] = vx[i] ? jx : 0;
        jys[i] = vy[i] ? jy : 0;
    }
#pragma unroll
    for (int iy = 0; iy < NC; iy++)
#pragma unroll
        for (int ix = 0; ix < NC; ix++) {
            const bool v = vy[iy] && vx[ix];
            const int k = v ? jys[iy] * J.nx + jxs[ix] : 0;
            G.wk[iy][ix] = rec_w[k];
            G.uk[iy][ix] = rec_u[k];
            G.g[iy][ix] = gtab[v ? (y - py[iy]) * P + (x - px[ix]) : 0];
            if (!v) G.wk[iy][ix] = T(0);
        }
}
template <typename T, bool U8, int NC, typename V>
__device__ __forceinline__ T dense_finish(const V &J, const int x, const int y, const KParams &kp,
                                          const DenseG<T, NC> &G) {
#pragma clang fp contract(off)
    if (!G.fast) return dense_value<T, U8, 3>(J, x, y, kp);
    T A = 0, B = 0;
#pragma unroll
    for (int iy = 0; iy < NC; iy++)
#pragma unroll
        for (int ix = 0; ix < NC; ix++)
            if (G.wk[iy][ix] > T(0)) {
                const T w = G.wk[iy][ix] * G.g[iy][ix];
                A += w;
                B += w * G.uk[iy][ix];
            }
    if (A > T(0)) return B / A;
    if (J.mode == 2) return (T)__builtin_nan("");
    if (J.mode == 1) return 0;
    return T(2) * bilinear_mix<T>(G.f00, G.f01, G.f10, G.f11, G.ffx, G.ffy);
}

// ---------------------------------------------------------------- LK + posterior

enum { ST_KEPT = 0, ST_DEGENERATE = 1, ST_DIVERGED = 2, ST_GATED = 3 };

// Patches per block and the widest span of right-image columns a block stages.
template <int P> struct LkShape {
    static constexpr int SEG = P <= 8 ? 8 : 16;  // lanes per patch (one per patch row)
    static constexpr int PPB = kBlock / SEG;     // patches per block, one patch row
    static constexpr int NCROW = 385;            // LDS row stride, elements
    static constexpr int PADC = P + 1;           // columns staged beyond each end of the span
    static constexpr int NCMAX = NCROW - 1 - 2 * PADC;  // widest span of image columns
};

template <int P>
__host__ __device__ constexpr int lk_blocks_per_row(int nx) {
    return (nx + LkShape<P>::PPB - 1) / LkShape<P>::PPB;
}

// A block takes up to PPB consecutive patches of one patch row.  It stages
// the P right-image rows of those patches in LDS over the columns their
// initial shifts reach, plus a margin of P + 2 (a kept patch ends within P
// of its start; the window adds 1), so every LK iteration and window sample
// reads LDS; an iterate outside the staged span reads global memory instead,
// with the same values.  The span is staged with P + 1 more columns at each
// end, indices clamped to the row: where it meets the image border those
// hold the border pixel, so a sample that the linear sampler clamps (Sec.
// 2.1, eq. (1)) reads the same LDS run as any other.
//
// One patch per segment of SEG lanes, one patch row per lane (lanes >= P of a
// 16-lane segment idle).  Per lane: the template row, the mean-normalised
// template gradient J (the inverse-compositional Jacobian, computed once on
// the left patch, Sec. 2.1), then K Gauss-Newton steps u <- u - sum(J e)/H
// sampling the right row at the current shift.  Because sum J = 0 over the
// left-valid pixels, sum J e equals sum J d without subtracting the residual
// mean.  A patch is kept only if the iteration converged (last step within
// conv_tol, shift within a patch side of its start).  Then the window
// energies E_i = sum (d - mean d)^2 at u + (i - c) step, the posterior
// p = 1 / sum_i exp(-(E_i - E_c) / tau) (eqs. (3)-(4)) and the gamma gate.
template <typename T, int P>
__host__ __device__ constexpr int lk_lds_bytes() { return P * LkShape<P>::NCROW * (int)sizeof(T); }

// Block lb of an LK job; Rs is the block's LDS staging area of
// lk_lds_bytes<T, P>() bytes.  WN >= kp.window bounds the window samples
// (5 for the paper's window, 9 for any allowed one).  FOLD compiles the
// densification of level + 1 in (used when J.rec_u1 is set); MERGE gathers
// the first pixel of the block's share of that field with the taps (more
// registers: for launches of at most two blocks per CU).
template <typename T, int P, bool U8, int WN = 9, bool FOLD = false, bool MERGE = false>
__device__ __forceinline__ void lk_block(const LkJob &J, const int lb, const KParams &kp, T *__restrict__ Rs) {
    // no implicit contraction: every fused multiply-add is written out, so
    // that the one-lane-per-pixel kernel can repeat the arithmetic exactly
#pragma clang fp contract(off)
    using S = LkShape<P>;
    constexpr int SEG = S::SEG, PPB = S::PPB, NCMAX = S::NCMAX, NCROW = S::NCROW, PADC = S::PADC;
    // patch sides up to 8: sums over the eight column slots of each row in
    // the fixed order of row_sum8 / row_dot8
    constexpr bool CAN = P <= 8;

    const int W = J.W;
    const int bpr = lk_blocks_per_row<P>(J.nx);
    const int jy = lb / bpr, jx0 = (lb - jy * bpr) * PPB;
    const int slot = (int)threadIdx.x / SEG, r = (int)threadIdx.x % SEG;
    const int jx_raw = jx0 + slot;
    const bool live = jx_raw < J.nx;
    const int jx = live ? jx_raw : J.nx - 1;  // idle segments shadow the row's last patch
    const int k = jy * J.nx + jx;
    const int x0 = grid_pos(jx, W, P, J.stride), y0 = grid_pos(jy, J.H, P, J.stride);
    const bool row_on = r < P;
    const int y = y0 + (row_on ? r : 0);
    const size_t row0 = (size_t)y * J.pitch;

    // template row and gradient (independent of the shift: issued first).
    // One read of the P + 2 columns x0 - 1 .. x0 + P, clamped to the row,
    // serves the template and both neighbours of the central difference.
    T Tv[P], Jg[P];
    uint32_t vmask = 0;
    {
        T raw[P + 2];
        bool rv[P + 2];
#pragma unroll
        for (int j = 0; j < P + 2; j++)
            raw[j] = pix<T, U8>(J.L, row0 + min(max(x0 - 1 + j, 0), W - 1), kp, rv[j]);
#pragma unroll
        for (int c = 0; c < P; c++) {
            Tv[c] = raw[c + 1];
            Jg[c] = T(0.5) * (raw[c + 2] - raw[c]);
            vmask |= (uint32_t)(rv[c + 1] && row_on) << c;
        }
    }

    const T ulo = -(T)(W + P + 2), uhi = (T)(W + 2);
    // densification of level + 1 when this launch does it (J.rec_u1 set)
    DenseView D;
    D.L = D.R = nullptr;
    D.rec_u = J.rec_u1; D.rec_w = J.rec_w1; D.gtab = J.gtab1; D.Uc = J.U2;
    D.pitch = 0; D.W = J.Wc; D.H = J.Hc; D.patch = P; D.stride = J.stride;
    D.nx = J.Wc < P ? 0 : (J.Wc - P + J.stride - 1) / J.stride + 1;
    D.ny = J.Hc < P ? 0 : (J.Hc - P + J.stride - 1) / J.stride + 1;
    D.Wc = (J.Wc + 1) / 2; D.Hc = (J.Hc + 1) / 2;
    D.mode = J.U2 ? 0 : 1;
    // Integer part (and fraction) of a shift for the sampler.  The sampler
    // clamps the shift to [ulo, uhi]; beyond that range every column of the
    // patch row lies outside the image and reads its border pixel whatever
    // the fraction is, so clamping the integer part alone gives the same
    // samples and keeps the clamp off the iteration's dependency chain.
    auto ishift = [&](T v, T &uf) -> int {
        const T fl = floor(v);
        uf = v - fl;
        return min(max((int)fl, -(W + P + 2)), W + 2);
    };
    T u0 = 0;

    // Staged span of the block's right rows, from static bounds so the loads
    // go out with the template and init loads: disparities d >= 0 shift the
    // right sample left (u = -d), so the span reaches `reach` columns left of
    // the first patch and a margin of P + 2 on both sides.
    // The rest of the NCMAX columns (they cost no extra load instruction:
    // the chunks are sized for NCMAX) widen the span on both sides, so that
    // an iterate that wanders beyond the expected disparities on its way
    // still reads LDS: every iteration outside the span is a round trip to
    // memory, and one such patch holds up its wave and its block.
    const int xf = grid_pos(jx0, W, P, J.stride);
    const int xl = grid_pos(min(jx0 + PPB, J.nx) - 1, W, P, J.stride);
    int col_hi = min(W - 1, xl + P + (P + 2));
    int col_lo = max(0, xf - J.reach - (P + 2));
    col_lo = max(col_lo, col_hi - NCMAX + 1);
    {
        // spare columns: half to each side where the row allows, the rest
        // to the side that has room (0 <= col_lo <= col_hi <= W - 1 and at
        // most NCMAX columns hold throughout)
        const int extra = NCMAX - (col_hi - col_lo + 1);
        int left = min(col_lo, extra / 2);
        const int right = min(W - 1 - col_hi, extra - left);
        left = min(col_lo, extra - right);
        col_lo -= left;
        col_hi += right;
    }
    // LDS row r holds R[clamp(k, 0, W - 1)] for the virtual columns
    // k = vlo .. vhi at index k - vlo
    const int vlo = col_lo - PADC, vhi = col_hi + PADC;
    const int nst = vhi - vlo + 1;
    // rows in passes of up to 8, columns in chunks of kBlock: every load of a
    // pass is issued before the LDS writes (one memory round trip per pass);
    // the first pass's loads go out before the initial shift waits for its
    // own, so template, staging and init share one round trip
    constexpr int CH = (NCROW - 1 + kBlock - 1) / kBlock;
#pragma unroll
    for (int r0 = 0; r0 < P; r0 += 8) {
        // Every lane loads (the column clamped into the staged span), with no
        // branch around the load and the uint8 -> T conversion left to the
        // LDS write: a load inside a branch, or converted inside one, is
        // waited for there, one memory round trip per load.
        using RawT = std::conditional_t<U8, uint8_t, T>;
        RawT buf[8][CH];
#pragma unroll
        for (int rr = 0; rr < 8; rr++)
#pragma unroll
            for (int q = 0; q < CH; q++) {
                const int cc = min((int)threadIdx.x + q * kBlock, nst - 1);
                if (r0 + rr < P) {
                    const size_t g = (size_t)(y0 + r0 + rr) * J.pitch + (size_t)min(max(vlo + cc, 0), W - 1);
                    buf[rr][q] = static_cast<const RawT *>(J.R)[g];
                }
            }
        if (r0 == 0 && J.Uc) {
            // initial shift: twice the coarse field at the patch centre (Sec. 2.1)
            T cx = (T)x0 + T(0.5) * (T)(P - 1), cy = (T)y0 + T(0.5) * (T)(P - 1);
            if (!FOLD || !J.rec_u1) {
                u0 = T(2) * bilinear<T>(static_cast<const T *>(J.Uc), J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy);
            } else if constexpr (FOLD) {
                // Level + 1 is densified here rather than by a launch of its
                // own: the block writes its share of that field (the next
                // level's fallback reads it) and evaluates the four bilinear
                // taps of each patch centre itself, lane r of a segment tap
                // r mod 4, with the same arithmetic as the densify kernel.
                int mx, my, mx1, my1;
                T fx, fy;
                bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * cx, T(0.5) * cy, mx, my, mx1, my1, fx, fy);
                const int tap = r & 3, tx = (tap & 1) ? mx1 : mx, ty = (tap & 2) ? my1 : my;
                T F;
                // this block's share of the level-(l+1) field, which the next
                // finer level reads where its own patches leave a pixel
                // uncovered.  Its first pixel per thread is gathered with the
                // tap, so that both go out in one round trip.  At level 0 (the
                // uint8 launch) there is no finer level: the output leaves
                // uncovered pixels unestimated, so the level-1 field is not
                // written.
                if constexpr (!U8 && MERGE) {
                    const int n1 = J.Wc * J.Hc, nblk = J.ny * bpr, chunk = (n1 + nblk - 1) / nblk;
                    const int i0 = lb * chunk, i1 = min(n1, (lb + 1) * chunk);
                    const double inv_wc = 1.0 / (double)J.Wc;
                    const int ia = i0 + (int)threadIdx.x;
                    // lanes past the share gather a pixel of it anyway (i0 < i1:
                    // every block has a share) and do not store it
                    const int ic = min(ia, i1 - 1);
                    const int ya = div_exact(ic, inv_wc), xa = ic - ya * J.Wc;
                    DenseG<T, 2> Gt, Gs;
                    dense_gather<T, 2>(D, tx, ty, Gt);
                    dense_gather<T, 2>(D, xa, ya, Gs);
                    F = dense_finish<T, false, 2>(D, tx, ty, kp, Gt);
                    const T Us = dense_finish<T, false, 2>(D, xa, ya, kp, Gs);
                    if (ia < i1) static_cast<T *>(J.Uc)[ia] = Us;
                    for (int i = ia + kBlock; i < i1; i += kBlock) {
                        const int yy = div_exact(i, inv_wc), xx = i - yy * J.Wc;
                        static_cast<T *>(J.Uc)[i] = dense_value<T, false, 3>(D, xx, yy, kp);
                    }
                } else {
                    F = dense_value<T, false, 3>(D, tx, ty, kp);
                    if constexpr (!U8) {
                        const int n1 = J.Wc * J.Hc, nblk = J.ny * bpr, chunk = (n1 + nblk - 1) / nblk;
                        const int i1 = min(n1, (lb + 1) * chunk);
                        const double inv_wc = 1.0 / (double)J.Wc;
                        for (int i = lb * chunk + (int)threadIdx.x; i < i1; i += kBlock) {
                            const int yy = div_exact(i, inv_wc), xx = i - yy * J.Wc;
                            static_cast<T *>(J.Uc)[i] = dense_value<T, false, 3>(D, xx, yy, kp);
                        }
                    }
                }
                const T f00 = dpp_v<0x00>(F), f01 = dpp_v<0x55>(F), f10 = dpp_v<0xAA>(F), f11 = dpp_v<0xFF>(F);
                u0 = T(2) * bilinear_mix<T>(f00, f01, f10, f11, fx, fy);
            }
        }
#pragma unroll
        for (int rr = 0; rr < 8; rr++)
#pragma unroll
            for (int q = 0; q < CH; q++) {
                int cc = (int)threadIdx.x + q * kBlock;
                if (r0 + rr < P && cc < nst) Rs[(r0 + rr) * NCROW + cc] = (T)buf[rr][q];
            }
    }
    __syncthreads();

    // LDS index of virtual column k of this lane's staged row is rbase + k,
    // which is >= 0 exactly for k >= vlo (the array is only ever indexed,
    // never offset before its start)
    const int rbase = (row_on ? r : 0) * NCROW - vlo;
    // raw right values (sign = validity above level 0) of columns
    // clamp(c0 + c, 0, W-1), c = 0..N-1: all reads issued back to back, from
    // LDS when the whole span is staged, else from global memory
    auto fetch = [&](int c0, T *v, auto N_) {
        constexpr int N = decltype(N_)::value;
        // Every value is read from LDS (indices kept inside the staged span),
        // and only the columns outside the span are then reloaded from
        // global memory.  The two reads stay distinct instructions: written as
        // alternatives, the compiler merges them into one flat load through a
        // generic pointer, which costs a memory round trip even for LDS.
        int idx[N];
#pragma unroll
        for (int c = 0; c < N; c++) {
            idx[c] = min(max(c0 + c, 0), W - 1);
            v[c] = Rs[rbase + min(max(idx[c], vlo), vhi)];
        }
        const bool staged = max(c0, 0) >= vlo && min(c0 + N - 1, W - 1) <= vhi;
        if (!staged) {
#pragma unroll
            for (int c = 0; c < N; c++) {
                if (idx[c] >= vlo && idx[c] <= vhi) continue;
                const size_t g = row0 + (size_t)idx[c];
                if constexpr (U8) v[c] = (T) static_cast<const uint8_t *>(J.R)[g];
                else v[c] = static_cast<const T *>(J.R)[g];
            }
        }
    };
    // Intensities R[clamp(xi0 + c, 0, W - 1)], c = 0..P, of this lane's row.
    // A start left of -(P + 1) or right of W - 1 gives the same values as
    // that bound (every column clamps to the border), so the clamped start
    // reads one contiguous run of the staged row; only a run that leaves the
    // staged span takes the per-column path.  The run is read from LDS in
    // any case, its start clamped into the span (no branch before the reads),
    // and read again per column only if that clamp moved it.
    auto load_run = [&](int xi0, T *v) {
        const int xc = min(max(xi0, -(P + 1)), W - 1);
        const int xs = min(max(xc, vlo), vhi - P);
#pragma unroll
        for (int c = 0; c <= P; c++) v[c] = Rs[rbase + xs + c];
        if (xs != xc) fetch(xi0, v, std::integral_constant<int, P + 1>());
#pragma unroll
        for (int c = 0; c <= P; c++)
            if constexpr (!U8) v[c] = fabs(v[c]);
    };

    int nloc = 0;
    T gsum = 0;
    if constexpr (CAN) {
        T t[8];
#pragma unroll
        for (int c = 0; c < 8; c++) t[c] = (c < P && ((vmask >> c) & 1u)) ? Jg[c < P ? c : 0] : T(0);
        gsum = row_sum8(t);
        nloc = __builtin_popcount(vmask);
    } else {
#pragma unroll
        for (int c = 0; c < P; c++)
            if ((vmask >> c) & 1u) { gsum += Jg[c]; nloc++; }
    }
    const int n = seg_sum_i<SEG>(nloc);
    gsum = seg_sum<SEG>(gsum);
    const T gmean = n > 0 ? gsum / (T)n : T(0);
    T hloc = 0;
#pragma unroll
    for (int c = 0; c < P; c++) Jg[c] = ((vmask >> c) & 1u) ? Jg[c] - gmean : T(0);
    // J and T in eight slots (zeros past the patch side)
    T J8[8], T8[8];
#pragma unroll
    for (int c = 0; c < 8; c++) {
        J8[c] = c < P ? Jg[c < P ? c : 0] : T(0);
        T8[c] = c < P ? Tv[c < P ? c : 0] : T(0);
    }
    if constexpr (CAN) {
        hloc = row_dot8(J8, J8);
    } else {
#pragma unroll
        for (int c = 0; c < P; c++) hloc = fma(Jg[c], Jg[c], hloc);
    }
    const T Hs = seg_sum<SEG>(hloc);

    int status = ST_KEPT;
    T u = u0, post = 0;
    if (n == 0 || !(Hs > (T)kp.eps_h * (T)n)) {
        status = ST_DEGENERATE;
    } else {
        T step = 0;
        const T invH = T(1) / Hs;
        // sum_c J_c T_c of this lane's row: the template part of sum J e
        T jt0 = 0, jt1 = 0;
        if constexpr (CAN) {
            jt0 = row_dot8(J8, T8);
        } else {
#pragma unroll
            for (int c = 0; c < P; c += 2) {
                jt0 = fma(Jg[c], Tv[c], jt0);
                if (c + 1 < P) jt1 = fma(Jg[c + 1], Tv[c + 1], jt1);
            }
        }
        // sum J T over the patch (constant over the iterations)
        const T JT = seg_sum<SEG>(CAN ? jt0 : jt0 + jt1);
        // The residual sum is linear in the fraction within one cell of the
        // shift: sum J I = A + f (B - A) over the patch, with A (B) the dot
        // product of J with the tap each sample takes at f = 0 (f = 1).
        // Inside the row those are R[m + c] and R[m + c + 1]; a column
        // clamped to the row's first (last) pixel takes that pixel at any f,
        // in A and in B alike.  A and B depend on the integer part only and f
        // is the same in every row, so they are reduced over the patch when
        // the iterate enters a cell, SA = A - sum J T and SD = B - A, and
        // every iteration in that cell (the common case once it is within a
        // pixel) is sum J e = SA + f SD: no cross-lane step, no LDS read.
        // The shift is the same in every lane of a segment (it comes from
        // segment totals), so the cell test is uniform per segment and the
        // reduction inside it sees its whole segment active.
        int xi_prev = INT_MIN;
        T SA = 0, SD = 0;
        for (int t = 0; t < kp.iters; t++) {
            T uf;
            const int xi0 = x0 + ishift(u, uf);
            if (xi0 != xi_prev) {
                xi_prev = xi0;
                // taps R[clamp(m + c)] and R[clamp(m + c + 1)] of the cell m
                T v[P + 1];
                load_run(xi0, v);
                T a0 = 0, a1 = 0, b0 = 0, b1 = 0;
                if constexpr (CAN) {
                    // row_dot8 of J with the taps at f = 0 and f = 1, pair by pair
                    T pa[4], pb[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int c0 = 2 * j, c1 = 2 * j + 1;
                        const T v0 = c0 < P ? v[c0 < P ? c0 : 0] : T(0), v1 = c1 < P ? v[c1 < P ? c1 : 0] : T(0);
                        const T v2 = c1 < P ? v[c1 < P ? c1 + 1 : 0] : T(0);
                        const T w1 = c0 < P ? v[c0 < P ? c0 + 1 : 0] : T(0);
                        pa[j] = fma(J8[c0], v0, J8[c1] * v1);
                        pb[j] = fma(J8[c0], w1, J8[c1] * v2);
                    }
                    a0 = (pa[0] + pa[1]) + (pa[2] + pa[3]);
                    b0 = (pb[0] + pb[1]) + (pb[2] + pb[3]);
                } else {
#pragma unroll
                    for (int c = 0; c < P; c += 2) {
                        a0 = fma(Jg[c], v[c], a0);
                        b0 = fma(Jg[c], v[c + 1], b0);
                        if (c + 1 < P) {
                            a1 = fma(Jg[c + 1], v[c + 1], a1);
                            b1 = fma(Jg[c + 1], v[c + 2], b1);
                        }
                    }
                }
                const T A = CAN ? a0 : a0 + a1, B = CAN ? b0 : b0 + b1;
                T ab[2] = {A, B};
                seg_sum_n<SEG, 2>(ab);
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
            // eqs. (3)-(4): residual energies E_i = sum (d - mean d)^2 of the
            // window samples u + (i - c) step, evaluated as
            // sum d^2 - (sum d)^2 / n with every window sum reduced at once
            // (in double precision the two forms agree to ~1e-13 relative)
            const int cw = (kp.window - 1) / 2;
            // The launches of at most two blocks per CU (MERGE) have the
            // registers to read every window sample's run, and the gate's
            // taps, in one batch (WBATCH); the others read them one by one.
            constexpr bool WBATCH = MERGE && P <= 12;
            // WN: compile-time bound on the window count (kp.window <= WN),
            // so that only the sums of samples that exist are reduced
            // waves whose patch rows are all left-valid (the common case)
            // skip the mask in the window sums; others apply it as a factor
            const bool allv = __all((int)(vmask == (1u << P) - 1u)) != 0;
            T mv[P];
#pragma unroll
            for (int c = 0; c < P; c++) mv[c] = ((vmask >> c) & 1u) ? T(1) : T(0);
            auto window_post = [&]() -> T {
                // With WBATCH the runs R[clamp(xi0 + c, 0, W-1)], c = 0..P,
                // of every sample are read before any is used: one LDS round
                // trip for all rather than one per sample.  A run inside the
                // staged span is read as is; any other is read with its start
                // clamped into the span and then again per column (load_run's
                // slow path).
                constexpr int WB = WBATCH ? WN : 1;
                int wxi[WB];
                T wuf[WB], wv[WB][P + 1];
                if constexpr (WBATCH) {
                    bool staged = true;
#pragma unroll
                    for (int i = 0; i < WN; i++) {
                        wxi[i] = 0;
                        wuf[i] = 0;
                        if (i < kp.window) {
                            const T ud = u + (T)(i - cw) * (T)kp.window_step;
                            wxi[i] = x0 + ishift(ud, wuf[i]);
                            const int xc = min(max(wxi[i], -(P + 1)), W - 1);
                            const int xs = min(max(xc, vlo), vhi - P);
                            staged = staged && xs == xc;
#pragma unroll
                            for (int c = 0; c <= P; c++) wv[i][c] = Rs[rbase + xs + c];
                        }
                    }
                    if (!staged) {
#pragma unroll
                        for (int i = 0; i < WN; i++) {
                            const int xc = min(max(wxi[i], -(P + 1)), W - 1);
                            if (i < kp.window && (xc < vlo || xc + P > vhi))
                                fetch(wxi[i], wv[i], std::integral_constant<int, P + 1>());
                        }
                    }
                }
                T acc[2 * WN];
#pragma unroll
                for (int i = 0; i < WN; i++) {
                    acc[2 * i] = 0;
                    acc[2 * i + 1] = 0;
                    if (i < kp.window) {
                        // I_r at x0 + c + shift, shift = xi0 - x0 + uf with
                        // 0 <= uf < 1, coordinate clamped to [0, W-1]:
                        // (1 - f) R[m] + f R[m + 1] on the clamped taps, which
                        // for a clamped column are the same pixel
                        T uf, v[P + 1];
                        if constexpr (WBATCH) {
                            uf = wuf[i];
#pragma unroll
                            for (int c = 0; c <= P; c++) v[c] = U8 ? wv[i][c] : T(fabs(wv[i][c]));
                        } else {
                            const T ud = u + (T)(i - cw) * (T)kp.window_step;
                            load_run(x0 + ishift(ud, uf), v);
                        }
                        const T omf = T(1) - uf;
                        // The left-valid mask enters as a 0/1 factor of the
                        // residual (the same bits as selecting it), and not
                        // at all in waves whose rows are all valid.
                        T s0 = 0, s1 = 0, e0 = 0, e1 = 0;
                        if constexpr (CAN) {
                            // row_sum8 of m = mask q and row_dot8 of (m, q),
                            // pair by pair (slots past the patch side:
                            // zeros); a wave whose rows are all valid takes
                            // m = q, the same bits as 1 q
                            T sp[4], ep[4];
                            auto pairs = [&](auto masked_) {
                                constexpr bool MASKED = decltype(masked_)::value;
#pragma unroll
                                for (int j = 0; j < 4; j++) {
                                    T qv[2] = {T(0), T(0)}, mq[2] = {T(0), T(0)};
#pragma unroll
                                    for (int h = 0; h < 2; h++) {
                                        const int c = 2 * j + h;
                                        if (c < P) {
                                            const int cc = c < P ? c : 0;
                                            qv[h] = fma(omf, v[cc], uf * v[cc + 1]) - Tv[cc];
                                            mq[h] = MASKED ? mv[cc] * qv[h] : qv[h];
                                        }
                                    }
                                    sp[j] = mq[0] + mq[1];
                                    ep[j] = fma(mq[0], qv[0], mq[1] * qv[1]);
                                }
                            };
                            if (allv) pairs(std::false_type());
                            else pairs(std::true_type());
                            s0 = (sp[0] + sp[1]) + (sp[2] + sp[3]);
                            e0 = (ep[0] + ep[1]) + (ep[2] + ep[3]);
                        } else if (allv) {
                            // two interleaved chains per sum: half the
                            // dependent adds
#pragma unroll
                            for (int c = 0; c < P; c++) {
                                const T q = fma(omf, v[c], uf * v[c + 1]) - Tv[c];
                                if (c & 1) { s1 += q; e1 = fma(q, q, e1); }
                                else { s0 += q; e0 = fma(q, q, e0); }
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < P; c++) {
                                const T q = fma(omf, v[c], uf * v[c + 1]) - Tv[c];
                                const T mq = mv[c] * q;
                                if (c & 1) { s1 = fma(mv[c], q, s1); e1 = fma(mq, q, e1); }
                                else { s0 = fma(mv[c], q, s0); e0 = fma(mq, q, e0); }
                            }
                        }
                        acc[2 * i] = CAN ? s0 : s0 + s1;
                        acc[2 * i + 1] = CAN ? e0 : e0 + e1;
                    }
                }
                seg_sum_n<SEG, 2 * WN>(acc);
                const T ninv = T(1) / (T)n;
                auto energy = [&](int i) -> T {
                    T E = T(0);
#pragma unroll
                    for (int j = 0; j < WN; j++)
                        if (j == i) E = acc[2 * j + 1] - acc[2 * j] * acc[2 * j] * ninv;
                    return E;
                };
                const T Ec = energy(cw);
                // p = 1 / sum_i exp(-(E_i - E_c) / tau): lane r of the
                // segment evaluates the term of sample r (and r + SEG); the
                // centre term is 1
                T term = 0;
#pragma unroll
                for (int q = 0; q < (WN + SEG - 1) / SEG; q++) {
                    int i = r + q * SEG;
                    if (i < kp.window) term += i == cw ? T(1) : exp(-(energy(i) - Ec) * (T)kp.inv_tau);
                }
                return T(1) / seg_sum<SEG>(term);
            };
            // gamma gate at the final shift: left valid, sample inside the
            // row, both right taps valid (Sec. 3, Sec. 3.2).  With WBATCH its
            // taps are read first, so that they arrive with the window's.
            T uc = fmin(fmax(u, ulo), uhi);
            T ui = floor(uc), uf = uc - ui;
            int xi0 = x0 + (int)ui;
            // taps m = min(xi, W-2) and m + 1 for xi = xi0 .. xi0+P-1
            int m0 = min(max(xi0, 0), W - 2);
            T v[P + 2];
            if constexpr (WBATCH) fetch(m0, v, std::integral_constant<int, P + 2>());
            post = window_post();
            if constexpr (!WBATCH) fetch(m0, v, std::integral_constant<int, P + 2>());
            uint32_t rmask = 0;  // bit j: right tap m0 + j is valid
#pragma unroll
            for (int j = 0; j < P + 2; j++) {
                bool vj;
                if constexpr (U8) vj = v[j] >= (T)kp.vlo && v[j] <= (T)kp.vhi;
                else vj = !signbit(v[j]);
                rmask |= (uint32_t)vj << j;
            }
            // Column c samples x = xi0 + c + uf: inside the row iff
            // 0 <= xi0 + c <= W - 2, or xi0 + c == W - 1 with uf == 0.  Its
            // taps are m0 + m and m0 + m + 1 with m = c + (xi0 - m0) inside,
            // and W - 2 - m0 at the last column.  As bit masks:
            // pairs (bit j: taps j, j + 1 valid) shifted to the columns,
            // cut to the in-row columns, plus the last-column case.
            const uint32_t pairs = rmask & (rmask >> 1);
            const int off = xi0 - m0;
            const uint32_t colpairs = off >= 0 ? (off < 32 ? pairs >> off : 0u) : (-off < 32 ? pairs << -off : 0u);
            const int clo = max(0, -xi0), chi = min(P, W - 1 - xi0);  // columns with 0 <= xi <= W - 2
            uint32_t good = chi > clo ? colpairs & (((1u << (chi - clo)) - 1u) << clo) : 0u;
            const int ce = W - 1 - xi0;  // the column at the last pixel
            if (uf == T(0) && ce >= 0 && ce < P && ((pairs >> ((W - 2 - m0) & 31)) & 1u)) good |= 1u << ce;
            int cnt = __builtin_popcount(vmask & good);
            cnt = seg_sum_i<SEG>(cnt);
            if (cnt < kp.min_valid) {
                status = ST_GATED;
                post = 0;
            }
        }
    }
    if (live && r == 0) {
        static_cast<T *>(J.rec_u)[k] = u;
        static_cast<T *>(J.rec_w)[k] = status == ST_KEPT ? post : T(0);
        J.rec_st[k] = (int8_t)status;
        static_cast<T *>(J.rec_u0)[k] = u0;
    }
}

// OCC: waves per SIMD the register allocation must allow.  3: small launches,
// which may also densify the next coarser level (few blocks, so the waves fit
// anyway); 2: the smallest, whose densification also gathers its first share
// pixel with the taps; 5: launches with many more blocks than the chip
// holds, where occupancy pays -- they never densify, so that code is left out.
template <typename T, int P, bool U8, int WN, int OCC>
__global__ __launch_bounds__(kBlock, OCC) void k_lk(const JobPack<LkJob> pk, KParams kp) {
    __shared__ T Rs[lk_lds_bytes<T, P>() / sizeof(T)];
    // Blocks in launch order (no XCD renumbering): at level 0 the many
    // blocks that stage the same few image lines contend for one L2 when
    // neighbouring patch rows share an XCD; spread over the XCDs they run
    // faster although more lines come from beyond the L2.
    const LkJob &J = pk.j[find_job(pk, (int)blockIdx.x)];
    lk_block<T, P, U8, WN, (OCC < 5), (OCC <= 2)>(J, (int)blockIdx.x - J.block0, kp, Rs);
}

// ---------------------------------------------------------------- densify

// One pixel of a densification job (see dense_value).
template <typename T, bool U8>
__device__ __forceinline__ void dense_pixel(const DenseJob &J, const int i, const KParams &kp) {
    if (J.keep && J.keep[i]) return;
    const int y = div_exact(i, 1.0 / (double)J.W), x = i - y * J.W;
    const T U = dense_value<T, U8>(J, x, y, kp);
    if (J.out) J.out[(size_t)y * J.out_pitch + x] = (float)(-U);
    if (J.U) static_cast<T *>(J.U)[i] = U;
}

// The pixels xs .. xs + strip - 1 of row y, strip = J.strip (the grid
// stride, strips aligned to it).  Where every pixel of the strip has the same
// candidate patches (the interior at most strides), the records of those
// patches are loaded once for the strip; each pixel then takes dense_value's
// fast path with its own spatial weights, in the same order and arithmetic,
// so the values are the same bits.  Other strips, and eq. (2)'s fusion, go
// pixel by pixel through dense_value.
template <typename T, bool U8>
__device__ __forceinline__ void dense_strip(const DenseJob &J, const int xs, const int y, const KParams &kp) {
#pragma clang fp contract(off)
    const int P = J.patch, st = J.stride, xe = min(xs + J.strip, J.W);
    auto put = [&](int x, T U) {
        if (J.out) J.out[(size_t)y * J.out_pitch + x] = (float)(-U);
        if (J.U) static_cast<T *>(J.U)[(size_t)y * J.W + x] = U;
    };
    const double inv_st = 1.0 / (double)st;
    auto range = [&](int v, int n, int cnt, int &lo, int &hi, int &extra) {
        int t = v - P + 1;
        lo = t > 0 ? div_exact(t + st - 1, inv_st) : 0;
        hi = min(cnt - 1, div_exact(v, inv_st));
        extra = (hi < cnt - 1 && v >= n - P) ? cnt - 1 : -1;
    };
    int xlo, xhi, xex, xlo1, xhi1, xex1, ylo, yhi, yex;
    range(xs, J.W, J.nx, xlo, xhi, xex);
    range(xe - 1, J.W, J.nx, xlo1, xhi1, xex1);
    range(y, J.H, J.ny, ylo, yhi, yex);
    const int ncx = xhi - xlo + 1 + (xex >= 0 ? 1 : 0), ncy = yhi - ylo + 1 + (yex >= 0 ? 1 : 0);
    // lo, hi and the snapped extra move monotonically with x (extra as the
    // pair (hi, extra) does), so equal at both ends means equal throughout
    const bool shared = kp.fusion == 0 && xlo == xlo1 && xhi == xhi1 && xex == xex1 && ncx <= 2 && ncy <= 2;
    if (!shared) {
        for (int x = xs; x < xe; x++)
            if (!(J.keep && J.keep[(size_t)y * J.W + x])) put(x, dense_value<T, U8>(J, x, y, kp));
        return;
    }
    const T *rec_u = static_cast<const T *>(J.rec_u);
    const T *rec_w = static_cast<const T *>(J.rec_w);
    const T *gtab = static_cast<const T *>(J.gtab);
    constexpr int NC = 2;
    int px[NC], py[NC], jxc[NC], jyc[NC];
    bool vy[NC];
#pragma unroll
    for (int i = 0; i < NC; i++) {
        jxc[i] = i <= xhi - xlo ? xlo + i : (i == xhi - xlo + 1 ? xex : -1);
        jyc[i] = i <= yhi - ylo ? ylo + i : (i == yhi - ylo + 1 ? yex : -1);
        px[i] = jxc[i] >= 0 ? grid_pos(jxc[i], J.W, P, st) : 0;
        py[i] = jyc[i] >= 0 ? grid_pos(jyc[i], J.H, P, st) : 0;
        vy[i] = jyc[i] >= 0 && y >= py[i] && y < py[i] + P;
    }
    // records of the (at most) 2 x 2 candidates, loaded once
    T wk[NC][NC], uk[NC][NC];
#pragma unroll
    for (int iy = 0; iy < NC; iy++)
#pragma unroll
        for (int ix = 0; ix < NC; ix++) {
            const bool v = vy[iy] && jxc[ix] >= 0;
            const int k = v ? jyc[iy] * J.nx + jxc[ix] : 0;
            wk[iy][ix] = rec_w[k];
            uk[iy][ix] = rec_u[k];
            if (!v) wk[iy][ix] = T(0);
        }
    for (int x = xs; x < xe; x++) {
        if (J.keep && J.keep[(size_t)y * J.W + x]) continue;
        // fallback taps loaded with the spatial weights, mixed at the end
        T f00 = 0, f01 = 0, f10 = 0, f11 = 0, ffx = 0, ffy = 0;
        if (J.mode == 0) {
            const T *Uc = static_cast<const T *>(J.Uc);
            int mx, my, mx1, my1;
            bilinear_taps<T>(J.Wc, J.Hc, T(0.5) * (T)x, T(0.5) * (T)y, mx, my, mx1, my1, ffx, ffy);
            f00 = Uc[(size_t)my * J.Wc + mx];
            f01 = Uc[(size_t)my * J.Wc + mx1];
            f10 = Uc[(size_t)my1 * J.Wc + mx];
            f11 = Uc[(size_t)my1 * J.Wc + mx1];
        }
        bool vx[NC];
        T g[NC][NC];
#pragma unroll
        for (int ix = 0; ix < NC; ix++) vx[ix] = jxc[ix] >= 0 && x >= px[ix] && x < px[ix] + P;
#pragma unroll
        for (int iy = 0; iy < NC; iy++)
#pragma unroll
            for (int ix = 0; ix < NC; ix++)
                g[iy][ix] = gtab[vy[iy] && vx[ix] ? (y - py[iy]) * P + (x - px[ix]) : 0];
        T A = 0, B = 0;
#pragma unroll
        for (int iy = 0; iy < NC; iy++)
#pragma unroll
            for (int ix = 0; ix < NC; ix++) {
                const T w0 = vx[ix] ? wk[iy][ix] : T(0);
                if (w0 > T(0)) {
                    const T w = w0 * g[iy][ix];
                    A += w;
                    B += w * uk[iy][ix];
                }
            }
        T U;
        if (A > T(0)) U = B / A;
        else if (J.mode == 2) U = (T)__builtin_nan("");
        else if (J.mode == 1) U = 0;
        else U = T(2) * bilinear_mix<T>(f00, f01, f10, f11, ffx, ffy);
        put(x, U);
    }
}

__host__ __device__ constexpr int dense_blocks(int w, int h, int ppt) {
    return (w * h + kBlock * ppt - 1) / (kBlock * ppt);
}
// Blocks of a densification job: one pixel per thread (ppt per thread in the
// persistent kernel's tasks), or one strip per thread.
__host__ __device__ constexpr int dense_job_blocks(const DenseJob &j) {
    return j.strip > 1 ? ((j.W + j.strip - 1) / j.strip * j.H + kBlock - 1) / kBlock : dense_blocks(j.W, j.H, j.ppt);
}

template <typename T, bool U8>
__device__ __forceinline__ void dense_block(const DenseJob &J, int lb, const KParams &kp) {
    if (J.strip > 1) {
        const int nsr = (J.W + J.strip - 1) / J.strip;
        const int s = lb * kBlock + (int)threadIdx.x;
        if (s >= nsr * J.H) return;
        const int y = div_exact(s, 1.0 / (double)nsr), xs = (s - y * nsr) * J.strip;
        dense_strip<T, U8>(J, xs, y, kp);
        return;
    }
    const int n = J.W * J.H;
    for (int q = 0; q < J.ppt; q++) {
        int i = (lb * J.ppt + q) * kBlock + (int)threadIdx.x;
        if (i < n) dense_pixel<T, U8>(J, i, kp);
    }
}

template <typename T, bool U8>
__global__ __launch_bounds__(kBlock) void k_dense(const JobPack<DenseJob> pk, KParams kp) {
    const int bid = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const DenseJob &J = pk.j[find_job(pk, bid)];
    dense_block<T, U8>(J, bid - J.block0, kp);
}

// ---------------------------------------------------------------- learned init

// Network input for one pyramid pixel: (L - 128)/64, (R - 128)/64, then
// |L(x) - R(x - d)| / 64 for d = 0..13 (R's column clamped), in the
// arithmetic type, rounded to bfloat16 through float.
__device__ inline uint16_t to_bf16(double v) {
    float f = (float)v;
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int kNetIn = 16;
constexpr int kNetDisp = kNetIn - 2;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_net_input(const JobPack<NetInJob> pk) {
    const NetInJob &J = pk.j[find_job(pk, (int)blockIdx.x)];
    const int i = ((int)blockIdx.x - J.block0) * kBlock + (int)threadIdx.x;
    if (i >= J.W * J.H) return;
    const int y = i / J.W, x = i - y * J.W;
    const T *L = static_cast<const T *>(J.L), *R = static_cast<const T *>(J.R);
    const double lv = (double)fabs(L[i]), rv = (double)fabs(R[i]);
    uint16_t *o = J.x + (size_t)i * kNetIn;
    o[0] = to_bf16((lv - 128.0) / 64.0);
    o[1] = to_bf16((rv - 128.0) / 64.0);
    for (int d = 0; d < kNetDisp; d++) {
        const int xs = x - d < 0 ? 0 : x - d;
        o[2 + d] = to_bf16(fabs(lv - (double)fabs(R[(size_t)y * J.W + xs])) / 64.0);
    }
}

// Bilinear read of channel ch of an interleaved 2-channel FP32 map, in the
// arithmetic type, coordinates clamped; SIG applies the logistic function to
// the four taps first.
template <typename T, bool SIG>
__device__ inline T bilinear2(const float *F, int W, int H, int ch, T X, T Y) {
    X = fmin(fmax(X, T(0)), (T)(W - 1));
    Y = fmin(fmax(Y, T(0)), (T)(H - 1));
    int mx = min(max((int)floor(X), 0), max(W - 2, 0));
    int my = min(max((int)floor(Y), 0), max(H - 2, 0));
    T fx = W > 1 ? X - (T)mx : T(0), fy = H > 1 ? Y - (T)my : T(0);
    int mx1 = W > 1 ? mx + 1 : mx, my1 = H > 1 ? my + 1 : my;
    auto at = [&](int yy, int xx) {
        T v = (T)F[((size_t)yy * W + xx) * 2 + ch];
        return SIG ? T(1) / (T(1) + exp(-v)) : v;
    };
    T a = (T(1) - fx) * at(my, mx) + fx * at(my, mx1);
    T b = (T(1) - fx) * at(my1, mx) + fx * at(my1, mx1);
    return (T(1) - fy) * a + fy * b;
}

// Learned field at the injection level: u = sd * disparity(x * sxy) and
// keep = confidence(x * sxy) >= thr, in the arithmetic type (sxy and sd are
// powers of two, exact in either).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gate(const JobPack<GateJob> pk) {
    const GateJob &J = pk.j[find_job(pk, (int)blockIdx.x)];
    const int i = ((int)blockIdx.x - J.block0) * kBlock + (int)threadIdx.x;
    if (i >= J.Wi * J.Hi) return;
    const int y = i / J.Wi, x = i - y * J.Wi;
    const T X = (T)x * (T)J.sxy, Y = (T)y * (T)J.sxy;
    const T d = bilinear2<T, false>(J.net, J.W4, J.H4, 0, X, Y);
    const T c = bilinear2<T, true>(J.net, J.W4, J.H4, 1, X, Y);
    static_cast<T *>(J.U)[i] = (T)J.sd * d;
    J.keep[i] = c >= (T)J.thr ? 1 : 0;
}

}  // namespace bdis
