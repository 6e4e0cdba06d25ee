// bdis_geometry.hpp -- the steps on either side of the matcher: rectifying
// and undistorting the raw images before it, and turning its disparity into
// depth after it.  Paper (arXiv 2106.07136): Sec. 1 (stereo under the
// pinhole camera model with rectification and undistortion before
// disparity estimation), Sec. 3 (the data are rectified and undistorted from
// their calibration), Sec. 3.2 (depth errors in mm; undistortion leaves
// invalid pixels at the image edges).  The lens model is the standard
// radial-tangential (Brown-Conrady) one.
//
// Both kernels recompute everything per pixel instead of reading a stored
// map: the source position costs about 40 FP64 operations, while a stored
// FP64 map would cost 16 bytes of HBM traffic per pixel (an FP32 map is not
// precise enough to round the interpolated gray level like the FP64
// definition does).
#pragma once
#include <hip/hip_runtime.h>

#include "bdis.h"
#include "bdis_kernels.hpp"

namespace bdis {

constexpr int kMaxRectifyJobs = 8;
constexpr int kRectPx = 4;  // output pixels per thread (one 32-bit store when aligned)

struct RectifyPack {
    int n;
    int blocks[kMaxRectifyJobs + 1];  // first block of each job, then the total
    bdis_rectify_job j[kMaxRectifyJobs];
};
static_assert(sizeof(bdis_rectify_job) == 2 * 8 + 6 * 4 + 22 * 8, "bdis_rectify_job has no padding");
static_assert(sizeof(RectifyPack) <= 4000, "rectify job pack too large for the kernel arguments");

// Raw-image position of rectified pixel (u, v): the rectified ray, rotated
// back into the raw camera frame (R^T), projected, moved by the lens
// (radial k1..k3, tangential p1, p2), mapped by the raw camera matrix.
// Contraction stays off so every operation rounds on its own, as written.
__device__ __forceinline__ void source_xy(const bdis_camera &c, double u, double v, double &xs, double &ys) {
#pragma clang fp contract(off)
    const double a = (u - c.ncx) / c.nfx, b = (v - c.ncy) / c.nfy;
    const double X = c.R[0] * a + c.R[3] * b + c.R[6];
    const double Y = c.R[1] * a + c.R[4] * b + c.R[7];
    const double Z = c.R[2] * a + c.R[5] * b + c.R[8];
    const double x = X / Z, y = Y / Z;
    const double r2 = x * x + y * y;
    const double radial = 1.0 + c.k1 * r2 + c.k2 * r2 * r2 + c.k3 * r2 * r2 * r2;
    const double xd = x * radial + 2.0 * c.p1 * x * y + c.p2 * (r2 + 2.0 * x * x);
    const double yd = y * radial + c.p1 * (r2 + 2.0 * y * y) + 2.0 * c.p2 * x * y;
    xs = c.fx * xd + c.cx;
    ys = c.fy * yd + c.cy;
}

// Bilinear gray level at (xs, ys), rounded half up; 0 (below the validity
// band, so the matcher ignores the pixel) outside the raw image.
__device__ __forceinline__ uint32_t sample_u8(const bdis_rectify_job &J, double xs, double ys) {
#pragma clang fp contract(off)
    const int sw = J.src_width, sh = J.src_height;
    if (!(xs >= 0.0 && ys >= 0.0 && xs <= (double)(sw - 1) && ys <= (double)(sh - 1))) return 0u;
    int mx = (int)floor(xs), my = (int)floor(ys);
    mx = max(min(mx, sw - 2), 0);
    my = max(min(my, sh - 2), 0);
    const double fx = sw > 1 ? xs - (double)mx : 0.0, fy = sh > 1 ? ys - (double)my : 0.0;
    const int mx1 = sw > 1 ? mx + 1 : mx, my1 = sh > 1 ? my + 1 : my;
    const uint8_t *r0 = J.src + (size_t)my * J.src_pitch, *r1 = J.src + (size_t)my1 * J.src_pitch;
    const double top = (1.0 - fx) * (double)r0[mx] + fx * (double)r0[mx1];
    const double bot = (1.0 - fx) * (double)r1[mx] + fx * (double)r1[mx1];
    const double val = (1.0 - fy) * top + fy * bot;
    const double q = floor(val + 0.5);
    return (uint32_t)(q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q));
}

// One thread: kRectPx consecutive pixels of one output row.  Blocks are
// renumbered so that each XCD takes a contiguous band of rows (their source
// rows overlap, and each XCD has its own L2).
__global__ __launch_bounds__(kBlock) void k_rectify(const RectifyPack pk) {
    const int bid = xcd_block((int)blockIdx.x, (int)gridDim.x);
    int ji = 0;
    while (ji + 1 < pk.n && pk.blocks[ji + 1] <= bid) ji++;
    const bdis_rectify_job &J = pk.j[ji];
    const int per_row = (J.dst_width + kRectPx - 1) / kRectPx;
    const int t = (bid - pk.blocks[ji]) * kBlock + (int)threadIdx.x;
    if (t >= per_row * J.dst_height) return;
    const int v = t / per_row, u0 = (t - v * per_row) * kRectPx;
    uint8_t *row = J.dst + (size_t)v * J.dst_pitch;
    uint32_t px[kRectPx];
#pragma unroll
    for (int k = 0; k < kRectPx; k++) {
        px[k] = 0u;
        if (u0 + k < J.dst_width) {
            double xs, ys;
            source_xy(J.cam, (double)(u0 + k), (double)v, xs, ys);
            px[k] = sample_u8(J, xs, ys);
        }
    }
    if (u0 + kRectPx <= J.dst_width && ((reinterpret_cast<uintptr_t>(row + u0) & 3u) == 0)) {
        *reinterpret_cast<uint32_t *>(row + u0) = px[0] | (px[1] << 8) | (px[2] << 16) | (px[3] << 24);
    } else {
#pragma unroll
        for (int k = 0; k < kRectPx; k++)
            if (u0 + k < J.dst_width) row[u0 + k] = (uint8_t)px[k];
    }
}

// Z = f B / d in FP64, stored as float; NaN where d is NaN or <= d_min.
// One thread per pixel of a row-major grid (pitches in elements).
__global__ __launch_bounds__(kBlock) void k_depth(const float *__restrict__ disp, int W, int H, int dpitch,
                                                        double fB, float d_min, float *__restrict__ depth,
                                                        int zpitch) {
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    if (i >= W * H) return;
    const int y = i / W, x = i - y * W;
    const float d = disp[(size_t)y * dpitch + x];
    const bool ok = isfinite(d) && d > d_min;
    depth[(size_t)y * zpitch + x] = ok ? (float)(fB / (double)d) : __builtin_nanf("");
}

}  // namespace bdis
