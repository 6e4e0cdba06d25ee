// bdisnet_fused.hpp -- the proposal network's inference for the stereo path
// in one kernel: per output tile of kFTX x kFTY pixels at the 1/16 level, a
// workgroup builds the 16 input channels of the tile plus a 4-pixel halo
// from the pyramid, then runs the four 3x3 layers through LDS, each layer on
// a region one pixel smaller on every side, and writes the 2-channel FP32
// output of the tile.  Activations between layers are bfloat16, as in the
// layer-by-layer kernels; out-of-image positions hold 0 at every layer (the
// convolutions' zero padding).
//
// Matrix cores: v_mfma_f32_16x16x32_bf16 (gfx950), one implicit GEMM per
// layer with M = 16 region pixels, N = 16 output channels and K = 32 of the
// 9 x C_in (tap, channel) products.  Lane l holds A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] (j = 0..7) and gets D[4 (l / 16) + j][l % 16]
// (j = 0..3).  Since C_in is a multiple of 8, a lane's 8 K entries are 8
// consecutive channels of one tap: one 16-byte LDS read.  A layer's B
// fragments are loaded into registers once per wave; the wave then walks
// its share of the region's 16-pixel tiles reading only A from LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdisnet_internal.hpp"
#include "bdisnet_kernels.hpp"

namespace bdisnet {

typedef short s8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ inline f4_t mfma32(s8_t a, s8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c, 0,
                                                   0, 0);
}

// K chunks of 32 and N tiles of 16 of a layer
template <int CI> struct KChunks { static constexpr int value = (9 * CI + 31) / 32; };
template <int CO> struct NTiles { static constexpr int value = (CO + 15) / 16; };

// LDS pixel strides in bfloat16 elements (8 of padding: 16-byte reads of 16
// consecutive pixels then cover distinct banks)
constexpr int kS0 = 16 + 8;
template <int C> struct HStride { static constexpr int value = C + 8; };

// One layer over an output region of WO x HO pixels whose input region (one
// pixel larger on every side, width WO + 2) is `in`.  Region pixel (r, c) is
// image pixel (gx0 + c, gy0 + r).  Hidden layers: ReLU, bfloat16 into `outl`
// (stride SO), 0 outside the image.  Last layer: FP32 into the image output
// `gout` (W x H x 2) for the region's pixels inside the image.
template <int CI, int SI, int CO, int SO, int WO, int HO, bool LAST>
__device__ __forceinline__ void fused_layer(const uint16_t *__restrict__ in, uint16_t *__restrict__ outl,
                                            const uint16_t *__restrict__ frag, const float *__restrict__ bias,
                                            int gx0, int gy0, int W, int H, float *__restrict__ gout) {
    constexpr int NQ = KChunks<CI>::value, NT = NTiles<CO>::value;
    constexpr int NPX = WO * HO, NMT = (NPX + 15) / 16, WI = WO + 2;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6, grp = lane >> 4;
    s8_t B[NQ][NT];
#pragma unroll
    for (int q = 0; q < NQ; q++)
#pragma unroll
        for (int t = 0; t < NT; t++)
            B[q][t] = *reinterpret_cast<const s8_t *>(frag + ((size_t)(q * NT + t) * 64 + lane) * 8);
    // this lane's (tap, first channel) of every K chunk: 8 consecutive
    // channels of one tap; entries past the 9 taps meet zero weights
    int aoff[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        const int k0 = 32 * q + 8 * grp;
        const int tap = k0 / CI < 9 ? k0 / CI : 8;
        const int ci0 = k0 / CI < 9 ? k0 - (k0 / CI) * CI : 0;
        aoff[q] = ((tap / 3) * WI + tap % 3) * SI + ci0;
    }
    float bv[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) {
        const int co = 16 * t + (lane & 15);
        bv[t] = co < CO ? bias[co] : 0.f;
    }
    for (int mt = wave; mt < NMT; mt += kBlock / 64) {
        const int m = min(mt * 16 + (lane & 15), NPX - 1);
        const int r = m / WO, c = m - r * WO;
        const uint16_t *base = in + (size_t)(r * WI + c) * SI;
        f4_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; t++) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const s8_t a = *reinterpret_cast<const s8_t *>(base + aoff[q]);
#pragma unroll
            for (int t = 0; t < NT; t++) acc[t] = mfma32(a, B[q][t], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; t++) {
            const int co = 16 * t + (lane & 15);
            if (co >= CO) continue;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int mo = mt * 16 + 4 * grp + j;
                if (mo >= NPX) continue;
                const int ro = mo / WO, cc = mo - ro * WO;
                const int gx = gx0 + cc, gy = gy0 + ro;
                const bool inside = gx >= 0 && gx < W && gy >= 0 && gy < H;
                const float v = acc[t][j] + bv[t];
                if constexpr (LAST) {
                    if (inside) gout[((size_t)gy * W + gx) * 2 + co] = v;
                } else {
                    outl[(size_t)mo * SO + co] = inside ? f2bf(v > 0.f ? v : 0.f) : (uint16_t)0;
                }
            }
        }
    }
}

// LDS elements (bfloat16) of the fused forward: buffer X holds regions 0 and
// 2, buffer Y regions 1 and 3.
template <int C>
__host__ __device__ constexpr int fused_x_elems() {
    return ((kFTX + 8) * (kFTY + 8) * kS0 > (kFTX + 4) * (kFTY + 4) * HStride<C>::value)
               ? (kFTX + 8) * (kFTY + 8) * kS0
               : (kFTX + 4) * (kFTY + 4) * HStride<C>::value;
}
template <int C>
__host__ __device__ constexpr int fused_y_elems() {
    return (kFTX + 6) * (kFTY + 6) * HStride<C>::value;
}

// Input channels of one 1/16-level pixel, as the network-input kernel of the
// stereo path computes them: (L - 128)/64, (R - 128)/64, |L(x) - R(x - d)|/64
// for d = 0..13 (R's column clamped at 0), in double, rounded to bfloat16
// through float.
template <typename T>
__device__ __forceinline__ void input_channels(const T *L, const T *R, int W, int x, int y, uint16_t *v) {
    const size_t row = (size_t)y * W;
    const double lv = (double)fabs(L[row + x]), rv = (double)fabs(R[row + x]);
    v[0] = f2bf((float)((lv - 128.0) / 64.0));
    v[1] = f2bf((float)((rv - 128.0) / 64.0));
#pragma unroll
    for (int d = 0; d < 14; d++) {
        const int xs = x - d < 0 ? 0 : x - d;
        v[2 + d] = f2bf((float)(fabs(lv - (double)fabs(R[row + xs])) / 64.0));
    }
}

template <typename T, int C>
__global__ __launch_bounds__(kBlock, (C <= 32 ? 2 : 1)) void k_net_fused(
    const FusedPack pk, const uint16_t *__restrict__ f0, const uint16_t *__restrict__ f1,
    const uint16_t *__restrict__ f2, const uint16_t *__restrict__ f3, const float *__restrict__ b0,
    const float *__restrict__ b1, const float *__restrict__ b2, const float *__restrict__ b3) {
    extern __shared__ __align__(16) uint16_t lds[];
    constexpr int SC = HStride<C>::value;
    constexpr int W0 = kFTX + 8, H0 = kFTY + 8;
    uint16_t *X = lds, *Y = lds + fused_x_elems<C>();
    int lo = 0, hi = pk.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pk.j[mid].block0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const FusedJob &J = pk.j[lo];
    const int lb = (int)blockIdx.x - J.block0;
    const int ty = lb / J.tiles_x, tx = lb - ty * J.tiles_x;
    const int ox = tx * kFTX, oy = ty * kFTY;
    const T *L = static_cast<const T *>(J.L), *R = static_cast<const T *>(J.R);
    // region 0: the input channels, 0 outside the image
    for (int p = (int)threadIdx.x; p < W0 * H0; p += kBlock) {
        const int r = p / W0, c = p - r * W0;
        const int x = ox - 4 + c, y = oy - 4 + r;
        uint16_t v[16];
        if (x >= 0 && x < J.W && y >= 0 && y < J.H) {
            input_channels<T>(L, R, J.W, x, y, v);
        } else {
#pragma unroll
            for (int k = 0; k < 16; k++) v[k] = 0;
        }
        s8_t lo8, hi8;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            lo8[k] = (short)v[k];
            hi8[k] = (short)v[8 + k];
        }
        *reinterpret_cast<s8_t *>(X + (size_t)p * kS0) = lo8;
        *reinterpret_cast<s8_t *>(X + (size_t)p * kS0 + 8) = hi8;
    }
    __syncthreads();
    fused_layer<16, kS0, C, SC, kFTX + 6, kFTY + 6, false>(X, Y, f0, b0, ox - 3, oy - 3, J.W, J.H, nullptr);
    __syncthreads();
    fused_layer<C, SC, C, SC, kFTX + 4, kFTY + 4, false>(Y, X, f1, b1, ox - 2, oy - 2, J.W, J.H, nullptr);
    __syncthreads();
    fused_layer<C, SC, C, SC, kFTX + 2, kFTY + 2, false>(X, Y, f2, b2, ox - 1, oy - 1, J.W, J.H, nullptr);
    __syncthreads();
    fused_layer<C, SC, 2, 1, kFTX, kFTY, true>(Y, nullptr, f3, b3, ox, oy, J.W, J.H, J.out);
}

// B fragments of one layer for mfma32 from the FP32 master weights
// [tap][ci][co]: frag[((q * NT + t) * 64 + l) * 8 + j] = w of K index
// k = 32 q + 8 (l / 16) + j (tap k / CI, channel k % CI) and output channel
// 16 t + l % 16; zero past the 9 taps or the CO channels.
__global__ void k_pack32(const float *__restrict__ w, int CI, int CO, uint16_t *__restrict__ frag) {
    const int NQ = (9 * CI + 31) / 32, NT = (CO + 15) / 16;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= NQ * NT * 64 * 8) return;
    const int j = i & 7, l = (i >> 3) & 63, qt = i >> 9;
    const int t = qt % NT, q = qt / NT;
    const int k = 32 * q + 8 * (l >> 4) + j, tap = k / CI, ci = k - tap * CI, co = 16 * t + (l & 15);
    frag[i] = (tap < 9 && co < CO) ? f2bf(w[((size_t)tap * CI + ci) * CO + co]) : (uint16_t)0;
}

}  // namespace bdisnet
