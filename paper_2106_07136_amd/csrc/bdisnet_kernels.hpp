// bdisnet_kernels.hpp -- gfx950 kernels of the learned proposal network.
//
// The network is an added serving pattern, not part of the paper's method:
// four 3x3 convolutions (ReLU between them) on the 1/16 pyramid level that
// predict a coarse disparity and a confidence logit.  Activations are NHWC
// bfloat16, weights bfloat16, every product accumulates in FP32 on the
// matrix cores: each convolution is an implicit GEMM with M = pixels,
// N = output channels and K = 9 taps x input channels, one
// v_mfma_f32_16x16x16_bf16 per 16-channel slice of one tap.
//
// Operand layout of v_mfma_f32_16x16x16bf16_1k (wave64), lane l:
//   A (16 x 16, M x K): A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, K x N): B[4 (l / 16) + j][l % 16]
//   D (16 x 16, M x N): D[4 (l / 16) + j][l % 16]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdisnet {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;  // 4 waves

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__device__ inline f4_t mfma16(s4_t a, s4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Image geometry of a convolution launch: N images of H x W pixels.
struct Geo {
    int N, H, W;
    int M;  // N * H * W
};

__device__ inline void pix_coords(const Geo &g, int m, int &n, int &y, int &x) {
    int hw = g.H * g.W;
    n = m / hw;
    int r = m - n * hw;
    y = r / g.W;
    x = r - y * g.W;
}

// 4 consecutive bf16 (8 bytes) at element offset e of a bf16 array
__device__ inline s4_t load4(const uint16_t *p, size_t e) {
    return *reinterpret_cast<const s4_t *>(p + e);
}

// Weight fragments: for tap t, K-chunk kc and N-tile nt, the 64 lanes' B
// operands, 4 bf16 each, contiguous: frag[((t * KC + kc) * NT + nt) * 256 + l * 4 + j].
__device__ inline s4_t load_frag(const uint16_t *frag, int t, int kc, int nt, int KC, int NT, int lane) {
    return load4(frag, (size_t)((t * KC + kc) * NT + nt) * 256 + (size_t)lane * 4);
}

// ---------------------------------------------------------------- forward

// y[m][co] = b[co] + sum_{tap, ci} x[m + tap][ci] w[tap][ci][co], ReLU unless
// the last layer; hidden outputs bfloat16 with CO channels, the last layer
// FP32 with 2 channels.  One wave: 16 pixels x all output channels.
template <int CI, int CO, bool LAST>
__global__ __launch_bounds__(kBlock) void k_conv_fwd(Geo g, const uint16_t *__restrict__ x,
                                                      const uint16_t *__restrict__ wfrag,
                                                      const float *__restrict__ bias,
                                                      uint16_t *__restrict__ y_bf, float *__restrict__ y_f) {
    constexpr int KC = CI / 16;
    constexpr int NT = (CO + 15) / 16;
    const int lane = (int)threadIdx.x & 63;
    const int m0 = ((int)blockIdx.x * (kBlock / 64) + (int)threadIdx.x / 64) * 16;
    if (m0 >= g.M) return;  // whole wave out of range (uniform per wave)
    const int mr = m0 + (lane & 15);  // A row of this lane
    int n, yy, xx;
    pix_coords(g, mr < g.M ? mr : g.M - 1, n, yy, xx);
    const bool rok = mr < g.M;
    f4_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        const int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
        const bool in = rok && sy >= 0 && sy < g.H && sx >= 0 && sx < g.W;
        const size_t base = (((size_t)n * g.H + (in ? sy : 0)) * g.W + (in ? sx : 0)) * CI;
#pragma unroll
        for (int kc = 0; kc < KC; kc++) {
            s4_t a = in ? load4(x, base + kc * 16 + (lane >> 4) * 4) : s4_t{0, 0, 0, 0};
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                acc[nt] = mfma16(a, load_frag(wfrag, tap, kc, nt, KC, NT, lane), acc[nt]);
        }
    }
    const int col = lane & 15;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const int co = nt * 16 + col;
        if (co >= CO) continue;
        const float bv = bias[co];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int m = m0 + (lane >> 4) * 4 + j;
            if (m >= g.M) continue;
            float v = acc[nt][j] + bv;
            if constexpr (LAST) {
                y_f[(size_t)m * CO + co] = v;
            } else {
                v = v > 0.f ? v : 0.f;
                y_bf[(size_t)m * CO + co] = f2bf(v);
            }
        }
    }
}

// ---------------------------------------------------------------- input gradient

// gx[m][ci] = sum_{tap, co} gz[m - tap][co] w[tap][ci][co] (gz zero outside the
// image), then masked by the ReLU of the layer input (x > 0) and rounded to
// bfloat16: the gradient at the previous layer's pre-activation.  gz has
// COP = 16 * ceil(CO / 16) channels (zero padded).
template <int CI, int CO>
__global__ __launch_bounds__(kBlock) void k_conv_dgrad(Geo g, const uint16_t *__restrict__ gz,
                                                        const uint16_t *__restrict__ wtfrag,
                                                        const uint16_t *__restrict__ x,
                                                        uint16_t *__restrict__ gzprev) {
    constexpr int COP = 16 * ((CO + 15) / 16);
    constexpr int KC = COP / 16;
    constexpr int NT = CI / 16;
    const int lane = (int)threadIdx.x & 63;
    const int m0 = ((int)blockIdx.x * (kBlock / 64) + (int)threadIdx.x / 64) * 16;
    if (m0 >= g.M) return;
    const int mr = m0 + (lane & 15);
    int n, yy, xx;
    pix_coords(g, mr < g.M ? mr : g.M - 1, n, yy, xx);
    const bool rok = mr < g.M;
    f4_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
        const int sy = yy - (tap / 3 - 1), sx = xx - (tap % 3 - 1);
        const bool in = rok && sy >= 0 && sy < g.H && sx >= 0 && sx < g.W;
        const size_t base = (((size_t)n * g.H + (in ? sy : 0)) * g.W + (in ? sx : 0)) * COP;
#pragma unroll
        for (int kc = 0; kc < KC; kc++) {
            s4_t a = in ? load4(gz, base + kc * 16 + (lane >> 4) * 4) : s4_t{0, 0, 0, 0};
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                acc[nt] = mfma16(a, load_frag(wtfrag, tap, kc, nt, KC, NT, lane), acc[nt]);
        }
    }
    const int col = lane & 15;
#pragma unroll
    for (int nt = 0; nt < NT; nt++) {
        const int ci = nt * 16 + col;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int m = m0 + (lane >> 4) * 4 + j;
            if (m >= g.M) continue;
            const float xv = bf2f(x[(size_t)m * CI + ci]);
            gzprev[(size_t)m * CI + ci] = f2bf(xv > 0.f ? acc[nt][j] : 0.f);
        }
    }
}

// ---------------------------------------------------------------- weight gradient

// Partial weight and bias gradients of one chunk of kWChunk pixels:
//   gw[tap][ci][co] = sum_m x[m + tap][ci] gz[m][co],  gb[co] = sum_m gz[m][co]
// Tile (tap, ci-tile, co-tile) per wave iteration: rows ci, columns co,
// K = 16 pixels per instruction.  part: [chunk][9 * CI * COP + COP] floats.
constexpr int kWChunk = 256;

template <int CI, int CO>
__global__ __launch_bounds__(kBlock) void k_conv_wgrad(Geo g, const uint16_t *__restrict__ x,
                                                        const uint16_t *__restrict__ gz,
                                                        float *__restrict__ part) {
    constexpr int COP = 16 * ((CO + 15) / 16);
    constexpr int CT = CI / 16, OT = COP / 16;
    constexpr int NTILE = 9 * CT * OT;
    constexpr int PSZ = 9 * CI * COP + COP;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x / 64;
    const int chunk = (int)blockIdx.x;
    const int p0 = chunk * kWChunk;
    float *out = part + (size_t)chunk * PSZ;
    for (int tile = wave; tile < NTILE; tile += kBlock / 64) {
        const int tap = tile / (CT * OT);
        const int ct = (tile / OT) % CT, ot = tile % OT;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        f4_t acc = f4_t{0.f, 0.f, 0.f, 0.f};
        for (int k0 = p0; k0 < p0 + kWChunk && k0 < g.M; k0 += 16) {
            short av[4], bv[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int m = k0 + (lane >> 4) * 4 + j;
                av[j] = 0;
                bv[j] = 0;
                if (m < g.M) {
                    int n, yy, xx;
                    pix_coords(g, m, n, yy, xx);
                    const int sy = yy + dy, sx = xx + dx;
                    if (sy >= 0 && sy < g.H && sx >= 0 && sx < g.W)
                        av[j] = (short)x[(((size_t)n * g.H + sy) * g.W + sx) * CI + ct * 16 + (lane & 15)];
                    bv[j] = (short)gz[(size_t)m * COP + ot * 16 + (lane & 15)];
                }
            }
            // A[row = ci][k = pixel]: lane holds row lane % 16, pixels 4 (lane / 16) + j
            acc = mfma16(s4_t{av[0], av[1], av[2], av[3]}, s4_t{bv[0], bv[1], bv[2], bv[3]}, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int ci = ct * 16 + (lane >> 4) * 4 + j;
            const int co = ot * 16 + (lane & 15);
            out[((size_t)tap * CI + ci) * COP + co] = acc[j];
        }
    }
    // bias: one column per thread over the chunk
    for (int co = (int)threadIdx.x; co < COP; co += kBlock) {
        float s = 0.f;
        for (int m = p0; m < p0 + kWChunk && m < g.M; m++) s += bf2f(gz[(size_t)m * COP + co]);
        out[9 * CI * COP + co] = s;
    }
}

// Sums the chunk partials in chunk order (deterministic) into the flat
// gradient of one layer: [tap][ci][co] (co < CO) then [co].
template <int CI, int CO>
__global__ __launch_bounds__(kBlock) void k_wgrad_reduce(const float *__restrict__ part, int nchunk,
                                                          float *__restrict__ grad) {
    constexpr int COP = 16 * ((CO + 15) / 16);
    constexpr int PSZ = 9 * CI * COP + COP;
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    const int nw = 9 * CI * CO;
    if (i >= nw + CO) return;
    int src;
    if (i < nw) {
        const int co = i % CO, r = i / CO;  // r = tap * CI + ci
        src = r * COP + co;
    } else {
        src = 9 * CI * COP + (i - nw);
    }
    float s = 0.f;
    for (int c = 0; c < nchunk; c++) s += part[(size_t)c * PSZ + src];
    grad[i] = s;
}

}  // namespace bdisnet
