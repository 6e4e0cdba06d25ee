// bdisnet_internal.hpp -- what the stereo runtime uses of the proposal
// network across translation units (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdis.h"

namespace bdisnet {

// Forward of x (NHWC bfloat16, 16 channels, n images of hh x ww) into out
// (NHWC FP32, 2 channels); acts[1..3] receive the hidden activations
// (channels(h) bfloat16 channels each, n * hh * ww pixels).
bdis_status forward_internal(bdisnet_t *h, const uint16_t *x, int n, int hh, int ww, float *out,
                             uint16_t *const *acts, hipStream_t s);
size_t act_bytes(const bdisnet_t *h, size_t pixels);
int channels(const bdisnet_t *h);
int device_of(const bdisnet_t *h);

}  // namespace bdisnet

namespace bdisnet {

// The network's inference for the stereo path in one launch (input channels
// and the four layers, per spatial tile): one job per pair.
struct FusedJob {
    const void *L, *R;  // the pair's 1/16 pyramid level (arithmetic type, sign bit = invalid)
    float *out;         // network output, H x W x 2 FP32 (disparity, confidence logit)
    int W, H;           // size of the 1/16 level
    int tiles_x;        // output tiles per row
    int block0;         // first block of this job in its launch
};
static_assert(sizeof(FusedJob) == 3 * 8 + 4 * 4, "FusedJob must have no padding");
constexpr int kFusedCap = 96;
struct FusedPack {
    int n;
    int pad_;
    FusedJob j[kFusedCap];
};
// Output tile of the fused forward, and its blocks for one W x H image.
constexpr int kFTX = 16, kFTY = 8;
inline int fused_tiles_x(int W) { return (W + kFTX - 1) / kFTX; }
inline int fused_blocks(int W, int H) { return fused_tiles_x(W) * ((H + kFTY - 1) / kFTY); }
// Enqueues the fused forward of the jobs of pk (`blocks` in all) on s;
// f64: the pyramid holds doubles (else floats).
bdis_status forward_fused(bdisnet_t *h, const FusedPack &pk, int blocks, bool f64, hipStream_t s);

}  // namespace bdisnet
