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
