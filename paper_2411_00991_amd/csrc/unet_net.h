// unet_net.h -- what the sampler runtime uses of a bdc_unet (same library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/bdc_unet.h"

namespace bdc {
namespace unet {

// Forward pass of a device batch on stream st; *out_dev points at the
// network's own [B][h][w][2] output buffer (valid until its next call).
bdc_status net_forward_on(bdc_unet* u, const float* x_dev, int B, int h, int w, float** out_dev, hipStream_t st,
                          std::string* err);
int net_levels(const bdc_unet* u);
int64_t net_max_pixels(const bdc_unet* u);

}  // namespace unet
}  // namespace bdc
