// bdc_consts.h -- sizes shared by the kernels and the host runtime.
#pragma once

namespace bdc {

constexpr int WG = 256;            // threads per workgroup of the sweep kernels
constexpr int XCDS = 8;            // accelerator dies of the device, each with its own L2
constexpr int INV_TABLE = 512;     // entries of the 1/(k+1) table staged in LDS

}  // namespace bdc
