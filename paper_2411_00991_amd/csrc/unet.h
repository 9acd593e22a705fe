// unet.h -- host view of the U-Net kernels (BF16 NHWC tensors, launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdc {
namespace unet {

// An NHWC BF16 tensor slice: channel c of pixel q at p[q * ld + off + c],
// pixels numbered (b * H + y) * W + x.
struct Tens {
    uint16_t* p;
    int C, ld, off, H, W;
};

hipError_t conv3_fwd(const Tens& x, const uint16_t* wf, const float* bias, int relu, const Tens& y, int64_t P,
                     hipStream_t st);
hipError_t conv3_dgrad(const Tens& g, const uint16_t* wd, const Tens& gx, const Tens* mask, int64_t P,
                       hipStream_t st);
hipError_t conv3_wgrad(const Tens& x, const Tens& g, float* part, int max_splits, float* dw, int64_t P,
                       hipStream_t st);
hipError_t up_fwd(const Tens& x, const uint16_t* wf, const float* bias, const Tens& y, int64_t P_lo, int Hl, int Wl,
                  hipStream_t st);
hipError_t up_dgrad(const Tens& g, const uint16_t* wd, const Tens& gx, const Tens* mask, int64_t P_lo, int Hl,
                    int Wl, hipStream_t st);
hipError_t up_wgrad(const Tens& x, const Tens& g, float* part, int max_splits, float* dw, int64_t P_lo, int Hl,
                    int Wl, hipStream_t st);
hipError_t bias_grad(const Tens& g, int64_t P, float* part, int max_wg, float* db, hipStream_t st);
hipError_t maxpool(const Tens& in, const Tens& out, int64_t P_out, hipStream_t st);
hipError_t maxpool_bwd(const Tens& in, const Tens& gin, const Tens& gout, int64_t P_out, hipStream_t st);
hipError_t to_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t st);
int head_partial_rows(int64_t P);
hipError_t head(const Tens& f, const float* w, const float* b, int64_t P, float* out, const float* target,
                uint16_t* gf, float* part, float* sums, hipStream_t st);
hipError_t adam(float* p, float* m1, float* m2, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st);
hipError_t weights_conv3(const float* W, int co_n, int ci_n, uint16_t* fwd, uint16_t* dgrad, hipStream_t st);
hipError_t weights_up(const float* W, int co_n, int ci_n, uint16_t* fwd, uint16_t* dgrad, hipStream_t st);
hipError_t gemm_nt(const uint16_t* a, const uint16_t* b, float* c, int64_t M, int N, int K, hipStream_t st);

}  // namespace unet
}  // namespace bdc
