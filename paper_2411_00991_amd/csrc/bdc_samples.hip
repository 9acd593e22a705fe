// bdc_samples.hip -- thinned posterior samples, per-pixel quantiles and the
// coefficient-of-variation map (Results, "Our package": the sampler returns
// many candidate deconvolved images with their mean; "Uncertainty": quantiles,
// variance and CV = std / mean per pixel).
#include "bdc_kernels.h"

namespace bdc {
namespace {

constexpr int QW = 64;                  // one wave per pixel in the quantile kernel

inline unsigned grid_n(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Copies every chain's rho into slot (t - burn_in) / thin of the stack when the
// sweep index t (read on the device: the kernel is replayed from a graph) is a
// post-burn-in multiple of thin and the slot exists.  Layout [slot][C][N].
__global__ void k_export(Frame f, const float* rho, const int64_t* tp, int burn_in, int thin, int cap, float* stack) {
    const int64_t t = *tp;
    if (t < burn_in || (t - burn_in) % thin != 0) return;
    const int64_t slot = (t - burn_in) / thin;
    if (slot >= cap) return;
    const int64_t CN = (int64_t)f.C * f.N;
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < CN) stack[slot * CN + i] = rho[i];
}

// Per-pixel quantiles of n values v[i * stride + pixel], i < n (n <= QMAX):
// one wave per pixel sorts its values in wave-private LDS (bitonic network over
// the next power of two, padded with +inf), then reads each requested quantile
// by linear interpolation between order statistics: h = (n - 1) p,
// q = x[floor h] + (h - floor h) (x[floor h + 1] - x[floor h])  (the default
// definition of numpy.quantile).
__global__ void __launch_bounds__(WG) k_quantiles(const float* v, int64_t n, int64_t stride, int64_t n_pix,
                                                  const float* probs, int n_probs, float* out) {
    extern __shared__ float lds_q[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t pix = (int64_t)blockIdx.x * (WG / QW) + wave;
    int P = 1;
    while (P < n) P <<= 1;
    float* x = lds_q + (size_t)wave * P;
    if (pix < n_pix) {
        for (int i = lane; i < P; i += QW) x[i] = i < n ? v[(int64_t)i * stride + pix] : INFINITY;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (pix >= n_pix) return;
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < P; i += QW) {
                const int l = i ^ j;
                if (l > i) {
                    const float a = x[i], b = x[l];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        x[i] = b;
                        x[l] = a;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    for (int q = lane; q < n_probs; q += QW) {
        const double h = (double)(n - 1) * (double)probs[q];
        const int64_t lo = (int64_t)floor(h);
        const double fr = h - (double)lo;
        double r = (double)x[lo];
        if (fr > 0.0 && lo + 1 < n) r += fr * ((double)x[lo + 1] - (double)x[lo]);
        out[(int64_t)q * n_pix + pix] = (float)r;
    }
}

// CV = sqrt(var) / mean per pixel.
__global__ void k_cv(const float* mean, const float* var, int64_t n, float* cv) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) cv[i] = sqrtf(fmaxf(var[i], 0.0f)) / mean[i];
}

}  // namespace

hipError_t launch_export(const Frame& f, const float* rho, const int64_t* tp, int burn_in, int thin, int cap,
                         float* stack, hipStream_t st) {
    hipLaunchKernelGGL(k_export, dim3(grid_n((int64_t)f.C * f.N, WG)), dim3(WG), 0, st, f, rho, tp, burn_in, thin,
                       cap, stack);
    return hipGetLastError();
}

size_t quantile_lds(int64_t n) {
    int64_t P = 1;
    while (P < n) P <<= 1;
    return (size_t)(WG / QW) * P * sizeof(float);
}

hipError_t launch_quantiles(const float* v, int64_t n, int64_t stride, int64_t n_pix, const float* probs, int n_probs,
                            float* out, hipStream_t st) {
    if (n < 1 || n > QMAX || n_pix < 1) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_quantiles, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)quantile_lds(QMAX));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_quantiles, dim3(grid_n(n_pix, WG / QW)), dim3(WG), quantile_lds(n), st, v, n, stride, n_pix,
                       probs, n_probs, out);
    return hipGetLastError();
}

hipError_t launch_cv(const float* mean, const float* var, int64_t n, float* cv, hipStream_t st) {
    hipLaunchKernelGGL(k_cv, dim3(grid_n(n, WG)), dim3(WG), 0, st, mean, var, n, cv);
    return hipGetLastError();
}

}  // namespace bdc
