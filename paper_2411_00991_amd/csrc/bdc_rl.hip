// bdc_rl.hip -- Richardson-Lucy deconvolution on the device, the paper's
// baseline (Introduction; Results, Simulated Data): for Poisson counts d
// blurred by the PSF P with the image formation of Methods, Eqs. 1-2
// (same-size convolution, object zero outside the frame),
//   rho <- rho * (P^T (d / (P rho))) / (P^T 1)      (Richardson 1972; Lucy 1974),
// with d = max(c, 0), c = (w - o) / G the frame's photon image, and rho_0 the
// mean of d.  Also the warm start that restarts the sampler's chains from it.
#include <algorithm>

#include "bdc_device.h"
#include "bdc_kernels.h"

namespace bdc {
namespace {

constexpr int RT = 32;                  // output tile side of the stencil kernels

inline unsigned grid_n(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// One RT x RT output tile of a same-size stencil with the PSF, FP64 sums.
// MODE 0: mu = P (x) rho (convolution, input rho), out q = d / mu (0 where mu <= 0).
// MODE 1: c = P^T (x) q (correlation, input q), rho <- rho * c / norm (in place).
// MODE 2: norm = P^T (x) 1 (correlation of an image of ones inside the frame).
template <int MODE>
__global__ void __launch_bounds__(WG) k_rl_stencil(Frame f, const float* in, float* out, float* rho,
                                                    const float* norm) {
    extern __shared__ float lds_r[];
    const int r = f.r, s = f.s, TW = RT + 2 * r;
    float* tl = lds_r;
    float* sp = lds_r + TW * TW;
    const int ntx = (f.W + RT - 1) / RT;
    const int ty0 = (blockIdx.x / ntx) * RT, tx0 = (blockIdx.x % ntx) * RT;
    for (int i = threadIdx.x; i < TW * TW; i += WG) {
        const int yy = ty0 - r + i / TW, xx = tx0 - r + i % TW;
        const bool inside = yy >= 0 && yy < f.H && xx >= 0 && xx < f.W;
        tl[i] = inside ? (MODE == 2 ? 1.0f : in[(int64_t)yy * f.W + xx]) : 0.0f;
    }
    for (int i = threadIdx.x; i < s * s; i += WG) sp[i] = f.psf[i];
    __syncthreads();
    for (int o = threadIdx.x; o < RT * RT; o += WG) {
        const int ly = o / RT, lx = o % RT;
        const int y = ty0 + ly, x = tx0 + lx;
        if (y >= f.H || x >= f.W) continue;
        double acc = 0.0;
        for (int dy = -r; dy <= r; ++dy) {
            const float* prow = sp + (dy + r) * s + r;
            // convolution reads rho at (y - dy, x - dx); correlation reads q at (y + dy, x + dx)
            const float* trow = MODE == 0 ? tl + (ly - dy + r) * TW + lx + r : tl + (ly + dy + r) * TW + lx + r;
#pragma unroll 4
            for (int dx = -r; dx <= r; ++dx)
                acc = fma((double)prow[dx], (double)(MODE == 0 ? trow[-dx] : trow[dx]), acc);
        }
        const int64_t n = (int64_t)y * f.W + x;
        if (MODE == 0) {
            const double d = fmax((double)f.pc[n].x, 0.0);
            out[n] = acc > 0.0 ? (float)(d / acc) : 0.0f;
        } else if (MODE == 1) {
            rho[n] = (float)((double)rho[n] * acc / (double)norm[n]);
        } else {
            out[n] = (float)acc;
        }
    }
}

// Per-workgroup partial sums of max(c, 0) -> part[wg].
__global__ void k_sum_pos(Frame f, double* part) {
    __shared__ double s_r[WG / 64];
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    double v = n < f.N ? fmax((double)f.pc[n].x, 0.0) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) s_r[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < WG / 64; ++w) t += s_r[w];
        part[blockIdx.x] = t;
    }
}

// rho = mean of d (fixed-order sum of the partials), every pixel.  One value
// per workgroup thread 0 reads; every thread writes its pixels.
__global__ void k_fill_mean(const double* part, int nw, int64_t N, float* rho) {
    __shared__ double s_m;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i) t += part[i];
        s_m = t / (double)N;
    }
    __syncthreads();
    const float m = (float)s_m;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < N; i += (int64_t)gridDim.x * WG) rho[i] = m;
}

// Chains restarted from the RL estimate: rho = max(rl, floor) exp(xi / 2), xi
// from the initial-state stream at sweep 0 (one draw per chain: overdispersed
// starts), every log step = log_step0.
__global__ void k_rl_init(Frame f, State S, const float* rl, float floor_v, float log_step0) {
    const int64_t n = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int chain = blockIdx.y;
    if (n >= f.N) return;
    const float xi = box_muller(draw(f.key, (uint32_t)n, 0u, (uint32_t)chain, STREAM_INIT));
    float v = fmaxf(rl[n], floor_v) * expf(0.5f * xi);
    if (!(v > 0.0f) || !isfinite(v)) v = fmaxf(f.pc[n].x, 0.5f);
    const int64_t i = (int64_t)chain * f.N + n;
    S.rho[i] = v;
    S.log_step[i] = log_step0;
}

size_t rl_lds(int s) {
    const int TW = RT + 2 * (s / 2);
    return (size_t)(TW * TW + s * s) * sizeof(float);
}

}  // namespace

// n_iter RL iterations into rho (N floats); q, norm: N floats each; part:
// grid(N) doubles.
hipError_t launch_richardson_lucy(const Frame& f, int n_iter, float* rho, float* q, float* norm, double* part,
                                  hipStream_t st) {
    const unsigned ntiles = (unsigned)(((f.H + RT - 1) / RT) * ((f.W + RT - 1) / RT));
    const size_t lds = rl_lds(f.s);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    const unsigned nw = grid_n(f.N, WG);
    hipLaunchKernelGGL(k_sum_pos, dim3(nw), dim3(WG), 0, st, f, part);
    hipLaunchKernelGGL(k_fill_mean, dim3(std::min<unsigned>(nw, 4096u)), dim3(WG), 0, st, part, (int)nw, f.N, rho);
    hipLaunchKernelGGL(k_rl_stencil<2>, dim3(ntiles), dim3(WG), lds, st, f, (const float*)nullptr, norm,
                       (float*)nullptr, (const float*)nullptr);
    for (int k = 0; k < n_iter; ++k) {
        hipLaunchKernelGGL(k_rl_stencil<0>, dim3(ntiles), dim3(WG), lds, st, f, (const float*)rho, q,
                           (float*)nullptr, (const float*)nullptr);
        hipLaunchKernelGGL(k_rl_stencil<1>, dim3(ntiles), dim3(WG), lds, st, f, (const float*)q, (float*)nullptr,
                           rho, (const float*)norm);
    }
    return hipGetLastError();
}

hipError_t launch_rl_init(const Frame& f, const State& S, const float* rl, float floor_v, float log_step0,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_rl_init, dim3(grid_n(f.N, WG), f.C), dim3(WG), 0, st, f, S, rl, floor_v, log_step0);
    return hipGetLastError();
}

}  // namespace bdc
